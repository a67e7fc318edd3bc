"""CPU tests of the HIP path's host side: the C-ABI library loads and exports every
entry point the header declares, descriptor validation fails cleanly without a GPU,
and the product's FP64 tables + line routine (compiled for the host) agree with the
oracle line by line."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2205_02380_amd import chasm, inputs
from tests import linetwin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chasm_advect.h")


def header_symbols():
    syms = set()
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            syms |= set(re.findall(r"\b(chasm_[a-z0-9]+_[a-z_]+)\s*\(", text))
    return sorted(syms)


def test_library_exports_every_declared_symbol():
    from paper_2205_02380_amd import ho2d, lpc1, theta
    syms = header_symbols()
    assert len(syms) >= 16
    L = chasm.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(chasm.EXPORTS) | set(theta.EXPORTS) | set(lpc1.EXPORTS) | set(ho2d.EXPORTS)
    assert "gfx950" in chasm.chasm_advect_version()


def test_desc_layout_matches_header():
    # 3*4*2 ints, 12 doubles, 3 ints + ghost, dt, 4 int32/uint32, schedule, history_cap,
    # 6 end-slope doubles
    d = chasm.chasm_advect_desc()
    assert ctypes.sizeof(d) == 24 + 96 + 16 + 8 + 24 + 48
    assert chasm.chasm_advect_desc.slope_lo.offset % 8 == 0
    assert chasm.chasm_advect_desc.dt.offset % 8 == 0


@pytest.mark.parametrize("mutate,status", [
    (lambda d: setattr(d, "ghost", 0), chasm.CHASM_EINVAL),
    (lambda d: d.nx.__setitem__(0, 1), chasm.CHASM_EINVAL),
    (lambda d: d.nk.__setitem__(2, 0), chasm.CHASM_EINVAL),
    (lambda d: d.x_hi.__setitem__(1, d.x_lo[1]), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "dtype", 7), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "closure", 9), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "nbatch", 0), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "flags", 1 << 9), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "dt", float("nan")), chasm.CHASM_EINVAL),
    (lambda d: (setattr(d, "closure", 1), setattr(d, "ghost", 2)), chasm.CHASM_EINVAL),
    (lambda d: setattr(d, "closure", 4), chasm.CHASM_EINVAL),
    (lambda d: (setattr(d, "closure", 3), d.slope_lo.__setitem__(1, float("inf"))), chasm.CHASM_EINVAL),
    # resource limits of the runtime-shape kernels, and schedules they do not provide
    (lambda d: d.nx.__setitem__(0, 5000), chasm.CHASM_EUNSUPPORTED),
    (lambda d: (d.patch.__setitem__(0, 7), setattr(d, "schedule", 2)), chasm.CHASM_EUNSUPPORTED),
    (lambda d: (d.nx.__setitem__(1, 40), setattr(d, "schedule", 1)), chasm.CHASM_EUNSUPPORTED),
])
def test_descriptor_validation(mutate, status):
    w = inputs.workload("C2")
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt)
    mutate(d)
    with pytest.raises(chasm.ChasmError) as ei:
        chasm.chasm_advect_workspace_bytes(d)
    assert ei.value.status == status
    assert chasm.chasm_advect_last_error()


@pytest.mark.parametrize("mutate", [
    lambda d: d.patch.__setitem__(0, 7),                    # unequal patch lengths
    lambda d: d.nx.__setitem__(0, 20),                      # unequal axes
    lambda d: setattr(d, "ghost", 9),                       # no compiled (patch, ghost)
    lambda d: setattr(d, "closure", 1),                     # no compiled POLY3 shape
    lambda d: (d.nx.__setitem__(0, 61), d.nx.__setitem__(1, 61), d.nx.__setitem__(2, 61),
               d.patch.__setitem__(0, 15), d.patch.__setitem__(1, 15), d.patch.__setitem__(2, 15),
               setattr(d, "ghost", 15)),                    # the paper's 61-node, 4-patch line
    lambda d: (d.nx.__setitem__(0, 40), d.nx.__setitem__(1, 48), d.nx.__setitem__(2, 36)),
    lambda d: (setattr(d, "closure", 3), d.slope_lo.__setitem__(0, 0.25)),
    lambda d: setattr(d, "flags", chasm.CHASM_FLAG_RUNTIME_SHAPE),
])
def test_any_valid_shape_is_accepted_by_the_runtime_kernels(mutate):
    """Descriptors without compiled kernels run on the runtime-shape kernels (PLAIN)."""
    w = inputs.workload("C2")
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt)
    mutate(d)
    assert chasm.chasm_advect_workspace_bytes(d) > 0
    d.schedule = chasm.CHASM_SCHED_PLAIN
    assert chasm.chasm_advect_workspace_bytes(d) > 0


def test_cube_schedule_rejected_when_cube_exceeds_lds():
    w = inputs.workload("C4")
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt, schedule="cube")
    with pytest.raises(chasm.ChasmError) as ei:
        chasm.chasm_advect_workspace_bytes(d)
    assert ei.value.status == chasm.CHASM_EUNSUPPORTED
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt)
    assert 0 < chasm.chasm_advect_workspace_bytes(d) < 64 << 20


def test_observe_workspace_adds_the_item_rows():
    grid = inputs.cubic_grid(32, 12.0, 4, 4.0)
    d0 = chasm.make_desc(grid, 8, 6, 0.02)
    d1 = chasm.make_desc(grid, 8, 6, 0.02, flags=chasm.CHASM_FLAG_OBSERVE)
    nitems = 4 ** 3
    rows = nitems * (32 * 32 + 16 * 32) * 8
    sums = (3 * 32 * 4 + 32 * 32) * 8
    extra = chasm.chasm_advect_workspace_bytes(d1) - chasm.chasm_advect_workspace_bytes(d0)
    assert rows + sums <= extra <= rows + sums + 1024
    d2 = chasm.make_desc(grid, 8, 6, 0.02, flags=1 << 7)
    with pytest.raises(chasm.ChasmError) as ei:
        chasm.chasm_advect_workspace_bytes(d2)
    assert ei.value.status == chasm.CHASM_EINVAL


def test_out_of_place_workspace_adds_one_field():
    for name, dtype, size in (("C2", "f32", 4), ("C1", "f64", 8)):
        w = inputs.workload(name)
        d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt, dtype)
        base = chasm.chasm_advect_workspace_bytes(d)
        d.flags = chasm.CHASM_FLAG_OUT_OF_PLACE
        assert chasm.chasm_advect_workspace_bytes(d) - base == w.grid.points * size + 256


def test_null_arguments_fail_without_device():
    L = chasm.lib()
    assert L.chasm_advect_create(None, None, None, None) == chasm.CHASM_EINVAL
    assert L.chasm_advect_step(None, 1) == chasm.CHASM_EINVAL
    assert L.chasm_advect_destroy(None) == chasm.CHASM_OK
    h = ctypes.c_void_p()
    w = inputs.workload("C1")
    d = chasm.make_desc(w.grid, w.patch, w.ghost, w.dt, dtype="f64")
    assert L.chasm_advect_create(ctypes.byref(d), None, None, ctypes.byref(h)) == chasm.CHASM_EINVAL
    assert h.value is None


# --------------------------------------------------------------------------- line algebra
ALPHAS = [0.0, 0.3, -0.3, 0.999, -0.999, 1.0, -1.0, 1.5, -2.5, 3.7, -4.2, 6.0, 0.02, -0.107, -9.5, 11.2, 70.0]


@pytest.mark.parametrize("N,M,G,CL", linetwin.SHAPES)
def test_product_line_algebra_matches_oracle_fp64(N, M, G, CL):
    """The product's compile-time PMBC rows and patch factors, its eq. 3.8 weight
    tables and its register line routine (reduced patch system, cell values, shifted
    store), compiled for the host in FP64, reproduce the oracle's dense per-patch
    solves for every shift class."""
    rng = np.random.default_rng(N * 100 + M + 7 * CL)
    h = 0.7
    # cubic-exact rows at g = 3 are an exactly determined 4-node Vandermonde solve:
    # both sides hold them to ~1e-12
    tol = 1e-13 if CL != 1 else 2e-11
    for a in ALPHAS:
        phi = rng.standard_normal(N)
        ref = oracle.line(N, M, G, h, a, phi, closure=CL)
        got = linetwin.line(True, N, M, G, CL, h, a, phi)
        assert np.max(np.abs(got - ref)) < tol, a


@pytest.mark.parametrize("N,M,G,CL", linetwin.SHAPES)
def test_compile_time_rows_match_host_tables_and_oracle(N, M, G, CL):
    """The kernels' compile-time interface rows equal the host FP64 table builder's
    rows and the oracle's rows (all times h)."""
    h = 0.35
    ct = linetwin.rows(N, M, G, CL)
    host = linetwin.rows(N, M, G, CL, h=h)
    orc = oracle.stencils(N, M, G, h, CL) * h
    tol = 1e-14 if CL != 1 else 1e-11
    assert np.max(np.abs(ct - host)) < tol
    P = ct.shape[0] - 1
    for q in range(P + 1):
        I = q * M if q < P else N - 1
        for t in range(2 * G + 1):
            j = I - G + t
            expect = orc[q, j] if 0 <= j < N else 0.0
            assert abs(ct[q, t] - expect) < tol


@pytest.mark.parametrize("N,M,G", [(16, 8, 4), (32, 8, 6), (48, 16, 8), (64, 16, 8)])
def test_product_line_algebra_fp32_on_smooth_data(N, M, G):
    """FP32 arithmetic on smooth data stays within 2e-7 of max|f| per sweep."""
    h = 0.7
    x = np.arange(N) * h
    phi = np.exp(-((x - x.mean()) / 3.0) ** 2).astype(np.float32).astype(np.float64)
    for CL in (0, 1):
        for a in (0.3, -0.3, 0.999, -0.999, 1.5, -2.5):
            ref = oracle.line(N, M, G, h, a, phi, closure=CL)
            got = linetwin.line(False, N, M, G, CL, h, a, phi)
            assert np.max(np.abs(got - ref)) < 2e-7 * np.max(np.abs(phi))


def test_product_line_algebra_exact_global_at_full_window():
    """With the stencil window covering the whole line (g = N-1), the product's
    patched line equals the oracle's global natural spline."""
    N, M, G = 16, 8, 15
    rng = np.random.default_rng(5)
    for a in (0.4, -0.6, 1.3):
        phi = rng.standard_normal(N)
        got = linetwin.line(True, N, M, G, 0, 0.5, a, phi)
        assert np.max(np.abs(got - oracle.global_line(N, 0.5, a, phi))) < 1e-13


def test_generator_cubes_match_full_field():
    grid = inputs.Grid((8, 8, 8), (-4.0,) * 3, (4.0,) * 3, (3, 4, 5), (-1.0, -2.0, -1.5), (1.0, 2.0, 1.5))
    pk = inputs.random_packets(3, 7)
    full = inputs.gaussian_field(grid, pk).numpy()
    kidx = inputs.k_sample(grid, 0.3, 1)
    cubes = inputs.gaussian_cubes(grid, pk, kidx)
    for n, (i1, i2, i3) in enumerate(kidx):
        assert np.allclose(cubes[n], full[i3, i2, i1], rtol=1e-14, atol=1e-300)


def test_compiled_shapes_cover_every_tuned_configuration():
    """The kernels the workloads and the autotuner need are compiled (the registry is
    enumerated through descriptor validation alone)."""
    s = set(chasm.compiled_shapes())
    need = {("f64", 16, 8, 4, "pmbc"), ("f64", 16, 8, 4, "poly3"), ("f32", 32, 8, 6, "pmbc"),
            ("f64", 32, 8, 6, "pmbc")}
    need |= {("f32", 48, m, g, "pmbc") for m in (8, 12, 16) for g in (4, 6, 8)}
    need |= {("f32", 64, m, g, "pmbc") for m in (8, 16) for g in (4, 6, 8)}
    need |= {("f32", n, 8, 6, "pmbc") for n in (16, 24, 32, 48)}     # serving shapes
    assert need <= s, need - s
    for dt, n, m, g, cl in s:
        assert n % m == 0 and 1 <= g < n


def test_autotune_candidates_weigh_placement_and_tile_shape():
    """Every (patch, ghost, schedule, tile) the C3 grid supports appears in place and out
    of place (48^3 cubes exceed LDS, so no cube schedule); the three tile shapes exist
    for every 48^3 (patch, ghost)."""
    from paper_2205_02380_amd import autotune
    w = inputs.workload("C3")
    cands = autotune.candidates(w.grid, w.dt, (8, 12, 16), (4, 6, 8), ("cube", "slab", "plain"))
    keys = {(c["patch"], c["ghost"], c["schedule"], c["tile"]) for c in cands}
    assert {c["schedule"] for c in cands} == {"slab", "plain"}
    assert {c["tile"] for c in cands} == {0, 1, 2}
    assert len(cands) == 2 * len(keys) == 2 * 9 * 2 * 3


def _tile_status(grid, M, g, schedule, tile, dtype="f32", runtime=False):
    flags = chasm.CHASM_FLAG_TILE(tile) | (chasm.CHASM_FLAG_RUNTIME_SHAPE if runtime else 0)
    try:
        chasm.chasm_advect_workspace_bytes(chasm.make_desc(grid, M, g, 0.02, dtype, flags=flags, schedule=schedule))
        return chasm.CHASM_OK
    except chasm.ChasmError as e:
        return e.status


def test_tile_variant_validation():
    g48 = inputs.cubic_grid(48, 16.0, 4, 4.0)
    g64 = inputs.cubic_grid(64, 16.0, 2, 4.0)
    g32 = inputs.cubic_grid(32, 12.0, 4, 4.0)
    for t in (0, 1, 2):
        for sc in ("slab", "plain"):
            assert _tile_status(g48, 12, 6, sc, t) == chasm.CHASM_OK
            assert _tile_status(g64, 16, 8, sc, t) == chasm.CHASM_OK
    assert _tile_status(g48, 12, 6, "auto", 1) == chasm.CHASM_EUNSUPPORTED       # schedule must be named
    assert _tile_status(g64, 16, 4, "slab", 1) == chasm.CHASM_EUNSUPPORTED       # not compiled in variants
    assert _tile_status(g32, 8, 6, "slab", 2) == chasm.CHASM_EUNSUPPORTED
    assert _tile_status(g48, 16, 8, "slab", 1, dtype="f64") == chasm.CHASM_EUNSUPPORTED
    assert _tile_status(g48, 12, 6, "plain", 1, runtime=True) == chasm.CHASM_EUNSUPPORTED
    assert _tile_status(g48, 12, 6, "slab", 3) == chasm.CHASM_EINVAL


def test_autotune_choice_breaks_timing_ties_by_accuracy():
    from paper_2205_02380_amd import autotune

    def c(M, g, sc, oop, ms, dev, ok=True):
        return {"patch": M, "ghost": g, "schedule": sc, "tile": 0, "out_of_place": oop, "ms_per_step": ms,
                "deviation": dev, "ok": ok}
    cands = [c(16, 8, "slab", False, 4.60, 0.0), c(16, 8, "slab", True, 4.58, 0.0),
             c(12, 8, "slab", False, 4.57, 2.5e-6), c(16, 4, "slab", False, 4.10, 4e-4, ok=False)]
    best = autotune.choose(cands, margin=0.01)
    # within 1 % of the fastest ok time (4.57): the most accurate, in place before out of place
    assert (best["patch"], best["ghost"], best["out_of_place"]) == (16, 8, False)
    best = autotune.choose(cands, margin=0.0)
    assert (best["patch"], best["ghost"]) == (12, 8)
    cands[1]["ms_per_step"] = 4.40            # out of place clearly faster: it wins
    assert autotune.choose(cands, margin=0.01)["out_of_place"] is True
    with pytest.raises(ValueError):
        autotune.choose([c(8, 4, "slab", False, 1.0, 1.0, ok=False)])


def test_autotune_cache_keys_keep_reduction_runs_apart(tmp_path):
    # a result tuned with the per-step diagnostics is cached apart from one tuned without
    from paper_2205_02380_amd import autotune
    w = inputs.workload("C3")
    path = str(tmp_path / "tune.json")
    plain = {"reduce_each_step": False, "best": {"tile": 1}}
    red = {"reduce_each_step": True, "best": {"tile": 0}}
    autotune.store(path, w.grid, w.dt, plain)
    autotune.store(path, w.grid, w.dt, red)
    assert autotune.lookup(path, w.grid, w.dt)["best"]["tile"] == 1
    assert autotune.lookup(path, w.grid, w.dt, reduce_each_step=True)["best"]["tile"] == 0
    assert autotune.cache_key(w.grid, w.dt) != autotune.cache_key(w.grid, w.dt, True)
