"""Served jobs on the GPU: continuous batching with shared launches gives every job the
same result as running it alone (bitwise), and a job whose field holds a NaN is caught
at retirement without touching the others."""
import numpy as np
import pytest
import torch

from paper_2205_02380_amd import chasm, inputs, serve

pytestmark = pytest.mark.gpu


def test_served_results_equal_solo_runs_and_faults_are_isolated():
    shapes = inputs.SERVING_SHAPES[:3]
    trace = inputs.serving_trace(n=14, rate=400.0, seed=11, shapes=shapes, steps_range=(3, 12))
    bad = trace[4].rid
    be = serve.ChasmBackend(keep=[r.rid for r in trace], nan_rids=[bad])
    rep = serve.Server(be, budget_bytes=3e9, max_active=6).run(trace)
    print(rep.as_dict(), flush=True)
    assert rep.failed == 1 and rep.results[bad]["status"] == "failed"
    assert rep.completed == len(trace) - 1
    assert rep.max_resident_bytes <= 3e9 and rep.max_active <= 6
    for r in trace:
        if r.rid == bad:
            continue
        f = inputs.gaussian_field(r.grid, r.packets, dtype=torch.float32, device="cuda:0")
        with chasm.Advect(f, r.grid, 8, 6, r.dt) as a:
            a.step(r.steps)
        torch.cuda.synchronize()
        assert torch.equal(f, be.kept[r.rid]), r.rid
        assert np.isfinite(rep.results[r.rid]["mass"])
