"""Host logic of bench.py's roofline pricing (no GPU): the measured-count files are
used only while their source digest matches, and the fallbacks say so."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_theta_roofline_uses_executed_flops_while_digest_matches(tmp_path, monkeypatch):
    f = tmp_path / "theta_flops.json"
    f.write_text(json.dumps({"16": {"executed_flops_per_xpoint": 2.0e6,
                                    "kernel_digest": bench.kernel_digest(bench.THETA_SOURCES)}}))
    monkeypatch.setattr(bench, "THETA_FLOPS_FILE", str(f))
    r = bench.theta_roofline(16, 1000, 2, 1e-3, "k")
    assert r["achieved"] == 2.0e6 * 1000 * 2 / 1e-3 / 1e12
    assert r["frac"] == r["achieved"] / 78.6 and r["executed_flops_per_xpoint"] == 2.0e6
    conv = bench.theta_flops_per_xpoint(16) * 1000 * 2 / 1e-3 / 1e12
    assert r["conventional"]["achieved"] == conv
    # no entry for this N_k: the conventional count, flagged
    r32 = bench.theta_roofline(32, 1000, 1, 1e-3, "k")
    assert r32["achieved"] == r32["conventional"]["achieved"] and "unavailable" in r32["flop_count"]


def test_theta_roofline_falls_back_when_sources_changed(tmp_path, monkeypatch):
    f = tmp_path / "theta_flops.json"
    f.write_text(json.dumps({"16": {"executed_flops_per_xpoint": 2.0e6, "kernel_digest": "0000000000000000"}}))
    monkeypatch.setattr(bench, "THETA_FLOPS_FILE", str(f))
    assert bench.theta_executed_flops_per_xpoint(16) is None
    r = bench.theta_roofline(16, 1000, 1, 1e-3, "k")
    assert "unavailable" in r["flop_count"] and "executed_flops_per_xpoint" not in r


def test_conventional_count_is_the_fft_convolution():
    # 2 x 5 P^3 log2(P^3) + 2 P^3 with P = 2 N_k
    P3 = 32 ** 3
    assert bench.theta_flops_per_xpoint(16) == 2 * 5 * P3 * 15 + 2 * P3


def test_committed_counts_are_sane():
    # executed counts below the conventional FFT count; counter traffic within 5 % of
    # the algorithmic bytes (bench reports them only while the source digests match)
    t = json.load(open(bench.THETA_FLOPS_FILE))
    for nk in ("16", "32"):
        assert 0 < t[nk]["executed_flops_per_xpoint"] < t[nk]["conventional_flops_per_xpoint"]
    t = json.load(open(bench.TRAFFIC_FILE))
    for wl in ("C2", "C3", "C4"):
        for e in t[wl].values():
            assert 1.0 <= e["hbm_bytes_per_launch"] / e["alg_bytes_per_launch"] < 1.05
