"""Scheduling invariants of the continuous-batching server on the host-only backend."""
import dataclasses

import numpy as np

from paper_2205_02380_amd import inputs, serve


def small_trace(n=40, rate=200.0, seed=7):
    shapes = inputs.SERVING_SHAPES[:3]
    return inputs.serving_trace(n=n, rate=rate, seed=seed, shapes=shapes, steps_range=(5, 30))


def test_every_request_completes_and_work_adds_up():
    tr = small_trace()
    be = serve.FakeBackend()
    rep = serve.Server(be, budget_bytes=4e9, max_active=8).run(tr)
    assert rep.completed == len(tr) and rep.failed == 0 and rep.rejected == 0
    assert rep.point_updates == sum(r.grid.points * r.steps for r in tr)
    assert all(v["steps"] == r.steps for r, v in zip(sorted(tr, key=lambda r: r.rid), [rep.results[r.rid] for r in sorted(tr, key=lambda r: r.rid)]))
    assert rep.p99_step_ms >= rep.p50_step_ms > 0


def test_budget_and_slots_are_never_exceeded():
    tr = small_trace(n=60, rate=1000.0)
    budget = 1.5e9
    be = serve.FakeBackend()
    rep = serve.Server(be, budget_bytes=budget, max_active=5).run(tr)
    assert rep.max_resident_bytes <= budget
    assert rep.max_active <= 5
    assert rep.completed == len(tr)


def test_admission_is_fifo():
    tr = small_trace(n=30, rate=5000.0)
    be = serve.FakeBackend()
    rep = serve.Server(be, budget_bytes=1e9, max_active=3).run(tr)
    order = sorted(tr, key=lambda r: (r.arrival, r.rid))
    admitted = [rep.results[r.rid]["admitted"] for r in order]
    assert admitted == sorted(admitted)


def test_oversized_request_is_rejected_others_served():
    tr = small_trace(n=10)
    big = dataclasses.replace(tr[3], grid=inputs.SERVING_SHAPES[3], rid=999)
    be = serve.FakeBackend()
    rep = serve.Server(be, budget_bytes=0.6e9, max_active=4).run(list(tr) + [big])
    assert rep.results[999]["status"] == "rejected"
    assert rep.rejected == 1 and rep.completed == len(tr)


def test_cancellation_frees_the_slot_early():
    tr = small_trace(n=12)
    victim = tr[2].rid
    be = serve.FakeBackend()
    rep = serve.Server(be, budget_bytes=4e9, max_active=4).run(tr, cancel_at={victim: 2})
    assert rep.results[victim]["status"] == "cancelled" and rep.results[victim]["steps"] == 2
    assert rep.completed == len(tr) - 1


def test_failed_job_is_isolated():
    tr = small_trace(n=12)
    bad = tr[5].rid
    be = serve.FakeBackend(nan_rids=[bad])
    rep = serve.Server(be, budget_bytes=4e9, max_active=4).run(tr)
    assert rep.results[bad]["status"] == "failed"
    assert rep.failed == 1 and rep.completed == len(tr) - 1


def test_replay_is_deterministic():
    tr = small_trace(n=25)
    a = serve.Server(serve.FakeBackend(), budget_bytes=2e9, max_active=6).run(tr).as_dict()
    b = serve.Server(serve.FakeBackend(), budget_bytes=2e9, max_active=6).run(tr).as_dict()
    assert a == b


def test_trace_statistics():
    tr = inputs.serving_trace()
    assert len(tr) == 200
    gaps = np.diff([r.arrival for r in tr])
    assert 0.035 < gaps.mean() < 0.065                   # mean inter-arrival 50 ms
    assert {r.dt for r in tr} <= {0.01, 0.02, 0.05}
    assert all(10 <= r.steps <= 200 for r in tr)
    assert {r.grid.nx[0] for r in tr} == {16, 24, 32, 48}
