"""The serving scheduler's host logic on a simulated clock (no GPU): FIFO
admission under a byte budget, admission at phase boundaries, deferral when
memory is short or a device allocation fails, a failing job that fails
alone, cancellation of queued and running jobs, rejection of jobs that can
never fit, and the budget never exceeded."""
import pytest

from paper_2208_06970_amd.serve import (CANCELLED, DONE, FAILED, REJECTED, Budget, DeferAdmission, Phase, Request,
                                        Scheduler, simulate)


def _req(i, arrival, resident, ws, names=None):
    names = names or [f"p{k}" for k in range(len(ws))]
    return Request(i, None, arrival, resident, [Phase(n, w) for n, w in zip(names, ws)])


def _events(s, what):
    return [(t, rid) for t, w, rid in s.events if w == what]


def _unit(req, phase):
    return 1.0


def test_fifo_admission_and_budget():
    reqs = [_req(i, 0.01 * i, 20, [30, 10]) for i in range(6)]     # footprint 50 each
    s = simulate(reqs, slots=4, budget_bytes=120, duration=_unit)
    assert all(r.status == DONE for r in reqs)
    assert s.budget.peak <= 120 and s.budget.used == 0
    admitted = [rid for _, rid in _events(s, "admitted")]
    assert admitted == sorted(admitted)                              # arrival order
    # two fit at first (100 <= 120); the third waits until both first jobs
    # have passed a phase boundary (50 -> 30 each): 30 + 30 + 50 <= 120
    assert _events(s, "admitted")[2][0] == pytest.approx(1.01)


def test_admission_at_phase_boundary():
    a = _req(0, 0.0, 10, [100, 10])        # footprint 110, then 20 after its first phase
    b = _req(1, 0.1, 10, [40])             # footprint 50: does not fit next to 110 under 150
    s = simulate([a, b], slots=2, budget_bytes=150, duration=_unit)
    t_b = dict((rid, t) for t, rid in _events(s, "admitted"))[1]
    assert t_b == pytest.approx(1.0)                                  # a's first phase ended
    assert a.done == pytest.approx(2.0) and b.done == pytest.approx(2.0)
    assert t_b < a.done                                              # b joined while a still ran
    assert s.budget.peak <= 150


def test_oom_deferral_and_retry():
    reqs = [_req(i, 0.0, 10, [20, 20]) for i in range(3)]

    def fail(req, phase, attempt):
        # the device refuses request 1's second phase once
        return DeferAdmission("out of memory") if req.id == 1 and phase.name == "p1" and attempt == 1 else None

    s = simulate(reqs, slots=3, budget_bytes=1000, duration=_unit, fail=fail)
    assert all(r.status == DONE for r in reqs)
    assert reqs[1].defers == 1
    assert len(_events(s, "deferred")) == 1
    assert reqs[1].done > reqs[0].done                                # it ran its phases again
    assert s.budget.used == 0


def test_invalid_job_fails_alone():
    reqs = [_req(i, 0.0, 10, [20, 20, 20]) for i in range(4)]

    def fail(req, phase, attempt):
        return ValueError("a seed outside the volume") if req.id == 2 and phase.name == "p1" else None

    s = simulate(reqs, slots=2, budget_bytes=60, duration=_unit, fail=fail)
    assert [r.status for r in reqs] == [DONE, DONE, FAILED, DONE]
    assert isinstance(reqs[2].error, ValueError)
    assert s.budget.used == 0 and s.budget.peak <= 60


def test_cancel_queued_and_running():
    reqs = [_req(i, 0.0, 10, [20, 20, 20]) for i in range(3)]
    # one slot: 0 runs, 1 and 2 wait; cancel 2 while queued and 0 while running
    s = simulate(reqs, slots=1, budget_bytes=100, duration=_unit, cancels=[(0.5, 2), (1.5, 0)])
    assert reqs[2].status == CANCELLED and reqs[2].start != reqs[2].start     # never started
    assert reqs[0].status == CANCELLED and reqs[0].done == pytest.approx(2.0)  # at its next boundary
    assert reqs[1].status == DONE and reqs[1].start == pytest.approx(2.0)
    assert s.budget.used == 0


def test_reject_never_fitting():
    reqs = [_req(0, 0.0, 10, [500]), _req(1, 0.0, 10, [20])]
    s = simulate(reqs, slots=2, budget_bytes=100, duration=_unit)
    assert reqs[0].status == REJECTED and reqs[1].status == DONE
    assert _events(s, "rejected") == [(0.0, 0)]


def test_latency_on_simulated_clock():
    reqs = [_req(i, float(i), 5, [10, 10]) for i in range(3)]       # arrivals 0, 1, 2; each job takes 2
    simulate(reqs, slots=1, budget_bytes=50, duration=_unit)
    assert [r.done - r.arrival for r in reqs] == pytest.approx([2.0, 3.0, 4.0])


def test_budget_accounting_direct():
    b = Budget(100)
    assert b.try_reserve(60) and not b.try_reserve(50) and b.try_reserve(40)
    b.release(100)
    assert b.used == 0 and b.peak == 100
    s = Scheduler(1, Budget(100))
    r = _req(0, 0.0, 10, [30, 50])
    s.submit(r, 0.0)
    assert s.admit(0.0) == [r] and r.reserved == 60
    assert s.phase_done(r, 1.0) and r.reserved == 60            # the remaining phase needs 50 + 10
    assert not s.phase_done(r, 2.0) and r.status == DONE and s.budget.used == 0
