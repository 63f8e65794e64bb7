"""Admission policy of the solve server on a virtual clock (no GPU).

helm_sched_simulate runs the server's own admission code (pick_next in server.cpp) against
synthetic arrivals, service times and footprints.  Checked invariants: the device-workspace
budget and the slot count are never exceeded; with no bypass window admission follows
arrival order; requests arriving while others run are admitted before those finish
(continuous batching, not batch-at-a-time); a large request is not starved by a stream of
small ones once its bypass window has passed; a request that can never fit is rejected.
"""
import numpy as np
import pytest

from paper_1107_2461_amd import HelmError, sched_simulate


def _load(admit, done, foot, t):
    run = (admit <= t) & (done > t)
    return run.sum(), int(np.asarray(foot)[run].sum())


def _check_capacity(admit, done, foot, slots, budget):
    for t in np.unique(np.concatenate([admit, done])):
        n, b = _load(admit, done, foot, t)
        assert n <= slots and b <= budget, (t, n, b)


def test_budget_and_slots_never_exceeded():
    rng = np.random.default_rng(0)
    n = 400
    arrival = np.cumsum(rng.exponential(0.01, n))
    service = rng.uniform(0.005, 0.05, n)
    foot = rng.integers(1, 9, n) * 1000
    for slots, budget in ((1, 8000), (4, 10000), (8, 20000)):
        admit, done = sched_simulate(arrival, service, foot, slots, budget, 20.0)
        assert np.all(admit >= arrival - 1e-15)
        np.testing.assert_allclose(done, admit + service)
        _check_capacity(admit, done, foot, slots, budget)


def test_fifo_without_bypass():
    rng = np.random.default_rng(1)
    n = 200
    arrival = np.cumsum(rng.exponential(0.01, n))
    service = rng.uniform(0.01, 0.03, n)
    foot = rng.integers(1, 9, n) * 1000
    admit, _ = sched_simulate(arrival, service, foot, 3, 12000, 0.0)
    assert np.all(np.diff(admit) >= -1e-15)          # admitted in arrival order


def test_mid_flight_admission():
    # two long requests start; a third arrives while they run and is admitted immediately
    arrival = [0.0, 0.0, 0.1]
    service = [1.0, 1.0, 0.2]
    foot = [1, 1, 1]
    admit, done = sched_simulate(arrival, service, foot, 3, 10, 0.0)
    assert admit[2] == pytest.approx(0.1)
    assert done[2] < done[0]


def test_bypass_window_then_no_starvation():
    # a big request (needs the whole budget) queued behind a running one, followed by a
    # stream of small ones that fit beside the running request
    arrival = [0.0, 0.01] + list(0.02 + 0.01 * np.arange(50))
    service = [0.1, 0.05] + [0.03] * 50
    foot = [6, 10] + [3] * 50
    admit, done = sched_simulate(arrival, service, foot, 4, 10, 30.0)
    big = 1
    # small requests may pass the big one only within its 30 ms window
    passed = [i for i in range(2, 52) if admit[i] < admit[big]]
    assert all(admit[i] <= arrival[big] + 0.030 + 1e-12 for i in passed)
    # the big one starts as soon as everything admitted before it has drained
    before = [i for i in range(52) if admit[i] < admit[big]]
    assert admit[big] == pytest.approx(max(done[i] for i in before))
    _check_capacity(admit, done, foot, 4, 10)


def test_request_larger_than_budget_is_rejected():
    with pytest.raises(HelmError, match="EINVAL"):
        sched_simulate([0.0], [1.0], [11], 2, 10, 0.0)


def test_one_big_solve_at_a_time():
    # big solves (each fills the GPU) run one after another; small ones arriving meanwhile are
    # admitted beside the running big one and pass the queued big one within its window
    arrival = [0.0, 0.0] + list(0.05 + 0.05 * np.arange(10))
    service = [1.0, 1.0] + [0.02] * 10
    foot = [1] * 12
    big = [1, 1] + [0] * 10
    admit, done = sched_simulate(arrival, service, foot, 4, 100, 2000.0, big=big)
    assert admit[0] == 0.0 and admit[1] == pytest.approx(done[0])
    np.testing.assert_allclose(admit[2:], arrival[2:])
    _check_capacity(admit, done, foot, 4, 100)
    for t in np.unique(np.concatenate([admit, done])):
        run = (admit <= t) & (done > t)
        assert (run & (np.asarray(big) == 1)).sum() <= 1, t
    # without the size classes the second big one starts at once
    admit0, _ = sched_simulate(arrival, service, foot, 4, 100, 2000.0)
    assert admit0[1] == 0.0


def test_blocked_big_head_holds_queue_after_window():
    # with no bypass window a big head that waits for the running big solve is not passed
    arrival = [0.0, 0.01, 0.02]
    service = [1.0, 1.0, 0.1]
    big = [1, 1, 0]
    admit, done = sched_simulate(arrival, service, [1, 1, 1], 4, 100, 0.0, big=big)
    assert admit[1] == pytest.approx(done[0])
    assert admit[2] == pytest.approx(admit[1])
