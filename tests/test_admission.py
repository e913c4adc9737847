"""Host-side checks of the serving admission policy (no GPU): first fit in
arrival order within a byte budget and a slot count."""
import ctypes

from paper_2401_13680_amd import _lib


def simulate(budget, slots, reqs):
    L = _lib.load()
    n = len(reqs)
    b = (ctypes.c_size_t * n)(*[r[0] for r in reqs])
    a = (ctypes.c_double * n)(*[r[1] for r in reqs])
    s = (ctypes.c_double * n)(*[r[2] for r in reqs])
    out = (ctypes.c_double * n)()
    rc = L.pst_admission_simulate(budget, slots, n, b, a, s, out)
    return rc, list(out)


def test_budget_defers_until_memory_frees():
    # (bytes, arrival, service)
    rc, start = simulate(100, 8, [(60, 0, 10), (50, 1, 10), (30, 2, 5)])
    assert rc == 0
    # 60 admitted at 0; 50 does not fit until t=10; 30 fits beside 60 at t=2
    assert start == [0, 10, 2]


def test_slots_limit_concurrency():
    rc, start = simulate(1000, 2, [(1, 0, 4), (1, 0, 4), (1, 0, 4), (1, 0, 4)])
    assert rc == 0 and start == [0, 0, 4, 4]


def test_oversized_request_rejected_others_served():
    rc, start = simulate(100, 4, [(120, 0, 1), (40, 0, 1), (70, 0, 1)])
    assert rc == _lib.PST_ENOMEM
    assert start[0] == -1 and start[1] == 0 and start[2] == 1


def test_request_bytes_covers_profile_set():
    L = _lib.load()
    n, m = 100_000, 256
    b = L.pst_request_bytes(n, m, 128, 4)
    assert b >= 4 * (n // m) * (n - m + 1) + 8 * n
    assert L.pst_request_bytes(100, 200, 50, 1) == 0


def simulate_ordered(budget, slots, reqs, priority):
    L = _lib.load()
    n = len(reqs)
    b = (ctypes.c_size_t * n)(*[r[0] for r in reqs])
    a = (ctypes.c_double * n)(*[r[1] for r in reqs])
    s = (ctypes.c_double * n)(*[r[2] for r in reqs])
    p = (ctypes.c_double * n)(*priority) if priority is not None else None
    out = (ctypes.c_double * n)()
    rc = L.pst_admission_simulate_ordered(budget, slots, n, b, a, s, p, out)
    return rc, list(out)


def test_ordered_without_priority_is_arrival_order():
    reqs = [(60, 0, 10), (50, 1, 10), (30, 2, 5), (20, 2, 1), (90, 3, 4)]
    assert simulate_ordered(100, 3, reqs, None) == simulate(100, 3, reqs)
    # priorities equal to the arrival index give arrival order as well
    assert simulate_ordered(100, 3, reqs, [0, 1, 2, 3, 4]) == simulate(100, 3, reqs)


def test_shortest_predicted_first_lowers_mean_wait():
    # one slot, everything queued at t=0: shortest first is the classic
    # mean-wait optimum (smallest total of start times)
    svc = [9.0, 1.0, 5.0, 2.0, 7.0]
    reqs = [(1, 0, s) for s in svc]
    _, fifo = simulate(100, 1, reqs)
    rc, spf = simulate_ordered(100, 1, reqs, svc)
    assert rc == 0
    assert fifo == [0, 9, 10, 15, 17]
    assert spf == [15, 0, 3, 1, 8]
    assert sum(spf) < sum(fifo)
    # equal predictions keep arrival order
    _, tie = simulate_ordered(100, 1, reqs, [1.0] * 5)
    assert tie == fifo


def test_ordered_still_first_fit_within_budget():
    # the shortest request does not fit yet: the next one that fits goes first
    reqs = [(70, 0, 10), (50, 1, 1), (20, 1, 3)]
    rc, start = simulate_ordered(100, 4, reqs, [10, 1, 3])
    assert rc == 0 and start == [0, 10, 1]
