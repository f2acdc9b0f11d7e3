"""The request server's admission and pool rule (kc_server_plan_admission),
checked on the CPU with fake request and context sizes: no device is needed,
the rule is the one the server's workers call.

Each branch of the rule (best-fit reuse, a new context beside the pool, the
least-growing pooled context, a new context after evictions, waiting), the
least-recently-used eviction order, the cap on bases in flight, and a
simulated stream of requests in which reservations plus pooled bytes never
exceed the budget and every request is eventually admitted.
"""
import random

import pytest

import paper_1712_03254_amd as kc

plan = kc.plan_admission


def test_best_fit_reuses_the_smallest_context_that_needs_no_memory():
    pool = [(50, 40, 1), (20, 20, 2), (30, 25, 3), (10, 12, 4)]
    assert plan(1000, 0, pool, 1, 100) == (1, 20, [])


def test_new_context_when_it_fits_beside_the_pool():
    # every pooled context would have to grow; a new one fits with the pool kept
    pool = [(10, 30, 1), (10, 40, 2)]
    assert plan(100, 50, pool, 1, 25) == (-1, 25, [])


def test_least_growing_context_when_a_new_one_does_not_fit_beside_the_pool():
    # new (35) + in use (40) + pooled (30) > 100; growing pool[1] by 5 costs less than 35
    pool = [(10, 30, 1), (20, 25, 2)]
    assert plan(100, 40, pool, 1, 35) == (1, 25, [])


def test_new_context_after_evicting_the_least_recently_used():
    # growing would take more than a new context: a new one, room made by eviction
    pool = [(20, 0, 5), (15, 0, 2), (25, 0, 9)]
    got = plan(100, 30, pool, 1, 50)
    assert got is not None
    choice, reserve, evict = got
    assert choice == -1 and reserve == 50
    # oldest first (stamps 2, 5, 9) until 30 + 50 + pooled <= 100: 140, 125, 105, 80
    assert evict == [1, 0, 2]
    assert 30 + 50 + sum(p[0] for i, p in enumerate(pool) if i not in evict) <= 100


def test_chosen_context_is_never_evicted():
    # pool[0] is the least recently used, but the request takes it (growing by
    # 5 < a new 60); room comes from pool[1]: 20 + 45 + 40 > 100
    pool = [(40, 45, 1), (40, 0, 2)]
    got = plan(100, 20, pool, 1, 60)
    choice, reserve, evict = got
    assert choice == 0 and reserve == 45
    assert 0 not in evict and evict == [1]


def test_waits_when_nothing_fits():
    assert plan(100, 90, [(5, 0, 1)], 1, 20) is None
    assert plan(100, 90, [(5, 60, 1)], 1, 20) is None


def test_cap_on_bases_in_flight():
    # a request larger than the cap runs only when nothing else does
    assert plan(1000, 100, [], job_bases=300, estimate=10, max_inflight=256, inflight=10,
                running=1) is None
    assert plan(1000, 0, [], job_bases=300, estimate=10, max_inflight=256, inflight=0,
                running=0) == (-1, 10, [])
    # small requests share the device up to the cap
    assert plan(1000, 100, [], job_bases=100, estimate=10, max_inflight=256, inflight=150,
                running=2) == (-1, 10, [])
    assert plan(1000, 100, [], job_bases=110, estimate=10, max_inflight=256, inflight=150,
                running=2) is None


def test_inconsistent_pool_sum_is_rejected():
    state = kc.KcAdmitState(100, 0, 7, 0, 0, 0, 0)  # pooled says 7, the pool holds 5
    arr = (kc.KcAdmitPooled * 1)(kc.KcAdmitPooled(5, 5, 1))
    out = [kc.ctypes.c_uint32(), kc.ctypes.c_int32(), kc.ctypes.c_uint64(),
           (kc.ctypes.c_uint32 * 1)(), kc.ctypes.c_uint32()]
    st = kc.load().kc_server_plan_admission(kc.ctypes.byref(state), arr, 1, 1, 5,
                                            kc.ctypes.byref(out[0]), kc.ctypes.byref(out[1]),
                                            kc.ctypes.byref(out[2]), out[3],
                                            kc.ctypes.byref(out[4]))
    assert st == kc.KC_ERR_INVALID_ARG


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_simulated_stream_stays_within_budget(seed):
    """Requests of log-uniform size arrive in a queue; up to four run at once;
    a finished request is released after a random delay and its context
    pooled.  A context's bytes after a job are the larger of what it holds and
    what the job needs (buffers only grow).  Admission follows the rule for
    the head of the queue; evictions are applied before the job starts."""
    rng = random.Random(seed)
    budget = 1 << 30
    sizes = [int(2 ** rng.uniform(16, 28)) for _ in range(400)]  # bytes a job needs
    queue = list(range(len(sizes)))
    running, done_waiting, pool = [], [], []  # running: (job, bytes reserved)
    in_use, stamp, admitted, created, reused = 0, 0, 0, 0, 0
    steps = 0
    while queue or running or done_waiting:
        steps += 1
        assert steps < 100_000
        progressed = False
        if queue and len(running) < 4:
            need = sizes[queue[0]]
            view = [(b, max(b, need), s) for b, s in pool]
            got = plan(budget, in_use, view, need, need)
            if got is not None:
                choice, reserve, evict = got
                assert choice == -1 or choice not in evict
                keep = [p for i, p in enumerate(pool) if i not in evict and i != choice]
                if choice >= 0:
                    reused += 1
                else:
                    created += 1
                pool = keep
                in_use += reserve
                assert in_use + sum(b for b, _ in pool) <= budget
                running.append((queue.pop(0), reserve))
                admitted += 1
                progressed = True
        if running and (rng.random() < 0.5 or not progressed):
            job, reserve = running.pop(rng.randrange(len(running)))
            done_waiting.append(reserve)
            progressed = True
        if done_waiting and (rng.random() < 0.5 or not progressed):
            reserve = done_waiting.pop(0)
            in_use -= reserve
            stamp += 1
            pool.append((reserve, stamp))
        assert in_use + sum(b for b, _ in pool) <= budget
    assert admitted == len(sizes)
    assert reused > 0 and created > 0
