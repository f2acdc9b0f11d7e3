"""Served form (kc_server_*): jobs of uneven size and configuration admitted
under an HBM budget and run concurrently; every job's result (table, Bloom
levels, statistics) is bit-identical to the same job run alone, and a subset
is checked against the CPU oracle.  Admission never lets the reserved bytes
exceed the budget.

Every case prints its name, seed and shape before touching the GPU.
"""
import threading
import time

import numpy as np
import pytest

import oracle
import paper_1712_03254_amd as kc
from kc_cases import (STAT_MAP, assert_same_table, note, oracle_params, pack_reads, random_reads,
                      to_device)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kc.load()
    yield


def make_jobs(seed, n_jobs):
    """Joint (normal, tumour) jobs of log-uniform size with their own Bloom
    size and partition count."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n_jobs):
        n = int(np.exp(rng.uniform(np.log(20), np.log(3000))))
        normal = random_reads(seed * 1000 + 2 * i, n, 60, 120, genome_len=4000)
        tumour = random_reads(seed * 1000 + 2 * i + 1, n, 60, 120, genome_len=4000)
        m = int(min(24, max(16, np.ceil(np.log2(8 * n * 90)))))
        cfg = kc.Config(k=int(rng.choice([21, 25, 31])), n_counters=2, bloom_bits_log2=m,
                        bloom_hashes=4, bloom_block_log2=min(14, m - 2),
                        partitions_log2=int(rng.integers(0, 10)), seed=seed * 7 + i)
        jobs.append((cfg, [pack_reads(normal), pack_reads(tumour)]))
    return jobs


def alone(cfg, parts):
    with kc.KmerCounter(cfg) as c:
        for t, (b, o) in enumerate(parts):
            c.insert_reads(b, o, counter=t)
        st = c.finalize()
        keys, counts = c.export()
        b1, b2 = c.export_bloom()
    return dict(keys=keys, counts=counts, b1=b1, b2=b2, stats=st)


def served(resp, cfg):
    keys, counts = kc.response_table(resp, cfg.n_counters)
    words = max(1, (1 << cfg.bloom_bits_log2) // 64)
    b1, b2 = kc.kc_export_bloom(kc.ctypes.c_void_p(resp.ctx), words)
    st = resp.stats.as_dict()
    return dict(keys=keys, counts=counts, b1=b1, b2=b2, stats=st)


def same(a, b):
    assert_same_table(a["keys"], a["counts"], b["keys"], b["counts"])
    assert np.array_equal(a["b1"], b["b1"]) and np.array_equal(a["b2"], b["b2"])
    for k in ("n_valid", "n_pass", "entries", "sum_counts", "fp_singletons", "b1_popcount",
              "b2_popcount"):
        assert a["stats"][k] == b["stats"][k], k


def test_served_results_equal_alone_and_oracle():
    note("case: 24 joint jobs, 4 workers, tight budget, seed 71")
    jobs = make_jobs(71, 24)
    dev = [(cfg, [to_device(b, o) for b, o in parts]) for cfg, parts in jobs]
    ref = [alone(cfg, parts) for cfg, parts in dev]
    # a budget a few times the largest job: jobs queue and are admitted as others release
    est = max(r["stats"]["n_valid"] for r in ref)
    budget = 160 << 20
    seen = {"max_in_use": 0}
    stop = threading.Event()
    with kc.Server(budget, workers=4) as srv:
        def watch():
            while not stop.is_set():
                seen["max_in_use"] = max(seen["max_in_use"], srv.usage()["in_use"])
                time.sleep(0.0005)
        th = threading.Thread(target=watch)
        th.start()
        tickets = [srv.submit(cfg, parts) for cfg, parts in dev]
        results = []
        for t, (cfg, _), r in zip(tickets, dev, ref):
            resp = srv.wait(t)
            assert resp.status == kc.KC_OK, resp.status
            assert resp.footprint_bytes <= budget
            same(served(resp, cfg), r)
            results.append((resp.submit_ms, resp.admit_ms, resp.done_ms, resp.worker))
            srv.release(t)
        stop.set()
        th.join()
        u = srv.usage()
        assert u["in_use"] == 0 and u["queued"] == 0 and u["running"] == 0
        # freed context buffers stay in the server's block cache, within one budget
        assert 0 < u["device_allocs"] and u["cached_bytes"] <= budget
        assert u["device_allocs"] - u["device_frees"] >= 1
    assert seen["max_in_use"] <= budget
    workers = {r[3] for r in results}
    assert len(workers) > 1  # jobs ran on several workers
    # overlap: some job was admitted before an earlier-admitted one finished
    spans = sorted((a, d) for _, a, d, _ in results)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    note("max reserved %.1f MiB of %.1f MiB; largest job %d k-mers" % (
        seen["max_in_use"] / 2**20, budget / 2**20, est))
    # a subset against the oracle
    for cfg, parts in jobs[:4]:
        bases = np.concatenate([parts[0][0], parts[1][0]])
        o0, o1 = parts[0][1], parts[1][1]
        offs = np.concatenate([o0, o1[1:] + o0[-1]])
        tags = np.concatenate([np.zeros(o0.size - 1, np.uint8), np.ones(o1.size - 1, np.uint8)])
        r = oracle.count(oracle_params(cfg), bases, offs, tags=tags)
        g = alone(cfg, [to_device(*parts[0]), to_device(*parts[1])])
        assert_same_table(g["keys"], g["counts"], r.keys, r.counts)
        for a, b in STAT_MAP.items():
            assert g["stats"][a] == r.stats[b]


def test_server_admission_errors_and_resident_tables():
    import torch
    note("case: over-budget job, queries on resident tables until release, seed 72")
    (cfg, parts), = make_jobs(72, 1)
    dev = [to_device(b, o) for b, o in parts]
    big = kc.Config(k=31, n_counters=2, bloom_bits_log2=34, bloom_hashes=4, bloom_block_log2=19,
                    seed=1)
    with kc.Server(64 << 20, workers=2) as srv:
        t_big = srv.submit(big, dev)  # its Bloom levels alone exceed the budget
        assert srv.wait(t_big).status == kc.KC_ERR_OVER_BUDGET
        srv.release(t_big)
        t = srv.submit(cfg, dev)
        resp = srv.wait(t)
        assert resp.status == kc.KC_OK
        keys, counts = kc.response_table(resp, 2)
        q = torch.from_numpy(keys.view(np.int64)).cuda()
        got = kc.response_query(resp, q, 2).cpu().numpy().astype(np.uint32)
        assert np.array_equal(got, counts)
        assert srv.usage()["in_use"] > 0
        srv.release(t)
        assert srv.usage()["in_use"] == 0 and srv.usage()["pooled"] > 0
        with pytest.raises(kc.KcError):
            srv.release(t)
        # the pooled context serves the same configuration again
        t2 = srv.submit(cfg, dev)
        r2 = srv.wait(t2)
        assert r2.status == kc.KC_OK and r2.stats.entries == resp.stats.entries
        srv.release(t2)


def test_overlap_cap_bounds_work_in_flight():
    """kc_server_set_overlap: a request starts only when none runs or the
    running ones and it hold at most the cap in bases; results stay equal to
    the same jobs run alone."""
    note("case: 16 joint jobs, 4 workers, overlap cap of twice the median job, seed 73")
    jobs = make_jobs(73, 16)
    dev = [(cfg, [to_device(b, o) for b, o in parts]) for cfg, parts in jobs]
    ref = [alone(cfg, parts) for cfg, parts in dev]
    sizes = [sum(int(o[-1]) for _, o in parts) for _, parts in jobs]
    cap = 2 * int(np.median(sizes))
    with kc.Server(256 << 20, workers=4, overlap_bases=cap) as srv:
        tickets = [srv.submit(cfg, parts) for cfg, parts in dev]
        spans = []
        for t, (cfg, _), r, n in zip(tickets, dev, ref, sizes):
            resp = srv.wait(t)
            assert resp.status == kc.KC_OK, resp.status
            same(served(resp, cfg), r)
            spans.append((resp.admit_ms, resp.done_ms, n))
            srv.release(t)
    overlapped = 0
    for a, d, n in spans:
        running = [m for a2, d2, m in spans if a2 < a < d2]
        assert not running or sum(running) + n <= cap, (running, n, cap)
        overlapped += bool(running)
    assert overlapped > 0  # small jobs still ran side by side
    note("cap %d bases; %d of %d jobs started beside others" % (cap, overlapped, len(spans)))


def test_submit_orders_after_the_producing_stream_and_holds_the_reads():
    """Reads copied to the device on a side stream, behind a spinning kernel,
    are submitted at once as temporaries: the worker waits for that stream
    (the request's ready event) and the server binding keeps the tensors alive,
    so the memory the caller drops is not reused under the running job."""
    import torch
    note("case: 6 joint jobs, reads copied behind a spin kernel on a side stream, seed 74")
    jobs = make_jobs(74, 6)
    ref = [alone(cfg, [to_device(b, o) for b, o in parts]) for cfg, parts in jobs]
    side = torch.cuda.Stream()
    with kc.Server(256 << 20, workers=3) as srv:
        tickets = []
        with torch.cuda.stream(side):
            for cfg, parts in jobs:
                torch.cuda._sleep(20_000_000)
                dev = [(torch.from_numpy(b).pin_memory().to("cuda", non_blocking=True),
                        torch.from_numpy(o.view(np.int64)).pin_memory().to("cuda", non_blocking=True))
                       for b, o in parts]
                tickets.append(srv.submit(cfg, dev))
                del dev
            # memory the caller has dropped, written over while the jobs run
            junk = [torch.full((int(o[-1]) + 64,), 0xFF, dtype=torch.uint8, device="cuda")
                    for _, parts in jobs for _, o in parts]
        for t, (cfg, _), r in zip(tickets, jobs, ref):
            resp = srv.wait(t)
            assert resp.status == kc.KC_OK, resp.status
            same(served(resp, cfg), r)
            srv.release(t)
        del junk
    torch.cuda.synchronize()
