#!/usr/bin/env python3
"""Benchmark of the MI355X k-mer counter (default: the 100 Mbp plain workload).

One step = one pass of the whole counting path over the workload's reads,
already resident in HBM: reset, insert (pack, extraction, two-level partition
shuffle), finalize (Bloom levels, screen, exact per-partition count, unify)
and one query batch.  With --workload batched_200mbp the step is one
kc_count_batch graph launch over the 256 chunks (the autotuner picks the
configuration first, untimed) plus the query batch.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                  [--workload plain_100mbp|batched_200mbp|...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "plain_100mbp"
METRIC = "k-mers/sec + HBM GB/s (plain vs batched/served); p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 64 integer lanes per clock x 2.4 GHz (32-bit integer VALU issue rate)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
MIX64_OPS = 17          # VALU instructions of one SplitMix64 output function on gfx950
SLOT_HASH_OPS = 6       # table slot hash: xor, 64-bit multiply (4), multiply-high
QUERY_BATCH = 1 << 20
COPY_BYTES = 1 << 30
KERNEL_SRC = os.path.join(ROOT, "paper_1712_03254_amd", "csrc", "kc_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "count_traffic.json")
STAGE_KERNEL = {"pack": "k_pack", "level1": "k_level1", "level2": "k_level2", "bloom": "k_bloom",
                "tally": "k_tally", "query": "k_query"}


def src_hash() -> str:
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stage_alu_ops(stage: str, w, st: dict) -> float:
    """Algorithmic integer ops of one launch: k_bloom evaluates one hash per
    occurrence (the h bit positions follow from it by double hashing, 2 ops
    each); k_tally one slot hash per occurrence and one hash per screened key
    (occurrences of failing keys plus the first arrival of each passing key);
    the shuffle levels one hash per occurrence."""
    n = st["n_valid"]
    if stage == "bloom":
        return (MIX64_OPS + 2 * w.bloom_hashes) * n
    if stage == "tally":
        screened = (n - st["n_pass"]) + st["passed_distinct"]
        return (MIX64_OPS + 2 * w.bloom_hashes) * screened + SLOT_HASH_OPS * n
    if stage in ("level1", "level2"):
        return MIX64_OPS * n
    return 0.0


def stage_bytes(stage: str, w, st: dict, cfg_eff: dict) -> float:
    """Algorithmic HBM bytes of a stage over one step (the whole input): the
    per-k-mer terms of the shuffle-once design (input, shuffle, Bloom, table,
    output) that fall in that stage, times the units of the step.  N valid k-mers, B
    bases, W = B/32 packed words, m Bloom bits per level, E table entries:
      pack    ASCII read + packed and flag words written: B + 16 W
      level1  packed and flag words read + keys written: 16 W + 8 N
      level2  keys read and written (the second scatter level): 16 N
      bloom   keys read + both levels written once, read once: 8 N + 4 m/8
      tally   keys read + level 2 read + table initialised and read back at
              load factor 1/2 + entries written: 8 N + m/8 + 2*S*E/0.5 + S*E
              (S = 8 + 4 n_counters bytes per slot)
    """
    total_bases, n_reads = cfg_eff["total_bases"], cfg_eff["n_reads"]
    nwords = (total_bases + 31) // 32
    n = st["n_valid"]
    m = 1 << w.bloom_bits_log2
    slot = 8 + 4 * w.n_counters
    if stage == "pack":
        return total_bases + nwords * 16 + (n_reads + 1) * 8
    if stage == "level1":
        return nwords * 16 + n * 8
    if stage == "level2":
        return n * 16
    if stage == "bloom":
        return n * 8 + 4 * m // 8
    if stage == "tally":
        e = st["entries"]
        return n * 8 + m // 8 + 2 * slot * e / 0.5 + slot * e
    if stage == "query":
        return QUERY_BATCH * (8 + 4 * w.n_counters)
    if stage == "graph":     # every stage of the batch in one launch
        return sum(stage_bytes(x, w, st, cfg_eff) for x in ("pack", "level1", "level2", "bloom",
                                                             "tally"))
    return 0.0


def host_description() -> dict:
    """The host the CPU baseline ran on: logical CPUs, CPUs this process may
    use, CPU model and RAM."""
    model, mem_kb = "", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_kb = int(line.split()[1])
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model,
            "ram_gib": round(mem_kb / 2**20, 1)}


def cpu_baseline(w, genome, n_reads=3_000_000):
    """The CPU oracle on the host's cores: value-range passes over the first
    n_reads reads of the workload (threads split the reads, one value range of
    the k-mer space per thread, Bloom levels, screen and table), timed from
    reads in host memory to the final result.  Threads: the CPUs this process
    may use, at most 16 (the host share of one GPU).  Beside it, one core on
    the whole 1 Mbp workload."""
    import oracle
    b, o = w.make_reads(genome, first=0, n=n_reads, threads=16)
    p = oracle.Params(k=w.k, n_counters=w.n_counters, min_count=w.min_count,
                      m_log2=w.bloom_bits_log2, h=w.bloom_hashes, block_log2=w.bloom_block_log2,
                      seed=w.seed)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    r = oracle.count_ranges(p, b, o, want_bloom=False, threads=threads)
    dt = time.perf_counter() - t0
    del b, o
    import synth
    w1 = synth.WORKLOADS["plain_1mbp"]
    g1 = w1.make_genome()
    b1, o1 = w1.make_reads(g1)
    p1 = oracle.Params(k=w1.k, m_log2=w1.bloom_bits_log2, h=w1.bloom_hashes,
                       block_log2=w1.bloom_block_log2, seed=w1.seed)
    t1 = time.perf_counter()
    r1 = oracle.count(p1, b1, o1, want_bloom=False)
    dt1 = time.perf_counter() - t1
    return {"value": r.stats["n_valid"] / dt, "unit": "k-mers/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %d reads of %s (%d k-mers, %.1f%% of the workload): value-range "
                      "passes on %d threads, sort + run-length count, Bloom levels, screen and "
                      "table in %.1f s"
                      % (n_reads, w.name, r.stats["n_valid"], 100.0 * n_reads / w.n_reads,
                         threads, dt),
            "host": host_description(),
            "single_core_1mbp": {"value": r1.stats["n_valid"] / dt1, "unit": "k-mers/s",
                                 "seconds": round(dt1, 2), "kmers": r1.stats["n_valid"]}}


def atomic_summary(w, st: dict, stages: dict) -> dict:
    """LDS atomic throughput of the Bloom and count kernels against the
    microbenchmark peak (libkc_probe.so) under their access pattern: random
    words of a block-sized array.  k_bloom issues h ORs with return per
    occurrence (the second-level ORs for bits already set are not counted);
    k_tally one add per passing occurrence and one CAS per inserted key."""
    from paper_1712_03254_amd import probe
    # one Bloom workgroup's level: up to four blocks smaller than 2^18 bits
    bl = w.bloom_block_log2
    bsub = min(2, 18 - bl) if 5 <= bl < 18 else 0
    bloom_words_log2 = max(6, min(15, bl - 5 + bsub))
    table_words_log2 = 12  # the count words of a ~3840-slot table
    peak_or = probe.lds_atomic_peak(probe.KCP_OR_RTN, bloom_words_log2)
    peak_add = probe.lds_atomic_peak(probe.KCP_ADD, table_words_log2)
    out = {"probe": {"or_rtn_per_s": peak_or, "or_words_log2": bloom_words_log2,
                     "add_per_s": peak_add, "add_words_log2": table_words_log2}}
    n = st["n_valid"]
    if "bloom" in stages:
        ops = w.bloom_hashes * n
        rate = ops / (stages["bloom"]["avg_ms"] * 1e-3)
        out["k_bloom"] = {"ops": ops, "per_s": rate, "frac": round(rate / peak_or, 4)}
    if "tally" in stages:
        ops = st["n_pass"] + st["passed_distinct"]
        rate = ops / (stages["tally"]["avg_ms"] * 1e-3)
        out["k_tally"] = {"ops": ops, "per_s": rate, "frac": round(rate / peak_add, 4)}
    return out


def stem_relayout(counter, reps: int = 3) -> dict:
    """kc_export_stems on the finalized table (Unify's stem items), outside the
    timed steps: HIP-event time of the call (three passes over the table
    slots, a prefix sum over the stem table), items written, and the output
    rate (72 B per item: 8 B stem, 32 two-byte counts)."""
    import torch
    counter.export_stems()
    torch.cuda.synchronize()
    before = counter.stats()["kernel_ms"]["stems"]
    t0 = time.perf_counter()
    for _ in range(reps):
        stems, _ = counter.export_stems()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ms = (counter.stats()["kernel_ms"]["stems"] - before) / reps
    n = int(stems.numel())
    del stems
    torch.cuda.empty_cache()
    return {"items": n, "entries": counter.stats()["entries"], "ms": round(ms, 3),
            "wall_ms": round(wall * 1e3, 3), "items_per_s": n / (ms * 1e-3),
            "out_gbs": round(n * 72 / (ms * 1e-3) / 1e9, 1)}


def filter_lookup(counter, chunks, n_valid: int, reps: int = 3) -> dict:
    """kc_filter_reads on the finalized table, re-reading the same resident
    reads (the Filter unit's second pass over the input), outside the timed
    steps: HIP-event time, window lookups per second and the selected
    windows (threshold: count >= 2, no normal counter)."""
    import torch
    b, o = chunks[0]
    counter.filter_reads(b, o, 2, 0)
    torch.cuda.synchronize()
    before = counter.stats()["kernel_ms"]["filter"]
    for _ in range(reps):
        sel = counter.filter_reads(b, o, 2, 0)
    torch.cuda.synchronize()
    ms = (counter.stats()["kernel_ms"]["filter"] - before) / reps
    picked = int(sel.to(torch.int64).sum().item())
    return {"windows": n_valid, "selected": picked, "ms": round(ms, 3),
            "lookups_per_s": n_valid / (ms * 1e-3)}


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or was taken on different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("src_sha256") != src_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes")


def _pmc_rows(directory: str):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    return rows


def _kernel_key(name: str):
    for k in STAGE_KERNEL.values():
        if k + "<" in name or k + "(" in name or name.endswith(k):
            return k
    return "copy" if "copy" in name.lower() else None


def pmc_summary(fetch_dir: str, write_dir: str, command: str):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the stage kernels and of
    the calibration copy; writes profiles/count_traffic.json and a markdown
    note.  Each counter is scaled by what it reads for a copy of known size."""
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in _pmc_rows(d):
            if r["Counter_Name"] != counter:
                continue
            key = _kernel_key(r["Kernel_Name"])
            if key:
                per.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)
        res[counter] = per
    copy_f = max(res["FETCH_SIZE"]["copy"])
    copy_w = max(res["WRITE_SIZE"]["copy"])
    f_factor, w_factor = copy_f / COPY_BYTES, copy_w / COPY_BYTES
    kernels = {}
    for k in STAGE_KERNEL.values():
        if k in res["FETCH_SIZE"] and k in res["WRITE_SIZE"]:
            rf, rw = np.median(res["FETCH_SIZE"][k]), np.median(res["WRITE_SIZE"][k])
            kernels[k] = {"fetch_raw": rf, "write_raw": rw, "fetch_bytes": rf / f_factor,
                          "write_bytes": rw / w_factor,
                          "traffic_bytes": rf / f_factor + rw / w_factor,
                          "launches": len(res["FETCH_SIZE"][k])}
    out = {"workload": WORKLOAD, "src_sha256": src_hash(), "copy_bytes": COPY_BYTES,
           "copy_fetch_raw": copy_f, "copy_write_raw": copy_w,
           "copy_fetch_factor": f_factor, "copy_write_factor": w_factor,
           "kernels": kernels, "command": command}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    md = os.path.join(ROOT, "profiles", "%s_hbm_traffic.md" % WORKLOAD)
    with open(md, "w") as f:
        f.write("# HBM traffic per launch, %s workload (rocprofv3 --pmc)\n\n" % WORKLOAD)
        f.write("Commands (FETCH_SIZE run, then WRITE_SIZE run):\n\n```\n%s\n```\n\n" % command)
        f.write("Calibration: a %d-byte device copy reads FETCH_SIZE %.4e B and WRITE_SIZE %.4e B, "
                "so the factors are %.4f and %.4f.\n\n" % (COPY_BYTES, copy_f, copy_w, f_factor,
                                                            w_factor))
        f.write("| kernel | FETCH raw | WRITE raw | read bytes | written bytes | total |\n"
                "|---|---|---|---|---|---|\n")
        for k, v in kernels.items():
            f.write("| %s | %.3e | %.3e | %.3e | %.3e | %.3e |\n" % (
                k, v["fetch_raw"], v["write_raw"], v["fetch_bytes"], v["write_bytes"],
                v["traffic_bytes"]))
        f.write("\nkc_kernels.hip sha256: `%s`\n" % out["src_sha256"])
    print(json.dumps(out))


def trace_summary(trace_dir: str, command: str):
    import csv
    import glob
    paths = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(paths[0])))
    md = os.path.join(ROOT, "profiles", "plain_100mbp_kernel_stats.md")
    with open(md, "w") as f:
        f.write("# Kernel time, %s workload (rocprofv3 --kernel-trace --stats)\n\n" % WORKLOAD)
        f.write("Command:\n\n```\n%s\n```\n\n" % command)
        f.write("| kernel | calls | total ms | average us | share % |\n|---|---|---|---|---|\n")
        for r in rows:
            f.write("| %s | %s | %.3f | %.1f | %.2f |\n" % (
                r["Name"][:60], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
        f.write("\nkc_kernels.hip sha256: `%s`\n" % src_hash())
    print(open(md).read())


def served_main(args, w):
    """The served workload: 512 joint (normal, tumour) count requests of
    log-uniform size through the request server under its HBM budget.
    "plain" = the same requests through a one-worker server (one job at a
    time, no overlap); "served" = concurrent workers.  Reports closed-loop
    throughput of both and p50/p99 latency under Poisson arrivals at offered
    loads rho x the plain capacity."""
    import threading
    import torch
    import paper_1712_03254_amd as kc

    kc.load()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    normal = w.make_genome(threads=16)
    tum = w.make_tumour(normal)
    reads = [w.make_sample_reads(normal, 0, threads=16), w.make_sample_reads(tum, 1, threads=16)]
    del normal, tum
    gen_s = time.perf_counter() - t0
    L = w.lmax
    assert w.lmin == w.lmax  # fixed-length reads: a slice's offsets are a prefix of the first
    dev_b = [torch.from_numpy(b).to(dev) for b, _ in reads]
    offs = torch.from_numpy(reads[0][1].view(np.int64)).to(dev)
    del reads
    plan = w.request_plan()

    def request(i):
        n, s0, s1 = (int(v) for v in plan[i])
        half = n // 2
        kmers, m, pl = w.request_params(n)
        cfg = kc.Config(k=w.k, n_counters=2, min_count=w.min_count, bloom_bits_log2=m,
                        bloom_hashes=w.bloom_hashes, bloom_block_log2=w.bloom_block_log2,
                        seed=w.seed, partitions_log2=pl)
        parts = [(dev_b[0][s0 * L:(s0 + half) * L], offs[:half + 1]),
                 (dev_b[1][s1 * L:(s1 + half) * L], offs[:half + 1])]
        return cfg, parts, kmers

    reqs = [request(i) for i in range(plan.shape[0])]
    warm, timed = reqs[:w.warmup_requests], reqs[w.warmup_requests:]
    total_kmers = sum(r[2] for r in timed)
    mean_kmers = total_kmers / len(timed)

    def run(srv, jobs, arrivals=None):
        """Submits jobs (at arrival offsets in seconds, or all at once);
        collectors wait and release each as it finishes."""
        tickets = [None] * len(jobs)
        ready = [threading.Event() for _ in jobs]
        out = [None] * len(jobs)
        nxt = {"i": 0}
        lock = threading.Lock()

        def collect():
            while True:
                with lock:
                    i = nxt["i"]
                    nxt["i"] += 1
                if i >= len(jobs):
                    return
                ready[i].wait()
                r = srv.wait(tickets[i])
                out[i] = (r.status, r.submit_ms, r.admit_ms, r.done_ms, r.worker)
                srv.release(tickets[i])

        cols = [threading.Thread(target=collect) for _ in range(2 * args.serve_workers)]
        for c in cols:
            c.start()
        start = time.perf_counter()
        for i, (cfg, parts, _) in enumerate(jobs):
            if arrivals is not None:
                wait = start + arrivals[i] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
            tickets[i] = srv.submit(cfg, parts)
            ready[i].set()
        for c in cols:
            c.join()
        assert all(o[0] == 0 for o in out), [o[0] for o in out if o[0]]
        lat = np.array([o[3] - o[1] for o in out])
        svc = np.array([o[3] - o[2] for o in out])
        span_ms = max(o[3] for o in out) - min(o[1] for o in out)
        u = srv.usage()
        return {"kmers_per_s": total_kmers / (span_ms * 1e-3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "mean_ms": round(float(lat.mean()), 2), "span_ms": round(span_ms, 1),
                "mean_service_ms": round(float(svc.mean()), 2),
                "contexts": {k: u[k] for k in ("created", "reused", "grown", "evicted",
                                               "pooled_contexts", "cached_bytes",
                                               "device_allocs", "device_frees")}}

    budget = w.serve_budget
    res = {}
    overlap = int(args.serve_overlap)
    with kc.Server(budget, workers=1) as plain, \
            kc.Server(budget, workers=args.serve_workers, overlap_bases=overlap) as srv:
        # warm-up: the warm requests, then one untimed pass of the timed set, so
        # both servers' context pools hold contexts for every request size
        for server in (plain, srv):
            run(server, warm)
            run(server, timed)
        closed_plain = run(plain, timed)
        closed = run(srv, timed)
        cap = closed_plain["kmers_per_s"]
        rng = np.random.default_rng(w.seed)
        gaps = rng.exponential(1.0, len(timed))
        for rho in args.loads:
            lam = rho * cap / mean_kmers  # requests per second
            arr = np.cumsum(gaps) / lam
            res[str(rho)] = {"served": run(srv, timed, arr), "plain": run(plain, timed, arr)}
            print("rho %.1f: %s" % (rho, res[str(rho)]), file=sys.stderr, flush=True)
    best = max([closed] + [v["served"] for v in res.values()], key=lambda d: d["kmers_per_s"])
    out = {
        "metric": METRIC, "value": closed["kmers_per_s"], "unit": "k-mers/s", "n_gpus": 1,
        "steps": len(timed), "warmup": len(warm),
        "ms_per_step": closed["span_ms"] / len(timed), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": w.name, "genome_bp": w.genome_len, "reads_per_sample": w.n_reads,
                   "read_len": L, "requests": len(timed), "request_reads": [w.req_lo, w.req_hi],
                   "k": w.k, "bloom_hashes": w.bloom_hashes,
                   "bloom_block_log2": w.bloom_block_log2, "n_counters": 2,
                   "hbm_budget_bytes": budget, "workers": args.serve_workers,
                   "overlap_bases": overlap,
                   "mean_request_kmers": mean_kmers},
        "served_closed_loop": closed,
        "plain_closed_loop": closed_plain,
        "served_vs_plain": round(closed["kmers_per_s"] / cap, 3),
        "latency_by_offered_load": res,
        "best_served_kmers_per_s": best["kmers_per_s"],
        "input_gen_s": round(gen_s, 2),
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run %d-byte device copies (counter calibration)" % COPY_BYTES)
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="offline: turn two rocprofv3 --pmc runs into profiles/ files")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="offline: turn a rocprofv3 --kernel-trace --stats run into a profiles/ file")
    ap.add_argument("--command", default="", help="command line recorded in the offline summaries")
    ap.add_argument("--serve-workers", type=int, default=8,
                    help="served workload: concurrent jobs (server worker threads)")
    ap.add_argument("--serve-overlap", type=float, default=float(1 << 28),
                    help="served workload: admission cap on the bases of requests running at "
                         "once (0: none)")
    ap.add_argument("--checkpoint", default="",
                    help="plain workloads: also time kc_checkpoint to this path and kc_restore from it")
    ap.add_argument("--loads", type=float, nargs="*", default=[0.3, 0.5, 0.7, 0.9],
                    help="served workload: offered loads as fractions of the plain capacity")
    ap.add_argument("--legs", default="",
                    help="comma-separated extra workloads run after the main one, each in a child "
                         "process, their results added to the line (batched,served,large); default: "
                         "all three with the default workload, none otherwise")
    ap.add_argument("--lean", action="store_true",
                    help="skip the stem, filter and atomics extras after the timed steps")
    ap.add_argument("--spill-budget-gib", type=float, default=0.0,
                    help="plain workloads: after the timed steps, count once more under this HBM "
                         "table budget and report the spill")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.command)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.command)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the counting path runs on a single MI355X "
              "(sharding by partition prefix across GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    if w.requests:
        out = served_main(args, w)
    else:
        out = count_main(args, w)
    legs = args.legs if args.legs else ("batched,served,large" if args.workload == WORKLOAD
                                        else "none")
    for leg in [x for x in legs.split(",") if x and x != "none"]:
        out[leg] = run_leg(leg, args)
    print(json.dumps(out), flush=True)


def count_main(args, w) -> dict:
    """Plain and batched workloads: warm-up, then the timed steps."""
    import torch
    import paper_1712_03254_amd as kc
    kc.load()
    batched = w.batch_chunks > 0
    t0 = time.perf_counter()
    genome = w.make_genome(threads=16)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if batched:
        sizes = w.chunk_plan()
        host_chunks = [w.make_chunk(genome, sizes, i, threads=16) for i in range(sizes.size)]
        n_reads = int(sizes.sum())
        total_bases = int(sum(int(o[-1]) for _, o in host_chunks))
    else:
        # one insert takes fewer than 2^32 bases: larger inputs go in as
        # consecutive slices of the read stream
        per = w.n_reads
        while per * w.lmax >= 1 << 32:
            per = (per + 1) // 2
        host_chunks = [w.make_reads(genome, first=f, n=min(per, w.n_reads - f), threads=16)
                       for f in range(0, w.n_reads, per)]
        n_reads = w.n_reads
        total_bases = int(sum(int(o[-1]) for _, o in host_chunks))
    gen_s = time.perf_counter() - t0
    pinned = [(torch.from_numpy(b).pin_memory(), torch.from_numpy(o.view(np.int64)).pin_memory())
              for b, o in host_chunks]
    chunks = [(b.to(dev, non_blocking=True), o.to(dev, non_blocking=True)) for b, o in pinned]
    torch.cuda.synchronize()
    cfg = kc.Config(k=w.k, n_counters=w.n_counters, min_count=w.min_count,
                    bloom_bits_log2=w.bloom_bits_log2, bloom_hashes=w.bloom_hashes,
                    bloom_block_log2=w.bloom_block_log2, seed=w.seed,
                    partitions_log2=w.partitions_log2, hbm_table_budget_bytes=w.table_budget)
    tune = None
    if batched:
        # the autotuner's trials run here, before warm-up and outside the timed steps
        t_tune = time.perf_counter()
        cfg, trials = kc.autotune_batch(cfg, chunks, stream=stream)
        tune = {"chosen": {"partitions_log2": cfg.partitions_log2, "table_slots": cfg.table_slots,
                           "scatter_bits": cfg.scatter_bits,
                           "shuffle_tile_log2": cfg.shuffle_tile_log2},
                "trials": [[t["partitions_log2"], t["table_slots"], t["scatter_bits"],
                            t["shuffle_tile_log2"], round(t["ms"], 3), t["status"]]
                           for t in trials],
                "seconds": round(time.perf_counter() - t_tune, 1)}
    counter = kc.KmerCounter(cfg)

    def count(src):
        counter.reset()
        if batched:
            return counter.count_batch(src, stream=stream)
        for b, o in src:
            counter.insert_reads(b, o, stream=stream)
        return counter.finalize(stream=stream)

    def step(q=None):
        st = count(chunks)
        if q is not None:
            counter.query(q, stream=stream)
        return counter.stats() if q is not None else st

    # query batch: half present (from the table), half random codes (all random
    # when the table is too large to copy to the host in passing)
    first = step()
    rng = np.random.default_rng(1)
    half = QUERY_BATCH // 2 if first["entries"] <= 1 << 28 else 0
    present = np.zeros(0, np.uint64)
    if half:
        keys, _ = counter.export()
        present = keys[rng.integers(0, keys.size, half)]
        del keys
    qk = np.concatenate([present, rng.integers(0, 1 << (2 * w.k), QUERY_BATCH - half,
                                               dtype=np.uint64)])
    q = torch.from_numpy(qk.view(np.int64)).to(dev)
    for _ in range(args.warmup):
        step(q)
    torch.cuda.synchronize()
    per_stage_ms = {}
    per_stage_n = {}
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = step(q)
        for s_, v in last["kernel_ms"].items():
            per_stage_ms[s_] = per_stage_ms.get(s_, 0.0) + v
            per_stage_n[s_] = per_stage_n.get(s_, 0) + last["kernel_launches"][s_]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_valid = last["n_valid"]
    value = n_valid * args.steps / elapsed

    # end-to-end figure with the reads crossing PCIe from pinned host memory
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fresh = [(b.to(dev, non_blocking=True), o.to(dev, non_blocking=True)) for b, o in pinned]
    count(fresh)
    torch.cuda.synchronize()
    e2e = n_valid / (time.perf_counter() - t1)
    del fresh

    plain_same = None
    if batched:
        # the same resident chunks and configuration through the plain path
        # (one kc_insert_reads per chunk, then kc_finalize); after this the
        # context holds no graph, so it runs last
        def plain_step():
            counter.reset()
            for b, o in chunks:
                counter.insert_reads(b, o, stream=stream)
            return counter.finalize(stream=stream)
        plain_step()
        torch.cuda.synchronize()
        reps = max(1, min(3, args.steps))
        t2 = time.perf_counter()
        for _ in range(reps):
            pst = plain_step()
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t2) / reps
        assert pst["n_valid"] == n_valid and pst["entries"] == last["entries"]
        plain_same = {"value": n_valid / pdt, "ms_per_step": round(pdt * 1e3, 2), "steps": reps,
                      "batched_over_plain": round(value / (n_valid / pdt), 3)}
        # ... and with the chunks concatenated on the device (untimed) into as few
        # inserts as the 2^32-base limit of one insert allows: the plain path
        # without per-chunk calls
        segs, cur_b, cur_o, base = [], [], [], 0
        for b, o in chunks:
            if cur_b and base + b.numel() >= (1 << 32):
                segs.append((torch.cat(cur_b), torch.cat(cur_o)))
                cur_b, cur_o, base = [], [], 0
            cur_o.append(o[(1 if cur_o else 0):] + base)
            cur_b.append(b)
            base += b.numel()
        if cur_b:
            segs.append((torch.cat(cur_b), torch.cat(cur_o)))
        torch.cuda.synchronize()
        # a context of its own (the first one holds the batch plan's and the
        # per-chunk inserts' key segments)
        counter.close()
        solo = kc.KmerCounter(cfg)

        def concat_step():
            solo.reset()
            for b, o in segs:
                solo.insert_reads(b, o, stream=stream)
            return solo.finalize(stream=stream)
        concat_step()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(reps):
            cst = concat_step()
        torch.cuda.synchronize()
        cdt = (time.perf_counter() - t3) / reps
        assert cst["n_valid"] == n_valid and cst["entries"] == last["entries"]
        plain_same["concatenated"] = {"value": n_valid / cdt, "ms_per_step": round(cdt * 1e3, 2),
                                      "inserts": len(segs),
                                      "batched_over_plain": round(value / (n_valid / cdt), 3)}
        solo.close()
        del segs

    cfg_eff = {"partitions_log2": last["partitions_log2"], "table_slots": last["table_slots"],
               "total_bases": total_bases, "n_reads": n_reads}
    stages = {}
    for s in per_stage_ms:
        if per_stage_n.get(s):
            avg = per_stage_ms[s] / per_stage_n[s]
            # stage_bytes covers the whole input; a stage launched once per insert
            # (or per spill wave) moves its share of it per launch
            b = stage_bytes(s, w, last, cfg_eff) / (per_stage_n[s] / args.steps)
            ops = stage_alu_ops(s, w, last)
            stages[s] = {"avg_ms": round(avg, 4), "launches_per_step": per_stage_n[s] / args.steps,
                         "alg_bytes": b,
                         "gbs": round(b / (avg * 1e-3) / 1e9, 1) if b and avg > 0 else None,
                         "alu_tops": round(ops / (avg * 1e-3) / 1e12, 3) if ops and avg > 0 else None}
    dom = max(stages, key=lambda s: stages[s]["avg_ms"] * stages[s]["launches_per_step"])
    d = stages[dom]
    hbm_frac = d["gbs"] / HBM_PEAK_GBS if d["gbs"] else 0.0
    roofline = {"bound": "hbm", "kernel": STAGE_KERNEL.get(dom, dom), "achieved": d["gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": None,
                "time_source": "HIP events on the launch stream, averaged over the timed steps",
                "alg_bytes_per_launch": d["alg_bytes"], "avg_ms": d["avg_ms"]}
    ops = stage_alu_ops(dom, w, last)
    if ops:
        tops = ops / (d["avg_ms"] * 1e-3) / 1e12
        roofline["alu_tops"] = round(tops, 3)
        roofline["alu_frac"] = round(tops / ALU_PEAK_TOPS, 4)
        roofline["hbm_gbs"] = d["gbs"]
        roofline["hbm_frac"] = round(hbm_frac, 4)
        if tops / ALU_PEAK_TOPS > hbm_frac:
            roofline.update({"bound": "alu", "achieved": round(tops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                             "unit": "T int-ops/s", "frac": round(tops / ALU_PEAK_TOPS, 4)})
    traffic = load_traffic(roofline["kernel"])
    if traffic is not None:
        roofline["traffic"] = traffic
    total_alg = sum(v["alg_bytes"] * v["launches_per_step"] for v in stages.values())

    out = {
        "metric": METRIC, "value": value, "unit": "k-mers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "genome_bp": w.genome_len, "reads": n_reads,
                   "bases": total_bases, "chunks": len(host_chunks),
                   "read_len": [w.lmin, w.lmax], "sub_rate": w.err, "n_rate": w.nrate, "k": w.k,
                   "bloom_bits_log2": w.bloom_bits_log2, "bloom_hashes": w.bloom_hashes,
                   "bloom_block_log2": w.bloom_block_log2,
                   "partitions": 1 << cfg_eff["partitions_log2"],
                   "table_slots": cfg_eff["table_slots"], "query_batch": QUERY_BATCH},
        "roofline": roofline,
        "stages": stages,
        "counts": {k: last[k] for k in ("n_valid", "n_pass", "entries", "sum_counts",
                                        "fp_singletons", "b1_popcount", "b2_popcount",
                                        "overflow_keys")},
        "pcie_inclusive_kmers_per_s": e2e,
        "step_alg_bytes_per_kmer": round(total_alg / n_valid, 2),
        "step_hbm_gbs": round(total_alg * args.steps / elapsed / 1e9, 1),
        "input_gen_s": round(gen_s, 2),
    }
    if tune is not None:
        out["autotune"] = tune
    if plain_same is not None:
        out["plain_same_workload"] = plain_same
    if not batched and not args.lean:
        out["atomics"] = atomic_summary(w, last, stages)
        out["stem_relayout"] = stem_relayout(counter)
        out["filter_lookup"] = filter_lookup(counter, chunks, n_valid)
    if not batched and args.checkpoint:
        t_a = time.perf_counter()
        counter.checkpoint(args.checkpoint)
        t_b = time.perf_counter()
        with kc.KmerCounter.restore(args.checkpoint) as back:
            torch.cuda.synchronize()
            t_c = time.perf_counter()
            same = all(back.stats()[k] == last[k] for k in ("entries", "sum_counts", "n_valid",
                                                              "fp_singletons", "b2_popcount"))
        size = os.path.getsize(args.checkpoint)
        os.remove(args.checkpoint)
        out["checkpoint"] = {"bytes": size, "write_s": round(t_b - t_a, 3),
                             "restore_s": round(t_c - t_b, 3),
                             "write_gbs": round(size / (t_b - t_a) / 1e9, 2),
                             "restore_gbs": round(size / (t_c - t_b) / 1e9, 2),
                             "restored_stats_equal": same}
    if args.copy_probe:
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    counter.close()
    if not batched and args.spill_budget_gib:
        # the same count under a table budget smaller than all tables: the
        # partitions past the budget are counted in waves and spilled to
        # pinned host memory
        import dataclasses
        scfg = dataclasses.replace(cfg, hbm_table_budget_bytes=int(args.spill_budget_gib * 2**30))
        with kc.KmerCounter(scfg) as sc:
            def spill_count():
                sc.reset()
                for b, o in chunks:
                    sc.insert_reads(b, o, stream=stream)
                return sc.finalize(stream=stream)
            spill_count()
            torch.cuda.synchronize()
            t_s = time.perf_counter()
            sst = spill_count()
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t_s
        out["spill"] = {"budget_bytes": scfg.hbm_table_budget_bytes,
                        "kmers_per_s": sst["n_valid"] / dt_s, "ms": round(dt_s * 1e3, 1),
                        "spilled_partitions": sst["spilled_partitions"],
                        "spilled_bytes": sst["spilled_bytes"],
                        "kernel_ms": {k: round(v, 2) for k, v in sst["kernel_ms"].items() if v},
                        "same_result": all(sst[k] == last[k] for k in (
                            "n_valid", "n_pass", "entries", "sum_counts", "fp_singletons",
                            "b1_popcount", "b2_popcount"))}
    del chunks, pinned, q
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, genome)
    return out


LEG_WORKLOAD = {"batched": "batched_200mbp", "served": "served_300mbp", "large": "spill_3gbp"}


def run_leg(leg: str, args) -> dict:
    """One extra workload in a child process (its own device memory), reduced
    to the figures that compare it with the plain path."""
    import subprocess
    wl = LEG_WORKLOAD[leg]
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", wl, "--legs", "none",
           "--no-cpu-baseline"]
    if leg == "batched":
        cmd += ["--steps", "3", "--warmup", "1"]
    elif leg == "large":
        cmd += ["--steps", "2", "--warmup", "1", "--lean", "--spill-budget-gib", "24"]
    print("leg %s: %s" % (leg, " ".join(cmd[1:])), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    wall = round(time.perf_counter() - t0, 1)
    lines = [l for l in res.stdout.splitlines() if l.startswith("{")]
    if res.returncode != 0 or not lines:
        return {"workload": wl, "status": "failed", "rc": res.returncode, "wall_s": wall}
    r = json.loads(lines[-1])
    print("leg %s done in %.1f s" % (leg, wall), file=sys.stderr, flush=True)
    if leg == "served":
        return {"workload": wl, "wall_s": wall,
                "served_kmers_per_s": r["served_closed_loop"]["kmers_per_s"],
                "plain_kmers_per_s": r["plain_closed_loop"]["kmers_per_s"],
                "served_vs_plain": r["served_vs_plain"],
                "closed_loop_p99_ms": {"served": r["served_closed_loop"]["p99_ms"],
                                       "plain": r["plain_closed_loop"]["p99_ms"]},
                "latency_by_offered_load": {
                    rho: {side: {k: v[side][k] for k in ("p50_ms", "p99_ms", "kmers_per_s")}
                          for side in ("served", "plain")}
                    for rho, v in r["latency_by_offered_load"].items()},
                "config": r["config"]}
    out = {"workload": wl, "wall_s": wall, "value": r["value"], "unit": r["unit"],
           "ms_per_step": r["ms_per_step"], "roofline": r["roofline"],
           "stages_ms": {k: v["avg_ms"] * v["launches_per_step"] for k, v in r["stages"].items()},
           "step_alg_bytes_per_kmer": r["step_alg_bytes_per_kmer"],
           "step_hbm_gbs": r["step_hbm_gbs"], "counts": r["counts"], "config": r["config"]}
    for k in ("plain_same_workload", "autotune", "spill"):
        if k in r:
            out[k] = r[k]
    if "plain_same_workload" in r:
        out["batched_over_plain"] = r["plain_same_workload"]["batched_over_plain"]
        if "concatenated" in r["plain_same_workload"]:
            out["batched_over_plain_concatenated"] = \
                r["plain_same_workload"]["concatenated"]["batched_over_plain"]
    return out


if __name__ == "__main__":
    main()
