"""Benchmark: unique formula semantics enumerated per second on one MI355X.

Workload (the medium synthesis problem): 3 atomic propositions, 32 positive
and 32 negative traces of lengths 8..32, per-proposition bit rates drawn from
U(0.3, 0.7), labels from a planted formula of cost 11 (seed 1).  The plain
solve of this problem stops at its minimal cost, which is small, so one
benchmark step is the whole hot path run exhaustively: encode, seed, and every
cost level 1..--bound generated, deduplicated and checked (the enumeration
does not stop at the first separating level).  The specification is uploaded
once before timing (inputs resident in HBM); each step is one ltlf_run.

value = sum over levels of |U_c| / step time.  Also reported: time to
formula of the plain solve (upload + enumeration to the minimal cost +
witness) on the medium problems of seeds 1..4, the roofline of the dominant
kernel (generation) from HIP events around its launches, the CPU oracle
on a bounded sample of the same problem, and the batched configuration
(256 problems of mixed shape) solved one by one and in one
ltlf_solve_batch call, and a served stream (Poisson arrivals) through the
request server and one at a time, with identical results required.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def profiled_traffic(kernel_prefix: str, workload_tag: str):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    summary (profiles/*.txt), if that summary was taken on the current kernel
    source (same sha256) and workload; else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2504_18943_amd", "csrc", "ltlf_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        fields = {}
        for line in open(path):
            if ":" in line:
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
        if (fields.get("kernel_source_sha256") == sha and workload_tag in fields.get("command", "")
                and fields.get("dominant_kernel", "").startswith(kernel_prefix)
                and "traffic_bytes_per_launch" in fields):
            return float(fields["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def large_config(synth, bound: int):
    """Large configuration (5 props, 512+512 traces, lengths 16-64, seed 1):
    every level to `bound` (its 328-chunk rows run on the wave kernel);
    unique semantics per second and the generation kernels' algorithmic
    GB/s, (row bytes + 8) per candidate over their summed launch time."""
    import torch
    import workload

    p = workload.large(1)
    synth.load(p)
    synth.run(bound, flags=0x1)  # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    r = synth.run(bound, flags=0x1 | 0x2)  # EXHAUST | PROFILE
    torch.cuda.synchronize()
    ms = (time.perf_counter() - a) * 1e3
    gbs = r.candidates * (r.row_bytes + 8) / (r.gen_ms / 1e3) / 1e9 if r.gen_ms > 0 else 0.0
    log(f"[bench] large config to cost {bound}: {ms:.1f} ms, {gbs:.0f} GB/s")
    # the configuration's own solve: bound 16, stop at the first separating level
    torch.cuda.synchronize()
    a = time.perf_counter()
    sol = synth.solve(p)
    torch.cuda.synchronize()
    ttf = (time.perf_counter() - a) * 1e3
    return {"workload": "large synthesis problem (5 props, 512+512 traces, lengths 16-64, planted cost 13, seed 1)",
            "cost_bound": bound, "row_bytes": r.row_bytes, "ms": round(ms, 2),
            "unique_per_s": round(r.unique_total / (ms / 1e3), 1), "unique_per_level": r.level_counts[1:bound + 1],
            "candidates": r.candidates, "gen_ms": round(r.gen_ms, 3), "kernel_bound": "hbm",
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "solve": {"cost_bound": p.cost_bound, "status": sol.status_name, "min_cost": sol.min_cost,
                      "formula": sol.formula, "time_to_formula_ms": round(ttf, 2),
                      "includes": "host-to-device upload of the specification"}}


def profiled_counters(kernel_prefix: str, workload_tag: str):
    """Per-launch hardware counters (atomics, L2 requests, hits, misses) of
    the dominant kernel from a committed rocprofv3 summary taken on the
    current kernel source and workload; else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2504_18943_amd", "csrc", "ltlf_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        fields = {}
        for line in open(path):
            if ":" in line:
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
        if (fields.get("kernel_source_sha256") == sha and workload_tag in fields.get("command", "")
                and fields.get("dominant_kernel", "").startswith(kernel_prefix)
                and "TCC_ATOMIC_sum_per_launch" in fields):
            return ({k: float(v) for k, v in fields.items() if k.endswith("_per_launch") or k.endswith("_weighted")},
                    os.path.basename(path))
    return None, None


def cpu_baseline(seed: int, bound: int):
    import oracle
    import workload

    p = workload.medium(seed)
    t0 = time.perf_counter()
    r = oracle.solve(p, cost_bound=bound, exhaust=True)
    wall = time.perf_counter() - t0
    uniq = sum(r.level_counts[1: r.levels_done + 1])
    return {"value": uniq / r.seconds, "unit": "unique semantics/s", "cores": 1, "kind": "oracle",
            "sample": f"medium seed {seed}, every level to cost {bound} ({uniq} unique CMs, "
                      f"{r.candidates} candidates), single-threaded C, {r.seconds:.2f} s "
                      f"enumeration, {wall:.2f} s wall"}


def compare_results(ps, xs, ys):
    """Exactness of two solves of the same problems (one by one against
    batched or served).  Per problem, every level both sides stored has the
    same count and the same digest (the set of CMs); with no overflow on
    either side, status, minimal cost, levels_done and every count and
    digest are identical.  A side whose store overflowed (the scheduler's
    large region is smaller than the whole workspace) may differ only as an
    overflow allows: counts and digests of the levels both stored are equal;
    if both found a formula the minimal costs are equal; a CAPACITY side
    rules out every formula up to its checked_level, so the other side's
    minimal cost, if any, lies above it.  Returns the names of the problems
    that differ by capacity; any other difference raises."""
    capacity = []
    for p, a, b in zip(ps, xs, ys):
        both = min(a.levels_done, b.levels_done)
        assert a.level_counts[: both + 1] == b.level_counts[: both + 1], p.name
        assert a.level_digests[: both + 1] == b.level_digests[: both + 1], p.name
        if not a.overflow_level and not b.overflow_level:
            assert (a.status, a.min_cost, a.levels_done, a.level_counts, a.level_digests) == \
                (b.status, b.min_cost, b.levels_done, b.level_counts, b.level_digests), p.name
            continue
        if a.status == 0 and b.status == 0:  # OK on both sides
            assert a.min_cost == b.min_cost, p.name
        for x, y in ((a, b), (b, a)):
            if x.status == 2:  # CAPACITY: nothing of cost <= checked_level separates
                assert y.status != 0 or y.min_cost > x.checked_level, p.name
        if (a.status, a.min_cost, a.levels_done, a.overflow_level, a.level_counts) != \
                (b.status, b.min_cost, b.levels_done, b.overflow_level, b.level_counts):
            capacity.append(p.name)
    return capacity


def batched_compare(synth, count: int):
    """The batched configuration (count problems, each to its own bound of
    planted cost + 3, plain solve): one by one (upload + solve each), then in
    one ltlf_solve_batch call; the results must agree."""
    import torch
    import workload

    ps = workload.batched(1, count)
    synth.solve(ps[0])  # warm-up
    torch.cuda.synchronize()
    solo, each = [], []
    t0 = time.perf_counter()
    for p in ps:
        a = time.perf_counter()
        solo.append(synth.solve(p))
        each.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    log(f"[bench] batched config: one by one {count} problems in {t_solo:.3f} s")
    t_batch = []
    for _ in range(2):
        torch.cuda.synchronize()
        a = time.perf_counter()
        bat = synth.solve_batch(ps)
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - a)
        log(f"[bench] batched config: ltlf_solve_batch {count} problems in {t_batch[-1]:.3f} s")
    capacity = compare_results(ps, solo, bat)
    each.sort()
    tb = min(t_batch)
    return {"problems": count, "one_by_one_problems_per_s": round(count / t_solo, 2),
            "batch_problems_per_s": round(count / tb, 2), "speedup": round(t_solo / tb, 3),
            "one_by_one_ms_p50": round(each[len(each) // 2], 3),
            "one_by_one_ms_p99": round(each[min(len(each) - 1, (len(each) * 99) // 100)], 3),
            "batch_wall_ms": round(tb * 1e3, 1), "batch_launches_per_level_loop": bat[0].gen_launches,
            "results_identical": not capacity, "differ_by_capacity": capacity,
            "config": "props U{2..5}, traces per class U{8..256}, lengths 4-64, planted cost U{6..12}, "
                      "bound planted+3, master seed 1"}


def served_compare(synth, count: int, outliers: float = 0.0):
    """Served stream: requests drawn from the batched configuration's shape
    mix (master seed 2) arrive as a Poisson process at 1.5 x the rate one at
    a time solving sustains; the request server (continuous batching) and a
    one-at-a-time FIFO loop face the same arrival times.  Time to formula =
    completion - arrival (host clock, upload included)."""
    import numpy as np
    import torch
    import workload

    import paper_2504_18943_amd as m

    ps = workload.served(2, count, outliers)
    synth.solve(ps[0])  # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    for p in ps:
        synth.solve(p)
        if "outlier" in p.name:
            log(f"[bench] served calibration: {p.name} done")
    torch.cuda.synchronize()
    solo_rate = count / (time.perf_counter() - a)
    rate = 1.5 * solo_rate
    rng = np.random.Generator(np.random.PCG64(7))
    arrive = np.cumsum(rng.exponential(1.0 / rate, size=count))

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, int(q * len(v)))]

    # one at a time, first come first served
    t0 = time.perf_counter()
    done_solo, res_solo = [], []
    for i, p in enumerate(ps):
        now = time.perf_counter() - t0
        if now < arrive[i]:
            time.sleep(arrive[i] - now)
        res_solo.append(synth.solve(p))
        done_solo.append(time.perf_counter() - t0)
        if "outlier" in p.name:
            log(f"[bench] served one at a time: {p.name} done")
    ttf_solo = [(d - arr) * 1e3 for d, arr in zip(done_solo, arrive)]
    span_solo = done_solo[-1]
    # the request server
    srv = m.Server(synth, max_resident=min(count, 512))
    t0 = time.perf_counter()
    nxt, tickets, done_srv, res_srv = 0, {}, [0.0] * count, [None] * count
    while len(tickets) or nxt < count:
        now = time.perf_counter() - t0
        while nxt < count and arrive[nxt] <= now:
            tickets[srv.submit(ps[nxt])] = nxt
            nxt += 1
        if not tickets:
            time.sleep(max(0.0, arrive[nxt] - now))
            continue
        srv.step()
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                i = tickets.pop(t)
                done_srv[i] = time.perf_counter() - t0
                res_srv[i] = r
                if "outlier" in ps[i].name:
                    log(f"[bench] served server: {ps[i].name} done")
    srv.close()
    ttf_srv = [(d - arr) * 1e3 for d, arr in zip(done_srv, arrive)]
    span_srv = max(done_srv)
    capacity = compare_results(ps, res_solo, res_srv)
    log(f"[bench] served: one at a time p50 {pct(ttf_solo, 0.5):.1f} ms p99 {pct(ttf_solo, 0.99):.1f} ms, "
        f"server p50 {pct(ttf_srv, 0.5):.1f} ms p99 {pct(ttf_srv, 0.99):.1f} ms")
    return {"requests": count, "arrival_rate_per_s": round(rate, 1),
            "one_at_a_time": {"ttf_ms_p50": round(pct(ttf_solo, 0.5), 2), "ttf_ms_p99": round(pct(ttf_solo, 0.99), 2),
                              "problems_per_s": round(count / span_solo, 2)},
            "server": {"ttf_ms_p50": round(pct(ttf_srv, 0.5), 2), "ttf_ms_p99": round(pct(ttf_srv, 0.99), 2),
                       "problems_per_s": round(count / span_srv, 2)},
            "results_identical": not capacity, "differ_by_capacity": capacity,
            "config": "Poisson arrivals at 1.5x the one-at-a-time rate; shapes of the batched configuration "
                      "(master seed 2), bound planted+3"
                      + (f"; {int(round(count * outliers))} outliers of the large configuration's size "
                         f"(5 props, 512+512 traces, lengths 16-64, same cost law)" if outliers else "")}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--bound", type=int, default=13)
    ap.add_argument("--workspace-gb", type=float, default=0.0)
    ap.add_argument("--cpu-bound", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttf", action="store_true")
    ap.add_argument("--served", type=int, default=128,
                    help="requests of the served stream (Poisson arrivals), server vs one at a "
                         "time (0 = skip)")
    ap.add_argument("--served-outliers", type=float, default=0.05,
                    help="fraction of served requests replaced by problems of the large "
                         "configuration's size")
    ap.add_argument("--batched", type=int, default=256,
                    help="problems of the batched configuration solved one by one and with "
                         "ltlf_solve_batch (0 = skip)")
    ap.add_argument("--large-bound", type=int, default=9,
                    help="enumerate the large configuration to this cost (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the batched and served legs with the built-in kernel choice")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.calibrate_copy_gib > 0:
        import torch
        n = int(args.calibrate_copy_gib * (1 << 30))
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {n} bytes")
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); independent problems "
              "would shard across GPUs without communication, and no multi-GPU path is implemented.",
              file=sys.stderr)
        return 2

    import torch

    import paper_2504_18943_amd as m
    import workload

    dev = 0
    free, total = torch.cuda.mem_get_info(dev)
    # the batched and served legs compare a whole-workspace solve with the
    # scheduler's large region (1/32 smaller): no problem of those
    # configurations should need a store between the two sizes
    ws = int(args.workspace_gb * (1 << 30)) if args.workspace_gb > 0 else \
        int(min(free * 0.8, 224 * (1 << 30)))
    log(f"[bench] workspace {ws / (1 << 30):.1f} GiB of {free / (1 << 30):.1f} GiB free")
    synth = m.Synthesizer(device=dev, workspace_bytes=ws)
    p = workload.medium(args.seed)
    synth.load(p)

    flags = m.FLAG_EXHAUST | m.FLAG_PROFILE
    for i in range(args.warmup):
        r = synth.run(args.bound, flags=flags)
        log(f"[bench] warmup {i}: status {r.status_name} levels {r.levels_done} "
            f"unique {r.unique_total} {r.enum_ms:.1f} ms")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = synth.run(args.bound, flags=flags)
        results.append(r)
        log(f"[bench] step {i}: {r.enum_ms:.1f} ms, unique {r.unique_total}, cand {r.candidates}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    last = results[-1]
    for r in results:
        assert r.level_counts == last.level_counts, "level counts changed between steps"
    unique = last.unique_total
    value = unique / (ms_per_step / 1e3)

    # roofline of the generation kernel: algorithmic bytes = (row bytes + 8)
    # per candidate (operands amortised; one probe; one verify read or row
    # write per candidate), over the summed event time of its launches
    gen_ms = sum(r.gen_ms for r in results) / len(results)
    launches = last.gen_launches
    bytes_per_step = last.candidates * (last.row_bytes + 8)
    achieved = bytes_per_step / (gen_ms / 1e3) / 1e9 if gen_ms > 0 else 0.0
    traffic, prof_file = profiled_traffic("ltlf::k_generate", f"--bound {args.bound} ")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic else None,
            "traffic_unit": "HBM bytes per launch (2 x FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": prof_file,
            "algorithmic_bytes_per_launch": round(bytes_per_step / max(launches, 1)),
            "kernel": "generation (k_generate*)", "launches_per_step": launches,
            "avg_launch_ms": round(gen_ms / max(launches, 1), 4),
            "bytes_per_candidate": last.row_bytes + 8}
    # hash-probe and atomic rates: every candidate that differs from its
    # operands probes at least one slot; atomics and L2 requests per launch
    # from the committed counter summary, over the live launch time
    counters, ctr_file = profiled_counters("ltlf::k_generate", f"--bound {args.bound} ")
    launch_s = gen_ms / max(launches, 1) / 1e3
    roof["rates"] = {
        "candidates_per_s": round(last.candidates / (gen_ms / 1e3)) if gen_ms > 0 else None,
        "atomics_per_s": round(counters["TCC_ATOMIC_sum_per_launch"] / launch_s) if counters else None,
        "atomics_to_memory_per_s": round(counters["TCC_EA0_ATOMIC_sum_per_launch"] / launch_s) if counters else None,
        "l2_requests_per_s": round(counters["TCC_REQ_sum_per_launch"] / launch_s) if counters else None,
        "l2_hit_rate": round(counters["TCC_HIT_sum_per_launch"] / (counters["TCC_HIT_sum_per_launch"]
                                                                   + counters["TCC_MISS_sum_per_launch"]), 4)
        if counters else None,
        "valu_busy_pct": counters.get("VALUBusy_pct_time_weighted") if counters else None,
        "valu_utilization_pct": counters.get("VALUUtilization_pct_time_weighted") if counters else None,
        "counters_source": ctr_file}

    ttf = None
    if not args.no_ttf:
        per_seed = {}
        for s in (1, 2, 3, 4):
            q = workload.medium(s)
            times = []
            for _ in range(3):
                torch.cuda.synchronize()
                a = time.perf_counter()
                rr = synth.solve(q)  # upload + plain solve + witness
                times.append((time.perf_counter() - a) * 1e3)
            per_seed[s] = {"ms": round(statistics.median(times), 3), "min_cost": rr.min_cost,
                           "formula": rr.formula}
            log(f"[bench] time-to-formula seed {s}: {per_seed[s]}")
        ttf = {"median_ms": round(statistics.median(v["ms"] for v in per_seed.values()), 3),
               "per_seed": per_seed, "includes": "host-to-device upload of the specification"}

    # measured kernel choice per row width; the batched and served legs (both
    # modes) run with it, the headline above with the built-in choice
    tuning = None
    if not args.no_autotune and (args.batched > 0 or args.served > 0):
        a = time.perf_counter()
        table = synth.autotune()
        tuning = {"seconds": round(time.perf_counter() - a, 2),
                  "classes": [{"chunks": e["chunks"], "kernel": e["kernel"], "ns_per_candidate": e["ns_per_candidate"]}
                              for e in table]}
        log(f"[bench] autotune {tuning}")

    batched = None
    if args.batched > 0:
        batched = batched_compare(synth, args.batched)
    served = None
    if args.served > 0:
        served = served_compare(synth, args.served, args.served_outliers)

    large = large_config(synth, args.large_bound) if args.large_bound > 0 else None

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.seed, args.cpu_bound)
    if cpu:
        log(f"[bench] cpu baseline {cpu['value']:.0f} unique/s")

    line = {
        "metric": "unique formula semantics enumerated/sec",
        "value": round(value, 1),
        "unit": "unique semantics/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"medium synthesis problem (3 props, 32+32 traces, lengths 8-32, "
                               f"planted cost 11, seed {args.seed}); every cost level 1..{args.bound} "
                               f"enumerated, deduplicated and checked",
                   "seed": args.seed, "cost_bound": args.bound, "row_bytes": last.row_bytes,
                   "unique_per_level": last.level_counts[1:last.levels_done + 1],
                   "candidates": last.candidates, "deferred": last.deferred,
                   "status": last.status_name, "min_cost": last.min_cost},
        "time_to_formula": ttf,
        "large": large,
        "autotune": tuning,
        "batched": batched,
        "served": served,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    synth.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
