"""Benchmark: unique formula semantics enumerated per second on one MI355X.

Headline workload (the large synthesis problem, seed 1): 5 atomic
propositions, 512 positive and 512 negative traces of lengths 16..64 (about
41,000 bits per characteristic matrix, 5,248-byte rows), per-proposition bit
rates drawn from U(0.3, 0.7), labels from a planted formula of cost 13.  Its
plain solve stops at its minimal cost (7), so one benchmark step is the whole
hot path run exhaustively with the semantic cache sized to HBM: encode, seed,
and every cost level 1..--bound (10: the deepest level whose rows fit the
workspace, ~3.5e7 CMs, ~185 GB) generated, deduplicated and checked.  The
specification is uploaded once before timing (inputs resident in HBM); each
step is one ltlf_run.

value = sum over levels of |U_c| / step time.  Also reported: the roofline of
the dominant kernel (the wave generation kernel) from HIP events around its
launches, with HBM traffic and counter rates from the committed rocprofv3
summary; the configuration's own solve (bound 16) as time to formula; the
medium problem enumerated to cost 13 (lane kernel); the CPU oracle on a
bounded sample of the headline problem (one core) and on the batched
configuration (a process pool over the host's cores); the batched
configuration (256 problems of mixed shape) solved one by one and in one
ltlf_solve_batch call; and a served stream (Poisson arrivals at a stable
rate) through the request server and one at a time, with identical results
(counts and per-level digests of the sets) required.
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


def large_workspace_bytes(free: int) -> int:
    """Workspace of the headline run: 85% of free HBM, at most 240 GiB (the
    large problem's level 10 needs ~185 GB of rows and derivations)."""
    return int(min(free * 0.85, 240 * (1 << 30)))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(bound: int):
    """The oracle (plain single-threaded C) on the headline problem, every
    level to `bound` (the levels it reaches in seconds)."""
    import oracle
    import workload

    p = workload.large(1)
    t0 = time.perf_counter()
    r = oracle.solve(p, cost_bound=bound, exhaust=True)
    wall = time.perf_counter() - t0
    uniq = sum(r.level_counts[1: r.levels_done + 1])
    return {"value": uniq / r.seconds, "unit": "unique semantics/s", "cores": 1, "kind": "oracle",
            "sample": f"large seed 1 (the headline problem), every level to cost {bound} ({uniq} unique CMs, "
                      f"{r.candidates} candidates), single-threaded C, {r.seconds:.2f} s enumeration, "
                      f"{wall:.2f} s wall",
            "cpu_model": cpu_model()}


def _oracle_one(args):
    """Pool worker: the oracle's plain solve of one problem (status, cost)."""
    import oracle
    p = args
    r = oracle.solve(p)
    return r.status, r.min_cost, r.levels_done


def cpu_pool_baseline(count: int, window_s: float):
    """The oracle over a process pool of the host's cores (at most 16) on the
    batched configuration's first `count` problems (plain solves at their own
    bounds), for at most window_s seconds: problems finished per second of
    wall time.  Problems still running when the window closes are reported
    as unfinished."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor, wait, FIRST_COMPLETED

    import workload

    ps = workload.batched(1, count)
    workers = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("spawn")
    ex = ProcessPoolExecutor(max_workers=workers, mp_context=ctx)
    try:
        ex.submit(_oracle_one, workload.tiny(1)).result()  # workers up before timing
        t0 = time.perf_counter()
        futs = {ex.submit(_oracle_one, p): i for i, p in enumerate(ps)}
        done, last = 0, t0
        pending = set(futs)
        while pending:
            left = window_s - (time.perf_counter() - t0)
            if left <= 0:
                break
            fin, pending = wait(pending, timeout=left, return_when=FIRST_COMPLETED)
            for f in fin:
                f.result()
                done += 1
                last = time.perf_counter()
        wall = last - t0
    finally:
        for proc in list(getattr(ex, "_processes", {}).values()):
            proc.kill()
        ex.shutdown(wait=False, cancel_futures=True)
    return {"value": round(done / wall, 2) if wall > 0 else 0.0, "unit": "problems/s", "cores": workers,
            "kind": "oracle", "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": f"batched configuration (master seed 1), first {count} problems, plain solves to their "
                      f"own bounds, {workers} worker processes, {window_s:.0f} s window: {done} finished in "
                      f"{wall:.1f} s, {count - done} unfinished"}


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
    one ltlf_solve_batch call; the results must agree, sets included (both
    modes compute per-level digests)."""
    import torch
    import workload

    import paper_2504_18943_amd as m

    D = m.FLAG_DIGEST
    ps = workload.batched(1, count)
    synth.solve(ps[0], flags=D)  # warm-up
    torch.cuda.synchronize()
    solo, each = [], []
    t0 = time.perf_counter()
    for p in ps:
        a = time.perf_counter()
        solo.append(synth.solve(p, flags=D))
        each.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    log(f"[bench] batched config: one by one {count} problems in {t_solo:.3f} s")
    t_batch = []
    for _ in range(2):
        torch.cuda.synchronize()
        a = time.perf_counter()
        bat = synth.solve_batch(ps, flags=D)
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
            "compared": "status, minimal cost, levels, per-level counts and digests (sets)",
            "config": "props U{2..5}, traces per class U{8..256}, lengths 4-64, planted cost U{6..12}, "
                      "bound planted+3, master seed 1"}


def serve_stream(synth, ps, arrive, D):
    """The request server over a stream: requests are submitted when their
    arrival time has passed, the server is stepped while any is open.
    Returns (completion times, results), clock from the start."""
    import paper_2504_18943_amd as m

    count = len(ps)
    srv = m.Server(synth, max_resident=min(count, 512))
    t0 = time.perf_counter()
    nxt, tickets, done, res = 0, {}, [0.0] * count, [None] * count
    while len(tickets) or nxt < count:
        now = time.perf_counter() - t0
        while nxt < count and arrive[nxt] <= now:
            tickets[srv.submit(ps[nxt], flags=D)] = nxt
            nxt += 1
        if not tickets:
            time.sleep(max(0.0, arrive[nxt] - now))
            continue
        srv.step()
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                i = tickets.pop(t)
                done[i] = time.perf_counter() - t0
                res[i] = r
    srv.close()
    return done, res


def served_compare(synth, count: int, outliers: float, factor: float):
    """Served stream: requests drawn from the batched configuration's shape
    mix (master seed 2, with a fraction replaced by problems of the large
    configuration's size) arrive as a Poisson process at `factor` x the
    server's measured capacity (all requests submitted at once, problems
    finished per second): a stable queue.  The request server (continuous
    batching) and a one-at-a-time FIFO loop face the same arrival times.
    Time to formula = completion - arrival (host clock, upload included)."""
    import numpy as np
    import torch
    import workload

    import paper_2504_18943_amd as m

    D = m.FLAG_DIGEST
    ps = workload.served(2, count, outliers)
    synth.solve(ps[0], flags=D)  # warm-up
    torch.cuda.synchronize()
    done_cap, _ = serve_stream(synth, ps, np.zeros(count), D)
    capacity = count / max(done_cap)
    rate = factor * capacity
    log(f"[bench] served: server capacity {capacity:.1f} problems/s, arrivals at {rate:.1f}/s")
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
        res_solo.append(synth.solve(p, flags=D))
        done_solo.append(time.perf_counter() - t0)
    ttf_solo = [(d - arr) * 1e3 for d, arr in zip(done_solo, arrive)]
    span_solo = done_solo[-1]
    log("[bench] served: one at a time done")
    done_srv, res_srv = serve_stream(synth, ps, arrive, D)
    ttf_srv = [(d - arr) * 1e3 for d, arr in zip(done_srv, arrive)]
    span_srv = max(done_srv)
    capacity_diff = compare_results(ps, res_solo, res_srv)
    log(f"[bench] served: one at a time p50 {pct(ttf_solo, 0.5):.1f} ms p99 {pct(ttf_solo, 0.99):.1f} ms, "
        f"server p50 {pct(ttf_srv, 0.5):.1f} ms p99 {pct(ttf_srv, 0.99):.1f} ms")
    return {"requests": count, "arrival_rate_per_s": round(rate, 2),
            "server_capacity_per_s": round(capacity, 2), "rate_factor": factor,
            "one_at_a_time": {"ttf_ms_p50": round(pct(ttf_solo, 0.5), 2), "ttf_ms_p99": round(pct(ttf_solo, 0.99), 2),
                              "problems_per_s": round(count / span_solo, 2)},
            "server": {"ttf_ms_p50": round(pct(ttf_srv, 0.5), 2), "ttf_ms_p99": round(pct(ttf_srv, 0.99), 2),
                       "problems_per_s": round(count / span_srv, 2)},
            "results_identical": not capacity_diff, "differ_by_capacity": capacity_diff,
            "compared": "status, minimal cost, levels, per-level counts and digests (sets)",
            "config": f"Poisson arrivals at {factor} x the server's capacity on this stream; shapes of the batched "
                      "configuration (master seed 2), bound planted+3"
                      + (f"; {int(round(count * outliers))} outliers of the large configuration's size "
                         f"(5 props, 512+512 traces, lengths 16-64, same cost law)" if outliers else "")}


def medium_leg(synth, bound: int, steps: int):
    """The medium problem (3 props, 32+32 traces, lengths 8..32, seed 1)
    with every level enumerated to `bound` (160-byte rows: the lane kernel)."""
    import torch
    import workload

    import paper_2504_18943_amd as m

    synth.load(workload.medium(1))
    flags = m.FLAG_EXHAUST | m.FLAG_PROFILE
    synth.run(bound, flags=flags)  # warm-up
    torch.cuda.synchronize()
    a = time.perf_counter()
    rs = [synth.run(bound, flags=flags) for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - a) * 1e3 / steps
    r = rs[-1]
    gen_ms = sum(x.gen_ms for x in rs) / steps
    gbs = r.candidates * (r.row_bytes + 8) / (gen_ms / 1e3) / 1e9 if gen_ms > 0 else 0.0
    log(f"[bench] medium to cost {bound}: {ms:.1f} ms per step, {gbs:.0f} GB/s")
    return {"workload": "medium synthesis problem (3 props, 32+32 traces, lengths 8-32, planted cost 11, seed 1)",
            "cost_bound": bound, "row_bytes": r.row_bytes, "ms_per_step": round(ms, 3),
            "unique_per_s": round(r.unique_total / (ms / 1e3), 1), "unique_per_level": r.level_counts[1:bound + 1],
            "candidates": r.candidates, "gen_ms": round(gen_ms, 3), "gen_launches": r.gen_launches,
            "kernel": "k_generate_lds (one candidate per lane)", "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def paper_example(synth, reps: int = 3):
    """The paper's 7+7 example (7 positive and 7 negative traces of length 6
    over {a, b}) solved to its minimum under the paper's grammar {p, not,
    and, X, F, U} with unit costs and bound 16: time to formula (upload +
    enumeration + witness), median of reps.  The paper reports about one
    second for its size-16 formula on an unnamed GPU (context only)."""
    import torch

    from tests import paper_fixtures as pf

    p = pf.spec_problem("seven_seven", 16)
    unit_paper = (1, 1, 1, 0, 1, 0, 1)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = synth.solve(p, cost_bound=16, op_cost=unit_paper)
        times.append((time.perf_counter() - a) * 1e3)
    out = {"ms": round(statistics.median(times), 2), "status": r.status_name, "min_cost": r.min_cost,
           "formula": r.formula, "candidates": r.candidates, "unique": r.unique_total,
           "unique_per_level": r.level_counts[1:r.levels_done + 1],
           "grammar": "p, not, and, X, F, U (unit costs), bound 16",
           "paper_context": "the paper's tool: 681,601,918 formulae, about 1 s, GPU model not stated"}
    log(f"[bench] paper 7+7 example: {out}")
    return out


def time_to_formula(synth, seeds, make, reps: int = 3):
    """Plain solves (upload + enumeration to the minimal cost + witness) at
    the configuration's own bound; median over reps per seed."""
    import torch

    per_seed = {}
    for sd in seeds:
        q = make(sd)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            rr = synth.solve(q)
            times.append((time.perf_counter() - a) * 1e3)
        per_seed[sd] = {"ms": round(statistics.median(times), 3), "status": rr.status_name,
                        "min_cost": rr.min_cost, "formula": rr.formula, "cost_bound": q.cost_bound}
        log(f"[bench] time-to-formula {q.name}: {per_seed[sd]}")
    return {"median_ms": round(statistics.median(v["ms"] for v in per_seed.values()), 3),
            "per_seed": per_seed, "includes": "host-to-device upload of the specification"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bound", type=int, default=10,
                    help="headline: enumerate the large problem's levels 1..bound (10 = the deepest that fits)")
    ap.add_argument("--workspace-gb", type=float, default=0.0)
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline steps only (profiling runs)")
    ap.add_argument("--only-medium", action="store_true",
                    help="time the medium problem's steps only (profiling runs of the lane kernel); "
                         "prints that leg's figures, not the headline line")
    ap.add_argument("--only-batched", action="store_true",
                    help="solve the batched configuration with ltlf_solve_batch only (a warm-up call, "
                         "then one timed call; profiling runs); prints that call's figures")
    ap.add_argument("--cpu-bound", type=int, default=6,
                    help="oracle baseline on the headline problem to this cost (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pool", type=int, default=64,
                    help="oracle pool baseline on this many batched-configuration problems (0 = skip)")
    ap.add_argument("--cpu-pool-window", type=float, default=30.0)
    ap.add_argument("--no-ttf", action="store_true")
    ap.add_argument("--medium-bound", type=int, default=13,
                    help="enumerate the medium problem to this cost (0 = skip)")
    ap.add_argument("--served", type=int, default=512,
                    help="requests of the served stream (Poisson arrivals), server vs one at a "
                         "time (0 = skip)")
    ap.add_argument("--served-outliers", type=float, default=0.05,
                    help="fraction of served requests replaced by problems of the large "
                         "configuration's size")
    ap.add_argument("--served-rate", type=float, default=0.7,
                    help="arrival rate as a fraction of the server's measured capacity")
    ap.add_argument("--batched", type=int, default=256,
                    help="problems of the batched configuration solved one by one and with "
                         "ltlf_solve_batch (0 = skip)")
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
    if args.only_medium:
        ws = int(args.workspace_gb * (1 << 30)) if args.workspace_gb > 0 else int(min(free * 0.6, 120 << 30))
        synth = m.Synthesizer(device=dev, workspace_bytes=ws)
        print(json.dumps({"medium": medium_leg(synth, args.medium_bound, args.steps)}), flush=True)
        synth.close()
        return 0
    ws = int(args.workspace_gb * (1 << 30)) if args.workspace_gb > 0 else large_workspace_bytes(free)
    log(f"[bench] workspace {ws / (1 << 30):.1f} GiB of {free / (1 << 30):.1f} GiB free")
    if args.only_batched:
        synth = m.Synthesizer(device=dev, workspace_bytes=ws)
        if not args.no_autotune:
            synth.autotune()
        ps = workload.batched(1, args.batched)
        synth.solve_batch(ps, flags=m.FLAG_DIGEST)  # warm-up
        torch.cuda.synchronize()
        a = time.perf_counter()
        rs = synth.solve_batch(ps, flags=m.FLAG_DIGEST)
        torch.cuda.synchronize()
        wall = time.perf_counter() - a
        print(json.dumps({"batched_only": {"problems": len(ps), "wall_ms": round(wall * 1e3, 1),
                                           "problems_per_s": round(len(ps) / wall, 2),
                                           "ok": sum(r.status == m.ltlf.OK for r in rs)}}), flush=True)
        synth.close()
        return 0
    synth = m.Synthesizer(device=dev, workspace_bytes=ws)
    p = workload.large(1)
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
    assert last.levels_done == args.bound and last.overflow_level == 0, \
        f"the workspace does not hold level {args.bound} (levels_done {last.levels_done})"
    unique = last.unique_total
    value = unique / (ms_per_step / 1e3)

    # roofline of the generation kernel: algorithmic bytes = (row bytes + 8)
    # per candidate (operands amortised over the pair tile; one probe; one
    # verification read or row write per candidate), over the summed event
    # time of its launches on the run's stream
    gen_ms = sum(r.gen_ms for r in results) / len(results)
    ver_ms = sum(r.verify_ms for r in results) / len(results)
    launches = last.gen_launches
    bytes_per_step = last.candidates * (last.row_bytes + 8)
    achieved = bytes_per_step / (gen_ms / 1e3) / 1e9 if gen_ms > 0 else 0.0
    tag = f"--bound {args.bound} "
    traffic, prof_file = profiled_traffic("ltlf::k_generate_wave", tag)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic) if traffic else None,
            "traffic_unit": "HBM bytes per launch (2 x FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": prof_file,
            "algorithmic_bytes_per_launch": round(bytes_per_step / max(launches, 1)),
            "kernel": "k_generate_wave (one wavefront per pair or operand, rows streamed 64 chunks per step)",
            "launches_per_step": launches, "avg_launch_ms": round(gen_ms / max(launches, 1), 4),
            "gen_ms_per_step": round(gen_ms, 3), "verify_ms_per_step": round(ver_ms, 3),
            "bytes_per_candidate": last.row_bytes + 8}
    # hash-probe and atomic rates: atomics and L2 requests per launch from the
    # committed counter summary, over the live launch time
    counters, ctr_file = profiled_counters("ltlf::k_generate_wave", tag)
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

    extras = {}
    if not args.only_headline:
        if not args.no_ttf:
            extras["time_to_formula"] = time_to_formula(synth, (1, 2, 3), workload.large)
        if args.medium_bound > 0:
            extras["medium"] = medium_leg(synth, args.medium_bound, 3)
        extras["paper_example"] = paper_example(synth)
        if not args.no_autotune and (args.batched > 0 or args.served > 0):
            a = time.perf_counter()
            table = synth.autotune()
            extras["autotune"] = {"seconds": round(time.perf_counter() - a, 2),
                                  "classes": [{"chunks": e["chunks"], "kernel": e["kernel"],
                                               "ns_per_candidate": e["ns_per_candidate"],
                                               "wave_tile": e["wave_tile"],
                                               "ns_wave_tile": e["ns_wave_tile"]} for e in table]}
            log(f"[bench] autotune {extras['autotune']}")
        if args.batched > 0:
            extras["batched"] = batched_compare(synth, args.batched)
        if args.served > 0:
            extras["served"] = served_compare(synth, args.served, args.served_outliers, args.served_rate)
    synth.close()

    cpu = None
    if not args.only_headline and not args.no_cpu_baseline and args.cpu_bound > 0:
        cpu = cpu_baseline(args.cpu_bound)
        log(f"[bench] cpu baseline {cpu['value']:.0f} unique/s")
        if args.cpu_pool > 0:
            cpu["pool"] = cpu_pool_baseline(args.cpu_pool, args.cpu_pool_window)
            log(f"[bench] cpu pool {cpu['pool']}")

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
        "config": {"workload": f"large synthesis problem (5 props, 512+512 traces, lengths 16-64, planted cost 13, "
                               f"seed 1); every cost level 1..{args.bound} enumerated, deduplicated and checked, "
                               f"semantic cache sized to HBM",
                   "seed": 1, "cost_bound": args.bound, "row_bytes": last.row_bytes,
                   "workspace_gib": round(ws / (1 << 30), 1),
                   "unique_per_level": last.level_counts[1:last.levels_done + 1],
                   "candidates": last.candidates,
                   "candidates_range": [min(r.candidates for r in results), max(r.candidates for r in results)],
                   "deferred": last.deferred,
                   "status": last.status_name, "min_cost": last.min_cost},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
