"""Benchmark of the MBR-filter spatial join on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input
already resident in HBM: choose the grid (features + statistics rule or
learned picker), partition R, partition S (validate, two-level count /
scan / scatter) and join (classify tiles, per-tile sort + forward-scan sweep
with the reference-point test, pair output and compaction).  The tuned
schedules run both partitions and the join as one call (sj_join_rects: one
status readback); with the grid choice that is two host synchronisations
per step.  Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload skewed10m]

The tuned run uses the learned picker when its weights are present (else the
rule) with the batched / split schedule; --compare (default) also times two
baselines: the statistics-rule K with the same autotuned schedule family
(rule_tuned: isolates what the learned grid choice gains) and the
statistics-rule K with the plain one-workgroup-per-tile schedule.  Schedules
come from the autotuner cache file (--tune-cache) when it holds the class,
so that separate runs (this one and its profiling run) use the same kernels;
--save-tune writes the cache back after tuning.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "skewed10m": "skewed 10M x 10M: 200-Gaussian mixture + 20% background, log-normal extents "
                 "(median 5e-5, sigma 1.0), float32",
    "uniform1m": "uniform 1M x 1M, extents U[0,2e-4], float32",
    "aniso4m": "anisotropic 4M x 4M: 100-Gaussian mixture + 10% background, long thin rectangles "
               "(median 2e-4, aspect 25, horizontal left of x = 0.5, vertical right of it), float32",
    "distance10m": "epsilon-distance join of skewed 10M x 10M points (centres of the skewed 10M "
                   "mixture), eps 1e-4, float32",
    "batch256": "256 independent joins, n/side log-uniform [1e3, 2e6], per-join mixture "
                "(clusters log-uniform [1,500], background U[0,0.5]), extents U[0,2e-4], float32",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="skewed10m", choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=0, help="fixed grid size (0: choose every step)")
    ap.add_argument("--split-tau", type=int, default=0)
    ap.add_argument("--picker", default="auto", choices=["auto", "rule", "learned"])
    ap.add_argument("--plain", action="store_true", help="time only the plain rule baseline")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--two-pass", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1908_11740_amd", "tune_cache.txt"),
                    help="autotuner cache file read before tuning (a class it holds is not re-tuned)")
    ap.add_argument("--save-tune", action="store_true", help="write the autotuner cache file afterwards")
    ap.add_argument("--tune-reps", type=int, default=2,
                    help="timed runs per candidate schedule when a class is tuned (not in the cache)")
    ap.add_argument("--stripes", action="store_true",
                    help="one-dimensional partitioning: K vertical stripes swept along y")
    ap.add_argument("--sweep-x", action="store_true",
                    help="sweep every tile along x (no per-tile sweeping-axis model)")
    ap.add_argument("--gbda", action="store_true",
                    help="join dense tiles as the 9 GBDA class mini-joins (no duplicate test)")
    ap.add_argument("--sorted", action="store_true",
                    help="write the pairs in lexicographic (r, s) order (SJ_SORTED_OUTPUT)")
    ap.add_argument("--cold", action="store_true",
                    help="write a 512 MiB buffer before every timed step, so that the inputs "
                         "and partitions are not served from the 256 MB Infinity Cache")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--count", action="store_true", help="count-only join mode")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (a known-size kernel "
                         "for scaling HBM byte counters) and exit")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def inputs(name):
    from paper_1908_11740_amd import datagen
    if name == "skewed10m":
        return datagen.skewed_10m()
    if name == "aniso4m":
        return datagen.anisotropic_4m()
    return datagen.uniform_1m()


PARTITION_KERNELS = ("k_l1_count", "k_l1_scatter", "k_l2_count", "k_l2_scatter")


def kernel_bytes(name, w, sides=1):
    """Algorithmic HBM bytes of one launch.  A partition kernel launched for
    one side takes the mean of the two sides (sides=1); launched once for
    both (sj_join_rects batches them: sides=2), the sum.  Entries are 20 B
    (box + id word), pairs 8 B."""
    n = (w["nR"] + w["nS"]) / 2 * sides
    m1 = (w["m1R"] + w["m1S"]) / 2 * sides
    m = (w["mR"] + w["mS"]) / 2 * sides
    st = w["stats"]
    table = {
        "k_features": 16 * (w["nR"] + w["nS"]),
        "k_l1_count": 16 * n,
        "k_l1_scatter": 16 * n + 20 * m1,
        "k_l2_count": 16 * m1,
        "k_l2_scatter": 20 * m1 + 20 * m,
        "k_classify": 8 * w["C"] + 16 * (st["small_tiles"] + st["medium_tiles"]),
        "k_dense_sort": 40 * st["dense_entries"],
        "k_axis": 8 * (st["medium_entries"] + st["dense_entries"]),
        "k_compact": 16 * w["P"],
    }
    if st["single_pass"]:
        table["k_span_units_single"] = 20 * st["small_entries"] + 8 * st["pairs_small"]
        table["k_lds_medium_single"] = 20 * st["medium_entries"] + 8 * st["pairs_medium"]
        table["k_dense_sweep_single"] = 20 * st["dense_entries"] + 8 * st["pairs_dense"]
    return table.get(name)


def host_cpu():
    """CPU model and logical cores of the host running the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def dominant(kernels):
    """The kernel with the largest share of the step among those whose
    algorithmic bytes are known (scans and tiny kernels are left out)."""
    known = [k for k in kernels if kernels[k]["alg_bytes"]]
    pool = known or list(kernels)
    return max(pool, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["calls"])


def source_digest():
    """Hash of the HIP sources (the kernels a stored traffic figure belongs to)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1908_11740_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    none for this workload or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if data.get("source_digest") != source_digest():
        return None
    k = data["kernels"].get(kernel)
    return None if k is None else int(k["fetch_bytes"] + k["write_bytes"])


def bench_batch(args, pk, sj, torch):
    """Many joins in one recorded graph: a step is one replay of the whole
    batch -- every join's partitions and classification, then one set of
    join launches over the work units of all joins (grids chosen once by the
    picker or the rule when the batch is planned)."""
    import numpy as np
    from paper_1908_11740_amd import datagen
    n = 256
    log("generating", n, "joins")
    host = [datagen.batch_instance(j)[:2] for j in range(n)]
    dev = [(torch.from_numpy(R).cuda(), torch.from_numpy(S).cuda()) for R, S in host]
    use_learned = args.picker == "learned" or (args.picker == "auto" and pk.weights_available())
    if use_learned:
        pk.load()
    else:
        sj.picker_unload()
    counting = sj.Batch(dev)
    _, counts = counting.run()
    counting.free()
    b = sj.Batch(dev, capacities=[int(c) for c in counts])
    for _ in range(max(1, args.warmup)):
        st, npairs = b.run()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        st, npairs = b.run()
        times.append(time.perf_counter() - t0)
    ms = sum(times) * 1e3 / len(times)
    ks, taus = b.grids()
    nrects = int(sum(R.shape[0] + S.shape[0] for R, S in host))
    # per-kernel times: the same kernels launched one by one (the recorded
    # graph hides them from the library's event brackets)
    sj.prof_enable(True)
    reps = max(1, min(args.steps, 5))
    for _ in range(reps):
        b.run(eager=True)
    torch.cuda.synchronize()
    kern = sj.prof_collect()
    sj.prof_enable(False)
    st_ = b.stats()
    m1, m = b.entries()
    nR = np.array([R.shape[0] for R, _ in host], np.float64)
    nS = np.array([S.shape[0] for _, S in host], np.float64)
    C = np.asarray(ks, np.float64) ** 2
    P = int(npairs.sum())
    # whole-batch algorithmic bytes per kernel name, averaged over its launches
    tot = {
        "k_l1_count": 16 * (nR.sum() + nS.sum()),
        "k_l1_scatter": 16 * (nR.sum() + nS.sum()) + 20 * m1.sum(),
        "k_l2_count": 16 * m1.sum(),
        "k_l2_scatter": 20 * m1.sum() + 20 * m.sum(),
        "k_classify": 8 * C.sum() + 16 * (st_["small_tiles"] + st_["medium_tiles"]),
        "k_span_units_batch": 20 * st_["small_entries"] + 8 * st_["pairs_small"],
        "k_lds_medium_batch": 20 * st_["medium_entries"] + 8 * st_["pairs_medium"],
        "k_dense_sweep_batch": 20 * st_["dense_entries"] + 8 * st_["pairs_dense"],
    }
    kernels = {}
    for name, (t, calls) in kern.items():
        per_step_calls = calls / reps
        avg = t / max(calls, 1)
        bb = tot.get(name)
        b_launch = None if bb is None else bb / max(per_step_calls, 1)
        kernels[name] = {"avg_ms": round(avg, 5), "calls": calls,
                         "alg_bytes": None if b_launch is None else int(b_launch),
                         "gbs": None if b_launch is None else round(b_launch / (avg * 1e-3) / 1e9, 1)}
    dom = dominant(kernels)
    dk = kernels[dom]
    roofline = {"kernel": dom, "bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": None if dk["gbs"] is None else round(dk["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("batch256", dom) if args.picker == "auto" else None,
                "avg_ms": dk["avg_ms"], "alg_bytes_per_launch": dk["alg_bytes"],
                "timing": "kernel times from an eager run of the same kernels (the graph replay "
                          "hides them from the event brackets)"}
    b_step = 32 * (nR.sum() + nS.sum()) + 40 * m.sum() + 8 * P + 32 * C.sum()
    # the same joins one by one through the single-join entry points (same
    # grids): what the batch saves
    outs = [torch.empty((int(c) + 1, 2), dtype=torch.int32, device="cuda") for c in counts]
    parts = [[None, None] for _ in range(n)]

    def sequential():
        for j, (Rd, Sd) in enumerate(dev):
            parts[j][0] = sj.partition(Rd, int(ks[j]), split_tau=int(taus[j]), reuse=parts[j][0])
            parts[j][1] = sj.partition(Sd, int(ks[j]), split_tau=int(taus[j]), reuse=parts[j][1])
            sj.join_into(parts[j][0], parts[j][1], outs[j])

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        sequential()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / max(1, args.steps // 2)
    for pr in parts:
        pr[0].free()
        pr[1].free()
    verified = None
    cpu = None
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        log("oracle pbsm per join on host cores")
        t_cpu, ok = 0.0, True
        for j, (R, S) in enumerate(host):
            pairs, tp, tj = oracle.pbsm(R, S, int(ks[j]), threads=0, timings=True, sort=False)
            ok = ok and len(pairs) == int(npairs[j])
            t_cpu += tp + tj
        verified = ok
        if not args.no_cpu_baseline:
            cpu = {"value": round(nrects / t_cpu, 1), "unit": "rects/s", "cores": oracle.max_threads(),
                   "kind": "oracle", "host": host_cpu(),
                   "sample": f"all {n} joins at the batch's grids, partition + join (Sec. 3.4), "
                             f"{t_cpu:.3f} s"}
    rec = {
        "metric": "input rects/s", "value": round(nrects / (ms * 1e-3), 1), "unit": "rects/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["batch256"], "joins": n, "rects": nrects,
                   "grid_choice": ("learned" if use_learned else "rule") + ", K^2 <= (nR + nS) / 4",
                   "grid_k_min": int(ks.min()), "grid_k_max": int(ks.max()),
                   "schedule": "one recorded graph: each partitioning launch and the "
                               "classification run the workgroups of all joins, then one set of "
                               "join launches over the work units of all joins",
                   "mode": "pairs"},
        "pairs_per_s": round(P / (ms * 1e-3), 1), "n_pairs": P,
        "pairs_match_oracle_count": verified, "median_ms_per_step": round(statistics.median(times) * 1e3, 4),
        "step_alg_bytes": int(b_step),
        "step_hbm_frac": round(b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "sequential_ms_per_step": round(ms_seq, 4), "speedup_vs_sequential": round(ms_seq / ms, 3),
        "roofline": roofline, "kernels": kernels, "join_stats": st_, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    b.free()


def bench_distance(args, pk, sj, torch):
    """Epsilon-distance join (Sec. 1): a step is one sj_distance_join over the
    resident point sets -- squares, grid choice, partition of both sides, and
    the intersection join with the distance check in its sweep."""
    from paper_1908_11740_amd import datagen
    log("generating", args.workload)
    P, Q, eps = datagen.skewed_points_10m()
    Pd, Qd = torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()
    nP, nQ = len(P), len(Q)
    # the picker's training corpus holds no point sets (equal squares): the
    # statistics rule unless the learned picker is asked for
    use_learned = args.picker == "learned"
    if use_learned:
        pk.load()
    else:
        sj.picker_unload()
    state = {"out": torch.empty((1 << 20, 2), dtype=torch.int32, device="cuda"), "n": 0, "g": None}

    def step():
        flags = (sj.SJ_STRIPES if args.stripes else 0) | (sj.SJ_TWO_PASS if args.two_pass else 0)
        flags |= 0 if use_learned else sj.SJ_RULE_ONLY
        g = sj.make_grid(args.k, args.split_tau, flags=flags)
        out = None if args.count else state["out"]
        st, n = sj.distance_join_into(Pd, Qd, eps, out, g)
        if st == sj.SJ_ERR_CAPACITY:
            state["out"] = torch.empty((int(n * 1.1) + 1024, 2), dtype=torch.int32, device="cuda")
            st, n = sj.distance_join_into(Pd, Qd, eps, state["out"], g)
        state["n"], state["g"] = n, g

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    tuning = None
    if not args.no_tune:
        # autotuner on the join of the squares: cached for this grid and size class
        tg = sj.make_grid(state["g"].k, state["g"].split_tau, flags=state["g"].flags)
        tuning = sj.distance_tune(Pd, Qd, eps, tg, reps=args.tune_reps)
        log("autotuned", tuning)
        step()
        torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = sum(times) * 1e3 / len(times)
    sj.prof_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kern = sj.prof_collect()
    sj.prof_enable(False)
    info = sj.distance_last_info()
    st = sj.last_join_stats()
    K, tau, n = state["g"].k, state["g"].split_tau, state["n"]
    nc = info["candidates"]
    w = dict(nR=nP, nS=nQ, m1R=info["level1_entries_p"], m1S=info["level1_entries_q"],
             mR=info["entries_p"], mS=info["entries_q"], C=K * K, P=n, stats=st)
    kernels = {}
    for name, (tot, calls) in kern.items():
        avg = tot / max(calls, 1)
        if name == "k_point_squares":
            b = 24 * (nP + nQ) / 2           # two launches: 8 B in, 16 B out per point
        else:  # the join writes the result pairs (the distance test is in its sweep)
            b = kernel_bytes(name, w)
        kernels[name] = {"avg_ms": round(avg, 5), "calls": calls,
                         "alg_bytes": None if b is None else int(b),
                         "gbs": None if b is None else round(b / (avg * 1e-3) / 1e9, 1)}
    dom = dominant(kernels)
    dk = kernels[dom]
    profiled = not (args.k or args.split_tau or args.stripes or args.two_pass or args.count or
                    args.no_tune or args.picker != "auto")
    roofline = {"kernel": dom, "bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": None if dk["gbs"] is None else round(dk["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom) if profiled else None,
                "avg_ms": dk["avg_ms"], "alg_bytes_per_launch": dk["alg_bytes"]}
    verified = None
    cpu = None
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        log("oracle filter-and-refine on host cores, K", K)
        t0 = time.perf_counter()
        ref = oracle.distance_filter_refine(P, Q, eps, K)
        secs = time.perf_counter() - t0
        verified = len(ref) == n
        if not args.no_cpu_baseline:
            cpu = {"value": round((nP + nQ) / secs, 1), "unit": "points/s",
                   "cores": oracle.max_threads(), "kind": "oracle",
                   "sample": f"the full workload at K={K}: squares, PBSM, distance check "
                             f"(Sec. 1), {secs:.3f} s, {len(ref)} pairs"}
    rec = {
        "metric": "input points/s", "value": round((nP + nQ) / (ms * 1e-3), 1), "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_p": nP, "n_q": nQ, "eps": eps,
                   "grid_k": K, "split_tau": tau,
                   "grid_choice": "fixed" if args.k else ("learned" if use_learned else "rule"),
                   "partitioning": "1-D stripes" if args.stripes else "2-D grid",
                   "mode": "count" if args.count else "pairs", "autotuned": tuning},
        "pairs_per_s": round(n / (ms * 1e-3), 1), "n_pairs": int(n), "n_candidates": int(nc),
        "pairs_match_oracle_count": verified,
        "median_ms_per_step": round(statistics.median(times) * 1e3, 4),
        "roofline": roofline, "kernels": kernels, "join_stats": st, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: only one GPU is supported (--gpus {args.gpus} given); sharding the "
              "tile rows over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB x 5 (read {args.copy_calibration} MiB + write "
            f"{args.copy_calibration} MiB per launch)")
        return

    from paper_1908_11740_amd import picker as pk
    from paper_1908_11740_amd import sj

    torch.cuda.set_device(0)
    if not args.no_tune and os.path.exists(args.tune_cache):
        log("autotuner cache:", sj.tune_load(args.tune_cache), "entries from", args.tune_cache)
    if args.workload == "batch256":
        return bench_batch(args, pk, sj, torch)
    if args.workload == "distance10m":
        bench_distance(args, pk, sj, torch)
        if not args.no_tune and args.save_tune:
            sj.tune_save(args.tune_cache)
        return
    log("generating", args.workload)
    R, S = inputs(args.workload)
    Rd = torch.from_numpy(R).cuda()
    Sd = torch.from_numpy(S).cuda()
    nR, nS = len(R), len(S)
    use_learned = args.picker == "learned" or (args.picker == "auto" and pk.weights_available())
    if use_learned:
        pk.load()
    state = {"PR": None, "PS": None, "pairs": 0, "K": 0, "tau": 0, "info": None,
             "out": torch.empty((1 << 20, 2), dtype=torch.int32, device="cuda")}

    def step(mode):
        plain = mode == "plain"
        stripes = ((sj.SJ_STRIPES if args.stripes else 0) | (sj.SJ_SWEEP_X if args.sweep_x else 0) |
                   (sj.SJ_GBDA if args.gbda else 0) | (sj.SJ_SORTED_OUTPUT if args.sorted else 0))
        if args.k:
            K, tau = args.k, args.split_tau
        else:
            fl = sj.SJ_RULE_ONLY if (mode != "tuned" or not use_learned) else 0
            K, tau, state["info"] = sj.choose_grid(Rd, Sd, split_tau=args.split_tau,
                                                   flags=fl | stripes)
        flags = stripes | (sj.SJ_PLAIN if plain else (sj.SJ_TWO_PASS if args.two_pass else 0))
        state["K"], state["tau"] = K, tau
        if not plain:
            # both partitions and the join, one status readback
            parts = (state["PR"], state["PS"]) if state["PR"] is not None else None
            out = None if args.count else state["out"]
            st, n, parts = sj.join_rects(Rd, Sd, K, split_tau=tau, flags=flags, out=out,
                                         parts=parts)
            if st == sj.SJ_ERR_CAPACITY:
                state["out"] = torch.empty((int(n * 1.1) + 1024, 2), dtype=torch.int32,
                                           device="cuda")
                st, n, parts = sj.join_rects(Rd, Sd, K, split_tau=tau, flags=flags,
                                             out=state["out"], parts=parts)
            state["PR"], state["PS"] = parts
            state["pairs"] = n
            return
        state["PR"] = sj.partition(Rd, K, split_tau=tau, flags=flags, reuse=state["PR"])
        state["PS"] = sj.partition(Sd, K, split_tau=tau, flags=flags, reuse=state["PS"])
        if args.count:
            state["pairs"] = sj.join_count(state["PR"], state["PS"])
            return
        st, n = sj.join_into(state["PR"], state["PS"], state["out"])
        if st == sj.SJ_ERR_CAPACITY:
            state["out"] = torch.empty((int(n * 1.1) + 1024, 2), dtype=torch.int32, device="cuda")
            st, n = sj.join_into(state["PR"], state["PS"], state["out"])
        state["pairs"] = n

    def timed(mode):
        plain = mode == "plain"
        for _ in range(max(1, args.warmup)):
            step(mode)
        torch.cuda.synchronize()
        state["tuning"] = None
        if not plain and not args.no_tune:
            # autotuner: schedule for this workload class, cached by the library
            # (and read from the cache file when it holds the class)
            cached = sj.tune_lookup(state["PR"], state["PS"], count_only=args.count)
            if cached is not None:
                state["tuning"] = dict(cached, source="cache file")
            else:
                state["tuning"] = sj.tune(state["PR"], state["PS"],
                                          None if args.count else state["out"], reps=args.tune_reps)
            log("autotuned", mode, state["tuning"])
            step(mode)
            torch.cuda.synchronize()
        # unprofiled: the reported time
        times = []
        flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda") if args.cold else None
        for _ in range(args.steps):
            if flush is not None:
                flush.fill_(1.0)
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(mode)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        del flush
        ms = sum(times) * 1e3 / len(times)
        # the same steps again with per-kernel HIP events on the launch stream
        sj.prof_enable(True)
        for _ in range(args.steps):
            step(mode)
        torch.cuda.synchronize()
        kern = sj.prof_collect()
        sj.prof_enable(False)
        return ms, statistics.median(times) * 1e3, kern

    res = {}
    modes = ["plain"] if args.plain else (
        ["tuned"] + ([] if args.no_compare else (["rule_tuned"] if use_learned and not args.k else []) +
                     ["plain"]))
    for mode in modes:
        log("timing", mode)
        ms, med, kern = timed(mode)
        _, mR, _ = state["PR"].info()
        _, mS, _ = state["PS"].info()
        m1R, _ = state["PR"].stats()
        m1S, _ = state["PS"].stats()
        res[mode] = dict(ms=ms, median=med, kern=kern, K=state["K"], tau=state["tau"],
                         P=state["pairs"], mR=mR, mS=mS, m1R=m1R, m1S=m1S,
                         stats=sj.last_join_stats(), info=state["info"],
                         tuning=state["tuning"])
        log(f"{mode}: {ms:.3f} ms/step (median {med:.3f}), K={state['K']} tau={state['tau']}, "
            f"{state['pairs']} pairs")
    main_mode = modes[0]
    r = res[main_mode]
    K, P = r["K"], r["P"]
    C = K * K
    w = dict(nR=nR, nS=nS, m1R=r["m1R"], m1S=r["m1S"], mR=r["mR"], mS=r["mS"], C=C, P=P,
             stats=r["stats"])
    kernels = {}
    for name, (tot, calls) in r["kern"].items():
        avg = tot / max(calls, 1)
        # partition kernels: one launch per side, or one for both sides
        sides = 2 if name in PARTITION_KERNELS and calls <= args.steps else 1
        b = kernel_bytes(name, w, sides)
        kernels[name] = {"avg_ms": round(avg, 5), "calls": calls,
                         "alg_bytes": None if b is None else int(b),
                         "gbs": None if b is None else round(b / (avg * 1e-3) / 1e9, 1)}
    steps = args.steps
    dom = dominant(kernels)
    dk = kernels[dom]
    # the committed counter summary covers the default configuration only
    profiled = (main_mode == "tuned" and not (args.k or args.split_tau or args.stripes or
                                              args.sweep_x or args.gbda or args.two_pass or
                                              args.count or args.no_tune or args.sorted or
                                              args.cold) and
                args.picker == "auto")
    roofline = {"kernel": dom, "bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": None if dk["gbs"] is None else round(dk["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom) if profiled else None,
                "avg_ms": dk["avg_ms"], "alg_bytes_per_launch": dk["alg_bytes"]}
    b_step = 32 * (nR + nS) + 40 * (r["mR"] + r["mS"]) + 8 * P + 32 * C
    ms = r["ms"]
    verified = None
    cpu = None
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        log("oracle pbsm on host cores, K", K)
        pairs, tp, tj = oracle.pbsm(R, S, K, threads=0, timings=True, sort=False)
        verified = all(int(len(pairs)) == int(res[m]["P"]) for m in res)
        if not args.no_cpu_baseline:
            secs = tp + tj
            # one host thread on a bounded sample: the first million rectangles of each side
            n1 = min(nR, nS, 1_000_000)
            _, tp1, tj1 = oracle.pbsm(R[:n1], S[:n1], K, threads=1, timings=True, sort=False)
            cpu = {"value": round((nR + nS) / secs, 1), "unit": "rects/s",
                   "cores": oracle.max_threads(), "kind": "oracle",
                   "sample": f"the full workload at K={K}: partition + join (Sec. 3.4), "
                             f"{secs:.3f} s, {len(pairs)} pairs",
                   "host": host_cpu(),
                   "one_thread": {"value": round(2 * n1 / (tp1 + tj1), 1), "unit": "rects/s",
                                  "sample": f"first {n1} rectangles of R and of S at K={K}, "
                                            f"{tp1 + tj1:.3f} s"}}
    rec = {
        "metric": "input rects/s",
        "value": round((nR + nS) / (ms * 1e-3), 1),
        "unit": "rects/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_r": nR, "n_s": nS, "grid_k": K,
                   "split_tau": r["tau"],
                   "grid_choice": "fixed" if args.k else ("learned" if use_learned and main_mode == "tuned"
                                                          and not args.stripes else "rule"),
                   "partitioning": "1-D stripes" if args.stripes else "2-D grid",
                   "sweep_axis": "y" if args.stripes else ("x" if args.sweep_x else "per-tile model"),
                   "dense_tiles": "GBDA mini-joins" if args.gbda else "Eq. (1) test",
                   "pair_order": "sorted (r, s)" if args.sorted else "unspecified",
                   "cache": "flushed before every step" if args.cold else "warm",
                   "schedule": main_mode, "mode": "count" if args.count else "pairs",
                   "autotuned": r["tuning"]},
        "pairs_per_s": round(P / (ms * 1e-3), 1),
        "n_pairs": int(P),
        "pairs_match_oracle_count": verified,
        "median_ms_per_step": round(r["median"], 4),
        "step_alg_bytes": int(b_step),
        "step_hbm_frac": round(b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels": kernels,
        "join_stats": r["stats"],
        "cpu_baseline": cpu,
    }
    if "rule_tuned" in res and main_mode == "tuned":
        b = res["rule_tuned"]
        rec["rule_tuned_baseline"] = {"ms_per_step": round(b["ms"], 4), "grid_k": b["K"],
                                      "split_tau": b["tau"], "n_pairs": int(b["P"]),
                                      "autotuned": b["tuning"]}
        rec["speedup_vs_rule_tuned"] = round(b["ms"] / ms, 3)
    if not args.no_tune and args.save_tune:
        sj.tune_save(args.tune_cache)
        log("autotuner cache written to", args.tune_cache)
    if "plain" in res and main_mode == "tuned":
        b = res["plain"]
        rec["plain_rule_baseline"] = {"ms_per_step": round(b["ms"], 4), "grid_k": b["K"],
                                      "n_pairs": int(b["P"])}
        rec["speedup_vs_plain_rule"] = round(b["ms"] / ms, 3)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
