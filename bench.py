"""Benchmark of the MBR-filter spatial join on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input
already resident in HBM: partition R, partition S (validate, count, scan,
scatter) and join (classify tiles, per-tile sort + forward-scan sweep with
the reference-point test, pair output).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload skewed10m]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "skewed10m": "skewed 10M x 10M: 200-Gaussian mixture + 20% background, log-normal extents "
                 "(median 5e-5, sigma 1.0), float32",
    "uniform1m": "uniform 1M x 1M, extents U[0,2e-4], float32",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="skewed10m", choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=0, help="grid size (0: statistics rule)")
    ap.add_argument("--plain", action="store_true", help="one-workgroup-per-tile schedule")
    ap.add_argument("--split-tau", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--count", action="store_true", help="count-only join mode")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def inputs(name):
    from paper_1908_11740_amd import datagen
    if name == "skewed10m":
        return datagen.skewed_10m()
    return datagen.uniform_1m()


def rule_k(R, S):
    """Grid size of the statistics rule (tile extent ~ 10x the mean rectangle
    extent), evaluated on the host for this benchmark's fixed inputs."""
    import numpy as np
    e = np.concatenate([(R[:, 2] - R[:, 0]).astype(np.float64) + (R[:, 3] - R[:, 1]),
                        (S[:, 2] - S[:, 0]).astype(np.float64) + (S[:, 3] - S[:, 1])]).mean() / 2
    return int(min(16384, max(1, round(1.0 / (10.0 * e)))))


def kernel_bytes(name, nR, nS, mR, mS, C, P):
    """Algorithmic HBM bytes of one launch of a kernel (per side for the
    partition kernels: the mean over the two sides)."""
    n = (nR + nS) / 2
    m = (mR + mS) / 2
    if name == "k_count":
        return 16 * n + 4 * C
    if name == "k_scan":
        return 8 * C
    if name == "k_scatter":
        return 16 * n + 20 * m + 4 * C
    if name in ("k_lds_units", "k_plain_tiles"):
        return 20 * (mR + mS) + 8 * P + 8 * C
    if name == "k_classify":
        return 8 * C
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1908_11740_amd import sj

    torch.cuda.set_device(0)
    log("generating", args.workload)
    R, S = inputs(args.workload)
    K = args.k if args.k > 0 else rule_k(R, S)
    flags = sj.SJ_PLAIN if args.plain else 0
    Rd = torch.from_numpy(R).cuda()
    Sd = torch.from_numpy(S).cuda()
    nR, nS = len(R), len(S)
    state = {"PR": None, "PS": None, "out": torch.empty((1 << 20, 2), dtype=torch.int32,
                                                       device="cuda")}

    def step():
        state["PR"] = sj.partition(Rd, K, split_tau=args.split_tau, flags=flags, reuse=state["PR"])
        state["PS"] = sj.partition(Sd, K, split_tau=args.split_tau, flags=flags, reuse=state["PS"])
        if args.count:
            return sj.join_count(state["PR"], state["PS"])
        st, n = sj.join_into(state["PR"], state["PS"], state["out"])
        if st == sj.SJ_ERR_CAPACITY:
            state["out"] = torch.empty((int(n * 1.1) + 1024, 2), dtype=torch.int32, device="cuda")
            st, n = sj.join_into(state["PR"], state["PS"], state["out"])
        return n

    log("warmup", args.warmup, "K", K)
    n_pairs = 0
    for _ in range(max(1, args.warmup)):
        n_pairs = step()
    torch.cuda.synchronize()
    sj.prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        n_pairs = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = sj.prof_collect()
    sj.prof_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, {n_pairs} pairs")
    _, mR, _ = state["PR"].info()
    _, mS, _ = state["PS"].info()
    C = K * K

    kernels = {}
    for name, (tot, calls) in kern.items():
        avg = tot / max(calls, 1)
        b = kernel_bytes(name, nR, nS, mR, mS, C, n_pairs)
        kernels[name] = {"avg_ms": round(avg, 5), "calls": calls,
                         "alg_bytes": None if b is None else int(b),
                         "gbs": None if b is None else round(b / (avg * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["calls"])
    dk = kernels[dom]
    roofline = {"kernel": dom, "bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": None if dk["gbs"] is None else round(dk["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": None}
    b_step = 32 * (nR + nS) + 40 * (mR + mS) + 8 * n_pairs + 32 * C
    verified = None
    cpu = None
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        log("oracle pbsm on host cores")
        pairs, tp, tj = oracle.pbsm(R, S, K, threads=0, timings=True, sort=False)
        verified = int(len(pairs)) == int(n_pairs)
        if not args.no_cpu_baseline:
            secs = tp + tj
            cpu = {"value": round((nR + nS) / secs, 1), "unit": "input rects/s",
                   "cores": oracle.max_threads(), "kind": "oracle",
                   "sample": f"full workload at K={K}: partition + join (Sec. 3.4), "
                             f"{secs:.3f} s, {len(pairs)} pairs"}
    rec = {
        "metric": "input rects/s",
        "value": round((nR + nS) / (ms * 1e-3), 1),
        "unit": "rects/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_r": nR, "n_s": nS, "grid_k": K,
                   "schedule": "plain" if args.plain else "tuned",
                   "mode": "count" if args.count else "pairs"},
        "pairs_per_s": round(n_pairs / (ms * 1e-3), 1),
        "n_pairs": int(n_pairs),
        "pairs_match_oracle_count": verified,
        "step_alg_bytes": int(b_step),
        "step_hbm_frac": round(b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
