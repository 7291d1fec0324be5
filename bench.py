"""Benchmark: SpGEMM GFLOP/s (2 * flops / s) and HBM roofline fraction on one
MI355X.

Default workload: R-MAT scale 20 (n = 1,048,576), edge factor 16,
(a, b, c) = (.57, .19, .19), symmetrized, deduplicated, float32 (0, 1];
C = A A with an HBM budget set so the batch planner picks 4 column batches.
A step is one whole product: symbolic pass, counts to the host, batch
planner, then per batch the numeric pass (and merge when layered); each
batch is handed to a consumer that discards it.  Inputs are resident in HBM
before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--scale", type=int, default=20, help="R-MAT scale (20 is the named workload)")
    p.add_argument("--batches", type=int, default=4)
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    return p.parse_args()


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2010_08526_amd as S
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    A = synth.rmat(args.scale, 16, synth.WORKLOADS["rmat20"].seed, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    print(f"# generated R-MAT scale {args.scale}: n={A.ncols} nnz={A.nnz} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    eng = S.Engine(A, A, 1, budget_bytes=1 << 62)
    plan = eng.plan()
    flops = plan.total_flops
    nnz_c = int(plan.nnz_host.sum())
    r = 8
    total_out = int((r * plan.nnz_host[0] + 8).sum())
    # budget: inputs + library reserve + a share of the output that yields the target batch count
    target = args.batches
    lo, hi = total_out // (target + 1) + 1, total_out // max(1, target - 1) + 1
    avail = None
    while lo <= hi:
        mid = (lo + hi) // 2
        try:
            b, _ = S.plan_batches(plan.nnz_host.reshape(-1), A.ncols, 1, 4, 0, mid, 0)
        except S.SpgemmError:
            lo = mid + 1
            continue
        nb = len(b) - 1
        if nb > target:
            lo = mid + 1
        else:
            avail = mid
            hi = mid - 1
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + avail
    print(f"# flops={flops:.4e} nnz(C)={nnz_c:.4e} cf={flops / nnz_c:.3f} out={total_out / 1e9:.1f} GB "
          f"budget={eng.budget_bytes / 1e9:.1f} GB", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    times = {"symbolic": [], "numeric": []}

    def step(record):
        e0 = ev(); e0.record(stream)
        pl = eng.plan()
        e1 = ev(); e1.record(stream)
        num = []
        for i in range(pl.nbatches):
            a = ev(); a.record(stream)
            eng.run_batch(pl, i)
            b = ev(); b.record(stream)
            num.append((a, b))
        if record:
            torch.cuda.synchronize()
            times["symbolic"].append(e0.elapsed_time(e1))
            times["numeric"].append(sum(a.elapsed_time(b) for a, b in num))
        return pl

    for _ in range(args.warmup):
        pl = step(False)
    torch.cuda.synchronize()
    eng.check()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        pl = step(True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    eng.check()
    ms = 1e3 * t_total / args.steps
    gflops = 2.0 * flops / (t_total / args.steps) / 1e9

    # Compulsory bytes of the numeric phase (per step, all batches): A is read
    # once per batch, B once, C written once, plus column pointers.
    nb = pl.nbatches
    num_bytes = nb * r * A.nnz + r * A.nnz + r * nnz_c + 8 * (A.ncols + nb)
    t_num = float(np.mean(times["numeric"])) / 1e3
    achieved = num_bytes / t_num / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, args.cpu_seconds)

    out = {
        "metric": "SpGEMM GFLOP/s (2*flops/s)",
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 values, f64 accumulation, int32 rows, int64 column pointers",
        "data": "synthetic, seeded R-MAT",
        "config": {"workload": f"rmat{args.scale}: C=A*A, R-MAT scale {args.scale} ef16 (.57,.19,.19) symmetrized "
                               f"fp32, {nb} column batches from an HBM budget",
                   "n": A.ncols, "nnz_A": A.nnz, "flops": flops, "nnz_C": nnz_c, "batches": nb,
                   "budget_bytes": eng.budget_bytes},
        "phases_ms": {"symbolic": round(float(np.mean(times["symbolic"])), 3),
                      "numeric_all_batches": round(t_num * 1e3, 3)},
        "roofline": {"bound": "hbm", "kernel": "numeric phase (all batches)", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(A, seconds: float):
    """The oracle (plain C, float64 dense accumulator, OpenMP over columns) on
    a seeded random sample of output columns of the same product."""
    import numpy as np

    import oracle

    Ah = oracle.as_mat(A)
    n = Ah.ncols
    rng = np.random.default_rng(12345)
    perm = rng.permutation(n)

    def sample(cnt):
        cols = np.sort(perm[:cnt])
        cp = np.zeros(cnt + 1, np.int64)
        lens = Ah.colptr[cols + 1] - Ah.colptr[cols]
        np.cumsum(lens, out=cp[1:])
        idx = np.concatenate([np.arange(Ah.colptr[c], Ah.colptr[c + 1]) for c in cols]) if cnt else np.zeros(0, int)
        return oracle.Mat(Ah.nrows, cnt, cp, Ah.rowidx[idx], Ah.values[idx])

    threads = oracle.max_threads()
    cnt = 64
    while True:
        Bs = sample(cnt)
        t = time.perf_counter()
        P = oracle.spgemm(Ah, Bs)
        dt = time.perf_counter() - t
        if dt > seconds / 4 or cnt >= n:
            break
        cnt = min(n, int(cnt * max(2.0, min(16.0, seconds / 2 / max(dt, 1e-3)))))
    fl = int(oracle.flops(Ah, Bs).sum())
    return {"value": round(2.0 * fl / dt / 1e9, 4), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{cnt} random output columns of the same product ({fl:.3e} flops, {dt:.1f} s)"}


if __name__ == "__main__":
    main()
