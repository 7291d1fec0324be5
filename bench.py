"""Benchmark: SpGEMM GFLOP/s (2 * flops / s) with the HBM-roofline fraction of
the dominant kernel, on one MI355X.

Headline workload: R-MAT scale 20 (n = 1,048,576), edge factor 16,
(a, b, c) = (.57, .19, .19), symmetrized, deduplicated, float32 (0, 1];
C = A A with an HBM budget set so that the batch planner picks 4 column
batches.  A step is one whole product: symbolic pass, counts to the host,
batch planner, then per batch the numeric pass; each batch is handed to a
consumer that discards it.  Inputs are resident in HBM before timing.

Also reported on the same GPU (same accuracy bar as the tests):
  fwd_bwd : Erdos-Renyi A, B (n = 262,144, 16 per column, N(0,1)): forward
            alone vs forward + backward (gradients of a loss on P(C)).
  batched : 4096 Erdos-Renyi pairs (n_i log-uniform in [256, 65536], 4-32
            per column) as one HIP-graph replay vs a loop of 4096 plain
            calls (column ranges of the same packed product); forward +
            fused backward as one graph.
  layered : protein-like n = 2,000,000, 16 inner-dimension layers merged
            sort-free under a 64 GB budget: symbolic, numeric partials and
            merge phases.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpGEMM GFLOP/s (2*flops/s) + % HBM roofline; fwd+bwd & batched vs plain"


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--scale", type=int, default=20, help="R-MAT scale (20 is the named workload)")
    p.add_argument("--batches", type=int, default=4)
    p.add_argument("--er-n", type=int, default=262_144)
    p.add_argument("--batch-count", type=int, default=4096)
    p.add_argument("--protein-n", type=int, default=2_000_000)
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the fwd_bwd, batched, layered, bsweep, prune, aat and sorted_output sections")
    p.add_argument("--extras", default="fwd_bwd,batched,layered,bsweep,prune,aat,sorted_output",
                   help="comma-separated extra sections to run")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of known size (to scale HBM byte counters) and exit")
    return p.parse_args()


def _timed(fn, reps, torch):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


# ----------------------------------------------------------------- headline
def headline(args, torch, np, S, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    A = synth.rmat(args.scale, 16, synth.WORKLOADS["rmat20"].seed, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"R-MAT scale {args.scale}: n={A.ncols} nnz={A.nnz} generated in {time.time() - t0:.1f}s")
    eng = S.Engine(A, A, 1, budget_bytes=1 << 62)
    plan = eng.plan()
    flops = plan.total_flops
    nnz_c = int(plan.nnz_host.sum())
    r = 8  # int32 row + float32 value
    total_out = int((r * plan.nnz_host[0] + 8).sum())
    # smallest output share that still gives the target batch count
    lo, hi, avail = total_out // (args.batches + 1) + 1, total_out // max(1, args.batches - 1) + 1, None
    while lo <= hi:
        mid = (lo + hi) // 2
        try:
            b, _ = S.plan_batches(plan.nnz_host.reshape(-1), A.ncols, 1, 4, 0, mid, 0)
        except S.SpgemmError:
            lo = mid + 1
            continue
        if len(b) - 1 > args.batches:
            lo = mid + 1
        else:
            avail, hi = mid, mid - 1
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + avail
    log(f"flops={flops:.4e} nnz(C)={nnz_c:.4e} cf={flops / nnz_c:.3f} C={total_out / 1e9:.1f} GB "
        f"budget={eng.budget_bytes / 1e9:.1f} GB")

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    phase = {"symbolic_plan": [], "numeric": []}

    def step(record):
        e0 = ev(); e0.record(stream)
        pl = eng.plan()
        e1 = ev(); e1.record(stream)
        spans = []
        for i in range(pl.nbatches):
            a = ev(); a.record(stream)
            eng.run_batch(pl, i)  # consumer: the batch is discarded
            b = ev(); b.record(stream)
            spans.append((a, b))
        if record:
            torch.cuda.synchronize()
            phase["symbolic_plan"].append(e0.elapsed_time(e1))
            phase["numeric"].append(sum(a.elapsed_time(b) for a, b in spans))
        return pl

    for _ in range(args.warmup):
        pl = step(False)
    torch.cuda.synchronize()
    eng.check()
    S.profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        pl = step(True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = S.profile_report()
    S.profile_enable(False)
    eng.check()
    nb = pl.nbatches
    ms = 1e3 * t_total / args.steps
    gflops = 2.0 * flops / (t_total / args.steps) / 1e9
    log(f"headline: {ms:.1f} ms/step, {gflops:.1f} GFLOP/s; kernels: " +
        ", ".join(f"{k}={v[0] / args.steps:.1f}ms" for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])))

    # Dominant kernel and its compulsory bytes per launch.
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    dom_name, (dom_ms, dom_calls) = dom[0], dom[1]
    bcp = A.colptr.cpu().numpy()
    bdeg = np.diff(bcp)
    u = plan.nnz_host[0]
    # heavy columns the item kernel takes: more than 5120 rows out, at most 1024
    # entries in B(:,j) (wider ones go to the dense-LDS wide kernel)
    heavy = (u > 5120) & (bdeg <= 1024)
    # per batch, those columns' B entries and outputs, plus one read of A
    per_batch = []
    fcol = eng.flops.cpu().numpy()
    gather = 0  # A entries fetched per multiplication by the item kernel (gather model)
    for i in range(nb):
        c0, c1 = pl.bounds[i], pl.bounds[i + 1]
        h = heavy[c0:c1]
        per_batch.append(r * int(bdeg[c0:c1][h].sum()) + r * int(u[c0:c1][h].sum()) + 8 * int(h.sum()) + r * A.nnz)
        gather += r * int(fcol[c0:c1][h].sum())
    num_bytes = nb * r * A.nnz + r * A.nnz + r * nnz_c + 8 * (A.ncols + nb)  # whole numeric phase
    launches = max(1.0, dom_calls / args.steps)
    if dom_name == "heavy_items":
        # the heavy columns of every batch, spread evenly over the item launches
        alg_bytes_per_launch = float(sum(per_batch)) / launches
        unit = ("item-kernel columns (more than 5120 rows out, at most 1024 entries in B(:,j)): "
                "r*(nnz(B) + nnz(C)) of those columns + 8 per column + r*nnz(A) per batch, "
                "summed over batches and divided by the item launches per step")
    else:
        alg_bytes_per_launch = num_bytes / launches
        unit = "share of the numeric phase's compulsory bytes"
    avg_launch_s = dom_ms / dom_calls / 1e3
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9
    gather_gbs = (alg_bytes_per_launch + gather / launches) / avg_launch_s / 1e9 if dom_name == "heavy_items" else None
    copy_gbs = measured_copy_gbs(torch)
    t_num = float(np.mean(phase["numeric"])) / 1e3
    res = {
        "metric": METRIC,
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "value_storage": "f32 values, int32 rows, int64 column pointers",
        "data": "synthetic, seeded R-MAT (no dataset)",
        "config": {"workload": f"rmat{args.scale}: C=A*A, R-MAT scale {args.scale} ef16 (.57,.19,.19) symmetrized, "
                               f"fp32 values, {nb} column batches from an HBM budget",
                   "n": A.ncols, "nnz_A": A.nnz, "flops": flops, "nnz_C": nnz_c, "batches": nb,
                   "budget_bytes": eng.budget_bytes},
        "phases_ms": {"symbolic_and_plan": round(float(np.mean(phase["symbolic_plan"])), 3),
                      "numeric_all_batches": round(t_num * 1e3, 3),
                      "numeric_phase_GBps_compulsory": round(num_bytes / t_num / 1e9, 2)},
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items()},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": measured_traffic(dom_name, f"rmat{args.scale}"),
                     "bytes_per_launch": int(alg_bytes_per_launch), "bytes_unit": unit,
                     "avg_launch_ms": round(avg_launch_s * 1e3, 3), "launches_per_step": dom_calls / args.steps,
                     "gather_model_GBps": None if gather_gbs is None else round(gather_gbs, 2),
                     "gather_model_note": "compulsory bytes plus r bytes of A per multiplication; caches can serve "
                                          "these re-reads, so this model may exceed the peak",
                     "measured_copy_GBps": round(copy_gbs, 1),
                     "measured_copy_note": "device-to-device copy of 2 GiB (read + write bytes over time)"},
    }
    return res, A


# -------------------------------------------------------------- fwd vs bwd
def fwd_bwd(args, torch, np, S, synth):
    dev = torch.device("cuda:0")
    A, B = synth.make_workload("er262k", device=dev, n=args.er_n)
    flops = args.er_n * 16 * 16
    eng = S.Engine(A, B, 1)
    pl = eng.plan()
    C = eng.run_batch(pl, 0)
    col = torch.repeat_interleave(torch.arange(C.ncols, device=dev), C.colptr[1:] - C.colptr[:-1])
    # targets are taken at the first forward's storage slots (one wavefront per
    # column keeps the slot order of these columns fixed from run to run)
    T = synth.target_values(C.rowidx, col, C.ncols, synth.WORKLOADS["er262k"].seed, torch.float32)
    bw = S.Backward(A, B, C)  # pattern transposes made once per structure

    def fwd():
        p = eng.plan()
        eng.run_batch(p, 0)

    def fwdbwd():
        p = eng.plan()
        Cb = eng.run_batch(p, 0)
        dC = Cb.values - T  # loss 0.5*||C - T||^2 on P(C); C's storage order is fixed by the forward
        bw.refresh_values(B)
        bw(dC)

    # the differentiated form as autograd runs it: SpGEMMFn's forward (a new
    # engine: symbolic pass, plan, numeric) and its backward, which forms the
    # transposes of A's, B's and C's patterns on every call
    a_vals = A.values.clone().requires_grad_(True)
    b_vals = B.values.clone().requires_grad_(True)
    Ap = S.CSC(A.nrows, A.ncols, A.colptr, A.rowidx, None)
    Bp = S.CSC(B.nrows, B.ncols, B.colptr, B.rowidx, None)

    def fwdbwd_autograd():
        c_vals, _, _ = S.SpGEMMFn.apply(a_vals, b_vals, Ap, Bp)
        loss = 0.5 * ((c_vals - T) ** 2).sum()
        a_vals.grad = None
        b_vals.grad = None
        loss.backward()

    import paper_2010_08526_amd.batched as Bt
    be = Bt.BatchedEngine(A, B, backward=True)
    be.forward()
    Cf = be.C
    colf = torch.repeat_interleave(torch.arange(Cf.ncols, device=dev), Cf.colptr[1:] - Cf.colptr[:-1])
    Tf = synth.target_values(Cf.rowidx, colf, Cf.ncols, synth.WORKLOADS["er262k"].seed, torch.float32)

    def fwd_fused():
        be.forward()
        be.backward((be.values[:be.nnz_c] - Tf).contiguous())

    fwd(); fwdbwd(); fwd_fused(); fwdbwd_autograd()
    reps = max(3, args.steps)
    t_f = _timed(fwd, reps, torch)
    t_fb = _timed(fwdbwd, reps, torch)
    t_ff = _timed(fwd_fused, reps, torch)
    t_fa = _timed(fwdbwd_autograd, reps, torch)
    bw.check()
    be.check()
    out = {"workload": f"er{args.er_n}: A, B independent Erdos-Renyi n={args.er_n}, 16 per column, fp32 N(0,1); "
                       "loss 0.5*||C-T||^2 on P(C)",
           "flops_forward": flops,
           "forward_ms": round(t_f * 1e3, 3), "forward_GFLOPs": round(2 * flops / t_f / 1e9, 2),
           "fwd_bwd_ms": round(t_fb * 1e3, 3), "fwd_bwd_GFLOPs": round(6 * flops / t_fb / 1e9, 2),
           "fwd_bwd_fused_ms": round(t_ff * 1e3, 3), "fwd_bwd_fused_GFLOPs": round(6 * flops / t_ff / 1e9, 2),
           "fwd_bwd_autograd_ms": round(t_fa * 1e3, 3), "fwd_bwd_autograd_GFLOPs": round(6 * flops / t_fa / 1e9, 2),
           "fwd_bwd_over_fwd_time": round(t_fb / t_f, 3),
           "fwd_bwd_autograd_over_fwd_time": round(t_fa / t_f, 3),
           "note": "fwd_bwd = forward + transpose-based backward (dA via B^T, dC^T) with the pattern transposes of "
                   "A, B and C made once per structure (outside the step); fwd_bwd_autograd = SpGEMMFn forward + "
                   "loss + backward through torch.autograd, every transpose (A, B, C patterns) and permutation "
                   "formed inside the step; fused = graph-capturable forward + one-pass backward (float64 atomics "
                   "for dA, no transposes); GFLOP/s counts 3x forward flops"}
    log(f"fwd_bwd: fwd {t_f * 1e3:.2f} ms, fwd+bwd {t_fb * 1e3:.2f} ms, autograd {t_fa * 1e3:.2f} ms, "
        f"fused {t_ff * 1e3:.2f} ms")
    return out


# ------------------------------------------------------- layered + merge
def layered(args, torch, np, S, synth):
    """protein2m: C = A A with the inner dimension split into 16 layers whose
    partial products are merged sort-free, under a 64 GB HBM budget."""
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS["protein2m"]
    t0 = time.time()
    A = synth.protein_like(args.protein_n, w.seed, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"protein-like n={A.ncols} nnz={A.nnz} generated in {time.time() - t0:.1f}s")
    L = 16
    eng = S.Engine(A, A, L, budget_bytes=64 * 10**9)
    stream = torch.cuda.current_stream()

    def step(marks):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pl = eng.plan()
        e1.record(stream)
        marks.append(("symbolic_and_plan", e0, e1))
        for i in range(pl.nbatches):
            eng.run_batch(pl, i, marks=marks)
        return pl

    step([])
    torch.cuda.synchronize()
    eng.check()
    marks = []
    S.profile_enable(True)
    t = time.perf_counter()
    pl = step(marks)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t
    prof = S.profile_report()
    S.profile_enable(False)
    eng.check()
    ph = {}
    for name, a, b in marks:
        ph[name] = ph.get(name, 0.0) + a.elapsed_time(b)
    flops = pl.total_flops
    r = 8
    nnz_d = int(pl.nnz_host[:L].sum())
    nnz_c = int(pl.nnz_host[L].sum())
    merge_bytes = r * nnz_d + r * nnz_c + 8 * (L + 1) * A.ncols
    num_bytes = pl.nbatches * r * A.nnz + r * A.nnz + r * nnz_d + 8 * L * A.ncols
    out = {"workload": f"protein{args.protein_n}: Chung-Lu power-law (2.1, mean 50, cap 5000), symmetric, "
                       "column-stochastic fp32; C=A*A with 16 inner-dimension layers merged sort-free, 64 GB budget",
           "n": A.ncols, "nnz_A": A.nnz, "flops": flops, "nnz_partials": nnz_d, "nnz_C": nnz_c,
           "layers": L, "batches": pl.nbatches, "budget_bytes": 64 * 10**9,
           "ms": round(t_total * 1e3, 3), "GFLOPs": round(2 * flops / t_total / 1e9, 2),
           "phases_ms": {k: round(v, 3) for k, v in ph.items()},
           "kernels_ms": {k: round(v[0], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])},
           "numeric_GBps_compulsory": round(num_bytes / (ph["numeric"] / 1e3) / 1e9, 2),
           "merge_GBps_compulsory": round(merge_bytes / (ph["merge"] / 1e3) / 1e9, 2),
           "roofline_merge": {"bound": "hbm", "phase": "merge (all batches)",
                              "achieved": round(merge_bytes / (ph["merge"] / 1e3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s",
                              "frac": round(merge_bytes / (ph["merge"] / 1e3) / 1e9 / HBM_PEAK_GBS, 5),
                              "bytes": merge_bytes,
                              "bytes_unit": "r*(sum of the partials' entries) read + r*nnz(C) written + 8 per column "
                                            "per partial and output (compulsory)"}}
    log(f"layered: {pl.nbatches} batches, {t_total * 1e3:.1f} ms, phases " +
        ", ".join(f"{k}={v:.1f}ms" for k, v in ph.items()) + "; kernels " +
        ", ".join(f"{k}={v[0]:.1f}ms" for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])[:12]))
    return out


# ------------------------------------------------------- batched vs plain
def batched(args, torch, np, S, synth):
    import paper_2010_08526_amd.batched as Bt
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS["batch4096"]
    spec = synth.batch_spec(args.batch_count, w.seed)
    t0 = time.time()
    A, B, off = synth.batch_packed(spec, w.seed, torch.float32, dev)
    torch.cuda.synchronize()
    flops = int((spec.n * spec.dA * spec.dB).sum())
    log(f"batch: {args.batch_count} instances, sum n={int(spec.n.sum())}, nnz(A)={A.nnz}, flops={flops:.4e}, "
        f"generated in {time.time() - t0:.1f}s")
    eng = Bt.BatchedEngine(A, B, backward=True)
    tune = Bt.autotune(eng, reps=1, use_cache=False)
    reps = max(3, args.steps)
    # forward and backward as one graph; dC = C (the loss 0.5*||C||^2 on P(C),
    # so that no target array is needed next to the 120 GB of C)
    g_fb = eng.capture(lambda: (eng.forward(), eng.backward(eng.values[:eng.nnz_c])))
    t_graph_fb = _timed(g_fb.replay, reps, torch)
    eng.check()
    eng.capture(eng.forward)
    t_graph = _timed(eng.replay, reps, torch)
    eng.check()
    nnz_c = eng.nnz_c
    # loop of plain calls: one column range (= one instance) per call
    offs = off.cpu().tolist()
    ws_sym = S.alloc_workspace(S.workspace_size(S.OP_SYMBOLIC, A, B, 0, B.ncols, 1))
    ws_num = S.alloc_workspace(S.workspace_size(S.OP_NUMERIC, A, B, 0, B.ncols, 1))
    ws_scan = S.alloc_workspace(S.workspace_size(S.OP_COLPTR, None, None, 0, B.ncols + 1))
    cnt = torch.empty(B.ncols, dtype=torch.int64, device=dev)
    cp = torch.empty(B.ncols + 1, dtype=torch.int64, device=dev)
    big = int((eng.colptr[off[1:]] - eng.colptr[off[:-1]]).max())
    ri = torch.empty(big, dtype=torch.int32, device=dev)
    vv = torch.empty(big, dtype=torch.float32, device=dev)

    def plain_loop():
        for i in range(args.batch_count):
            c0, c1 = offs[i], offs[i + 1]
            S.symbolic(A, B, c0, c1, 1, None, cnt[c0:c1], ws_sym)
            S.colptr(cnt[c0:c1], cp[c0:c1 + 1], ws_scan)
            S.numeric(A, B, c0, c1, 0, 1, None, cp[c0:c1 + 1], ri, vv, ws_num)

    plain_loop()
    t_plain = _timed(plain_loop, 1, torch)
    S.check_ws(ws_num, "plain loop")
    out = {"workload": f"batch{args.batch_count}: independent Erdos-Renyi pairs, n_i log-uniform [256, 65536], "
                       "4-32 per column, fp32 (0,1]; one packed block-diagonal product",
           "flops": flops, "nnz_C": nnz_c,
           "batched_graph_ms": round(t_graph * 1e3, 3), "batched_GFLOPs": round(2 * flops / t_graph / 1e9, 2),
           "plain_loop_ms": round(t_plain * 1e3, 3), "plain_loop_GFLOPs": round(2 * flops / t_plain / 1e9, 2),
           "speedup_batched_over_plain": round(t_plain / t_graph, 2),
           "batched_fwd_bwd_graph_ms": round(t_graph_fb * 1e3, 3),
           "batched_fwd_bwd_GFLOPs": round(6 * flops / t_graph_fb / 1e9, 2),
           "fwd_bwd_over_fwd_time": round(t_graph_fb / t_graph, 3),
           "fwd_bwd_note": "graph of forward + fused backward with dC = C; GFLOP/s counts 3x forward flops",
           "autotuned_caps": tune["caps"], "autotuned_num_bpc": tune["num_bpc"],
           "autotuned_sym_bpc": tune["sym_bpc"], "autotune_default_ms": round(tune["default_ms"], 3),
           "autotune_best_ms": round(tune["ms"], 3)}
    # compulsory bytes of one replay of the forward: the symbolic and the
    # numeric pass each read the stored inputs once (r bytes per entry of A
    # and B), the numeric pass writes C (r per entry) and its column pointers
    r = 8
    fwd_bytes = 2 * r * (A.nnz + B.nnz) + r * nnz_c + 8 * (B.ncols + 1)
    out["roofline_forward"] = {"bound": "hbm", "phase": "batched forward (one graph replay)",
                               "achieved": round(fwd_bytes / t_graph / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(fwd_bytes / t_graph / 1e9 / HBM_PEAK_GBS, 5), "bytes": fwd_bytes,
                               "bytes_unit": "symbolic and numeric passes each reading A and B once (r per entry), "
                                             "C written once (r per entry) and its column pointers (compulsory)"}
    log(f"batched: graph {t_graph * 1e3:.1f} ms vs plain loop {t_plain * 1e3:.1f} ms; fwd+bwd graph "
        f"{t_graph_fb * 1e3:.1f} ms")
    return out


def bsweep(args, torch, np, S, synth):
    """The headline product at several batch counts b (a one-GPU analog of
    the paper's runtime-versus-batches study): for each b the smallest HBM
    budget that gives b batches, then one warm-up and one timed product."""
    dev = torch.device("cuda:0")
    A = synth.rmat(args.scale, 16, synth.WORKLOADS["rmat20"].seed, dtype=torch.float32, device=dev)
    eng = S.Engine(A, A, 1, budget_bytes=1 << 62)
    plan = eng.plan()
    flops = plan.total_flops
    r = 8
    total_out = int((r * plan.nnz_host[0] + 8).sum())
    rows = []
    # fewest batches last: the engine's output buffers only grow
    for b in (64, 16, 8, 4, 2, 1):
        lo, hi, avail = total_out // (b + 1) + 1, total_out // max(1, b - 1) + 1 if b > 1 else total_out, None
        while lo <= hi:
            mid = (lo + hi) // 2
            try:
                bb, _ = S.plan_batches(plan.nnz_host.reshape(-1), A.ncols, 1, 4, 0, mid, 0)
            except S.SpgemmError:
                lo = mid + 1
                continue
            if len(bb) - 1 > b:
                lo = mid + 1
            else:
                avail, hi = mid, mid - 1
        if avail is None:
            rows.append({"b_target": b, "skipped": "no budget gives this many batches"})
            continue
        eng.release_buffers()  # the next plan's buffers replace them, not join them
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info()
        if avail > 0.8 * free:
            rows.append({"b_target": b, "skipped": f"output share {avail / 1e9:.1f} GB exceeds free HBM"})
            continue
        eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + avail
        times = []
        for rep in range(3):  # warm-up, timed, then one with per-kernel events
            torch.cuda.synchronize()
            if rep == 2:
                S.profile_enable(True)
            t0 = time.perf_counter()
            pl = eng.plan()
            for i in range(pl.nbatches):
                eng.run_batch(pl, i)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        prof = S.profile_report()
        S.profile_enable(False)
        eng.check()
        t = times[1]
        top = sorted(prof.items(), key=lambda kv: -kv[1][0])[:8]
        rows.append({"b": pl.nbatches, "budget_bytes": eng.budget_bytes, "ms": round(t * 1e3, 2),
                     "GFLOPs": round(2 * flops / t / 1e9, 2),
                     "kernels_ms": {k: round(v[0], 2) for k, v in top},
                     "launches": int(sum(v[1] for v in prof.values()))})
        log(f"bsweep: b={pl.nbatches} {t * 1e3:.1f} ms ({2 * flops / t / 1e9:.1f} GFLOP/s); " +
            ", ".join(f"{k}={v[0]:.1f}" for k, v in top[:5]))
    del eng
    return {"workload": "rmat20 headline product at several batch counts (one warm-up, one timed product, then one "
                        "with per-kernel HIP events for kernels_ms)",
            "flops": flops, "runs": rows}


def cpu_baseline(A, seconds: float):
    """The oracle (plain C, float64 dense accumulator, OpenMP over columns) on
    a seeded random sample of output columns of the headline product."""
    import numpy as np

    import oracle

    Ah = oracle.as_mat(A)
    n = Ah.ncols
    perm = np.random.default_rng(12345).permutation(n)

    def sample(cnt):
        cols = np.sort(perm[:cnt])
        lens = Ah.colptr[cols + 1] - Ah.colptr[cols]
        cp = np.zeros(cnt + 1, np.int64)
        np.cumsum(lens, out=cp[1:])
        idx = np.concatenate([np.arange(Ah.colptr[c], Ah.colptr[c + 1]) for c in cols])
        return oracle.Mat(Ah.nrows, cnt, cp, Ah.rowidx[idx], Ah.values[idx])

    threads = oracle.max_threads()
    cnt = 64
    while True:
        Bs = sample(cnt)
        t = time.perf_counter()
        oracle.spgemm(Ah, Bs)
        dt = time.perf_counter() - t
        if dt > seconds / 4 or cnt >= n:
            break
        cnt = min(n, int(cnt * max(2.0, min(16.0, seconds / 2 / max(dt, 1e-3)))))
    fl = int(oracle.flops(Ah, Bs).sum())
    return {"value": round(2.0 * fl / dt / 1e9, 4), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{cnt} seeded random output columns of the headline product ({fl:.3e} flops, {dt:.1f} s, "
                      f"float64, structure + values)"}


# ------------------------------------------------------------ HBM traffic
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 1 << 31


def copy_calibration(torch):
    """A plain device-to-device copy of COPY_BYTES, five times: the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    x = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    x.fill_(1)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 5}), flush=True)


def measured_copy_gbs(torch, reps=5):
    """Read + write bytes per second of a plain 2 GiB device copy."""
    x = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    x.fill_(1)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    del x, y
    return 2.0 * COPY_BYTES * reps / t / 1e9


def source_digest():
    """Digest of the sources of the product kernels (kernels.hip, the
    translation unit of the item kernel, and every device header); measured
    traffic is tied to it.  The other translation units (backward, prune,
    sort) build none of the product kernels."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2010_08526_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f == "kernels.hip" or f.endswith(".hpp"):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter runs, or None when there are none for the current sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("workload") != workload or t.get("source_digest") != source_digest():
        return None
    return int(t["hbm_bytes_per_launch"])


def aat(args, torch, np, S, synth):
    """The paper's second workload shape, A*A^T (products of the Rice-kmers
    matrix with its transpose): A with m = 1,000,000 rows, k = 50,000,000
    columns and two entries per column at distinct uniform rows (k >> m, cf
    about 2, light columns only).  The transpose runs on the GPU; one
    warm-up, then one timed transpose and one timed product."""
    dev = torch.device("cuda:0")
    m, k = 1_000_000, 50_000_000
    A = synth.erdos_renyi(m, k, 2, 201008526 + 7, torch.float32, device=dev)
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        At, _ = S.transpose(A, perm=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        eng = S.Engine(A, At, 1, None)
        C, pl = eng.run()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
        nnz_c, flops = C.nnz, pl.total_flops
        del C, eng, At
        torch.cuda.empty_cache()
    tt, tp = times[-1]
    log(f"aat: m={m} k={k} nnz(A)={A.nnz} flops={flops:.4e} nnz(C)={nnz_c:.4e} cf={flops / nnz_c:.2f}, "
        f"transpose {tt * 1e3:.1f} ms, product {tp * 1e3:.1f} ms ({2 * flops / tp / 1e9:.1f} GFLOP/s, {pl.nbatches} batch)")
    del A
    return {"workload": f"A*A^T, A {m} x {k}, 2 entries per column at distinct uniform rows, float32",
            "flops": flops, "nnz_c": nnz_c, "cf": round(flops / nnz_c, 3), "transpose_ms": round(tt * 1e3, 2),
            "product_ms": round(tp * 1e3, 2), "GFLOPs": round(2 * flops / tp / 1e9, 2), "batches": pl.nbatches}


def prune(args, torch, np, S, synth):
    """The consumer the paper puts after each batch (an application prunes
    every batch of C before the next; Markov clustering keeps the largest
    entries of each column): the headline product at its default budget,
    every batch pruned to its 100 largest entries per column.  Kernel times
    come from the library's per-launch HIP events; bytes are the compulsory
    ones (rows and values read once, column pointers, per-column selection
    state written and read once, kept entries written)."""
    dev = torch.device("cuda:0")
    A = synth.rmat(args.scale, 16, synth.WORKLOADS["rmat20"].seed, dtype=torch.float32, device=dev)
    eng = S.Engine(A, A, 1, budget_bytes=1 << 62)
    plan = eng.plan()
    total_out = int((8 * plan.nnz_host[0] + 8).sum())
    eng.budget_bytes = eng.input_bytes + eng.reserve_bytes + total_out // args.batches + int(plan.nnz_host[0].max()) * 8 + 8
    k = 100
    stats = {"entries": 0, "kept": 0, "cols": 0}
    ws = {}

    def consume(c0, c1, Cb):
        if "ws" not in ws or ws["ws"].numel() < S.workspace_size(S.OP_PRUNE, Cb):
            ws["ws"] = S.alloc_workspace(S.workspace_size(S.OP_PRUNE, Cb), dev)
        G = S.prune_topk(Cb, 0.0, k, ws=ws["ws"])
        stats["entries"] += Cb.nnz
        stats["kept"] += G.nnz
        stats["cols"] += Cb.ncols

    eng.run(consume=consume)  # warm-up
    stats = {"entries": 0, "kept": 0, "cols": 0}
    S.profile_enable(True)
    pl = eng.run(consume=consume)
    prof = S.profile_report()
    S.profile_enable(False)
    ms = sum(prof.get(n, (0.0, 0))[0] for n in ("prune_select", "prune_fill"))
    nbytes = 8 * stats["entries"] + 2 * 8 * (stats["cols"] + pl.nbatches) + 2 * 20 * stats["cols"] + 8 * stats["kept"]
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
    log(f"prune: {pl.nbatches} batches, {stats['entries']:.4e} entries -> {stats['kept']:.4e} kept (k={k}), "
        f"select {prof.get('prune_select', (0, 0))[0]:.1f} ms + fill {prof.get('prune_fill', (0, 0))[0]:.1f} ms, "
        f"{gbs:.0f} GB/s compulsory")
    del eng
    return {"workload": f"rmat20 headline product, each of its batches pruned to the {k} largest entries per column",
            "batches": pl.nbatches, "entries": stats["entries"], "kept": stats["kept"], "k": k,
            "select_ms": round(prof.get("prune_select", (0.0, 0))[0], 3),
            "fill_ms": round(prof.get("prune_fill", (0.0, 0))[0], 3),
            "compulsory_bytes": nbytes, "achieved_GBps": None if gbs is None else round(gbs, 1),
            "frac_of_hbm_peak": None if gbs is None else round(gbs / 8000.0, 4)}


def sorted_output(args, torch, np, S, synth):
    """Row-sorted output columns (the paper keeps its final Merge-Fiber
    output sorted) on the headline product in 16 even column batches, one
    layer: the unsorted product; every column hashed then sorted into a
    second buffer; and the hybrid, where columns of at most 4096 terms and
    compression ratio up to cf are formed in row order by expand-sort-compress
    (the paper finds its CPU hybrid ahead at one layer and low compression
    ratio), at several cf.  Kernel times from the library's HIP events; the
    sort pass's compulsory bytes: every entry it sorts read and written once
    (r bytes each)."""
    dev = torch.device("cuda:0")
    A = synth.rmat(args.scale, 16, synth.WORKLOADS["rmat20"].seed, dtype=torch.float32, device=dev)
    bounds = np.linspace(0, A.ncols, 16 + 1).astype(np.int64)
    runs = {}
    nnz_c = 0
    for sorted_flag in (False, True):
        eng = S.Engine(A, A, 1, budget_bytes=1 << 62, sorted_output=sorted_flag)
        plan = eng.plan()
        # the same column ranges in every run (the sorted runs hold each
        # batch twice, so batches are kept small)
        plan.bounds = bounds.tolist()
        plan.batch_nnz = np.stack([plan.nnz_host[:, a:b].sum(1) for a, b in zip(bounds[:-1], bounds[1:])])
        nnz_c = int(plan.nnz_host[0].sum())

        def step():
            for i in range(plan.nbatches):
                eng.run_batch(plan, i)

        for cf in ((None,) if not sorted_flag else (0.0, 1.25, 2.0, 4.0, 1e9)):
            if cf is not None:
                eng.esc_cf = cf
            step()
            torch.cuda.synchronize()
            eng.check()
            S.profile_enable(True)
            t = _timed(step, 1, torch)
            prof = S.profile_report()
            S.profile_enable(False)
            eng.check()
            name = "unsorted" if cf is None else ("sorted_hash_all" if cf == 0 else
                                                 ("sorted_hybrid_all_small" if cf >= 1e9 else f"sorted_hybrid_cf{cf:g}"))
            runs[name] = {"ms": round(t * 1e3, 3),
                          "kernels_ms": {k: round(v[0], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])
                                         if v[0] >= 0.05}}
            if cf is not None:
                runs[name]["esc_cf"] = cf
        del eng
        torch.cuda.empty_cache()
    t_u = runs["unsorted"]["ms"]
    h = runs["sorted_hash_all"]
    sort_ms = h["kernels_ms"].get("sort_columns", 0.0)
    sort_bytes = 2 * 8 * nnz_c + 8 * (A.ncols + len(bounds))
    gbs = sort_bytes / (sort_ms * 1e-3) / 1e9 if sort_ms > 0 else None
    best = min((k for k in runs if k.startswith("sorted_hybrid")), key=lambda k: runs[k]["ms"])
    log(f"sorted: unsorted {t_u:.1f} ms, hash+sort {h['ms']:.1f} ms (sort pass {sort_ms:.1f} ms, "
        f"{gbs or 0:.0f} GB/s compulsory), best hybrid {best} {runs[best]['ms']:.1f} ms; "
        + ", ".join(f"{k}={v['ms']:.1f}" for k, v in runs.items()))
    return {"workload": "rmat20 headline product, one layer, 16 even column batches: unsorted, row-sorted with "
                        "every column hashed then sorted, and row-sorted by the hybrid at several cf",
            "batches": len(bounds) - 1, "nnz_C": nnz_c, "runs": runs,
            "numeric_unsorted_ms": t_u, "numeric_sorted_ms": h["ms"],
            "sorted_over_unsorted_time": round(h["ms"] / t_u, 3),
            "best_hybrid": best, "best_hybrid_over_hash_sort_time": round(runs[best]["ms"] / h["ms"], 3),
            "sort_pass_ms": sort_ms, "sort_compulsory_bytes": sort_bytes,
            "sort_achieved_GBps": None if gbs is None else round(gbs, 1),
            "sort_frac_of_hbm_peak": None if gbs is None else round(gbs / HBM_PEAK_GBS, 4)}


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2010_08526_amd as S
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
        return
    res, A = headline(args, torch, np, S, synth)
    torch.cuda.empty_cache()
    if not args.no_extras:
        for name, fn in (("fwd_bwd", fwd_bwd), ("batched", batched), ("layered", layered), ("bsweep", bsweep),
                         ("prune", prune), ("aat", aat), ("sorted_output", sorted_output)):
            if name in args.extras.split(","):
                res[name] = fn(args, torch, np, S, synth)
                torch.cuda.empty_cache()
    res["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(A, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
