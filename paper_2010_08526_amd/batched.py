"""Batched products in one graph-capturable launch sequence.

A batch of independent products C_i = A_i B_i is the product of the
block-diagonal packings of the A_i and the B_i: one symbolic pass, one scan
and one numeric pass cover every instance, and the column binning evens out
the uneven instances.  BatchedEngine runs that sequence with no host
synchronization (spgemm_batched_forward / spgemm_batched_backward), so it
can be captured once in a HIP graph and replayed.  The autotuner picks the
bin thresholds (spgemm_set_bin_caps) by timing replays; thresholds change
speed, never results.

Argument marshalling only: all arithmetic runs in the library.
"""
from __future__ import annotations

import ctypes
import json
import os
import time

import numpy as np
import torch

from . import (CSC, F32, OP_BATCHED_BACKWARD, OP_BATCHED_FORWARD, OP_SYMBOLIC, _check, _lib, _ptr, _stream,
               alloc_workspace, check_ws, desc, spgemm_csc, symbolic, workspace_size)


SYM_TABLE_CAP = (32, 128, 512, 2048, 16384)
NUM_TABLE_CAP = (32, 128, 512, 2048, 5120)


def set_bin_caps(which: int, caps=None):
    """Bin thresholds for the symbolic (0) or numeric/masked (1) kernels, or
    workgroups per compute unit of the numeric (2) or symbolic (3) bin
    kernels; None restores the defaults."""
    arr = None if caps is None else np.ascontiguousarray(np.asarray(caps, dtype=np.int64))
    _check(_lib.spgemm_set_bin_caps(which, None if arr is None else arr.ctypes.data), "spgemm_set_bin_caps")


def batch_pack(instances, device="cuda", stream=None):
    """Block-diagonal packing of a list of CSC instances (device tensors).
    Returns (packed CSC, offsets int64 [count+1, 3] of (row, col, entry))."""
    count = len(instances)
    arr = (spgemm_csc * count)(*[desc(M) for M in instances])
    offs = np.zeros(3 * (count + 1), np.int64)
    rows = sum(int(M.nrows) for M in instances)
    cols = sum(int(M.ncols) for M in instances)
    nnz = sum(int(M.rowidx.numel()) for M in instances)
    vdt = instances[0].values.dtype if instances[0].values is not None else None
    cp = torch.empty(cols + 1, dtype=torch.int64, device=device)
    ri = torch.empty(max(1, nnz), dtype=torch.int32, device=device)
    v = torch.empty(max(1, nnz), dtype=vdt, device=device) if vdt is not None else None
    ws = alloc_workspace(64 * max(1, count), device)
    _check(_lib.spgemm_batch_pack(arr, count, _ptr(cp), _ptr(ri), _ptr(v), offs.ctypes.data, _ptr(ws), ws.numel(),
                                  _stream(stream)), "spgemm_batch_pack")
    return CSC(rows, cols, cp, ri[:nnz], None if v is None else v[:nnz]), offs.reshape(count + 1, 3)


# Scratch of the allocation-free forward (SPGEMM_NOALLOC_SCRATCH_BYTES in spgemm.h).
NOALLOC_SCRATCH_BYTES = 64 << 20
_lib.spgemm_batched_forward_noalloc.argtypes = [ctypes.POINTER(spgemm_csc), ctypes.POINTER(spgemm_csc),
                                                ctypes.c_int64] + [ctypes.c_void_p] * 6


def batched_forward_noalloc(A, B, nnz_cap: int, flops, nnz, colptr, rowidx, values, stream=None):
    """spgemm_batched_forward without a workspace argument: the library's
    fixed per-device scratch serves it (inputs whose workspace would exceed
    NOALLOC_SCRATCH_BYTES are refused).  Outputs are the caller's; the call
    allocates nothing."""
    _check(_lib.spgemm_batched_forward_noalloc(ctypes.byref(desc(A)), ctypes.byref(desc(B)), int(nnz_cap),
                                               _ptr(flops), _ptr(nnz), _ptr(colptr), _ptr(rowidx), _ptr(values),
                                               _stream(stream)), "spgemm_batched_forward_noalloc")


class BatchedEngine:
    """Forward (and the fused backward) of a packed product, host-sync free.

    The output capacity is set once from a synchronizing symbolic pass, so
    replays with the same patterns never overflow it."""

    def __init__(self, A, B, backward: bool = False, device="cuda"):
        self.A, self.B = A, B
        dev = device
        n = B.ncols
        ws = alloc_workspace(workspace_size(OP_SYMBOLIC, A, B, 0, n, 1), dev)
        cnt = torch.empty(n, dtype=torch.int64, device=dev)
        symbolic(A, B, 0, n, 1, None, cnt, ws)
        self.nnz_c = int(cnt.sum())
        del ws, cnt
        vdt = A.values.dtype
        self.flops = torch.empty(n, dtype=torch.int64, device=dev)
        self.nnz = torch.empty(n, dtype=torch.int64, device=dev)
        self.colptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        self.rowidx = torch.empty(max(1, self.nnz_c), dtype=torch.int32, device=dev)
        self.values = torch.empty(max(1, self.nnz_c), dtype=vdt, device=dev)
        self.ws = alloc_workspace(workspace_size(OP_BATCHED_FORWARD, A, B, 0, n), dev)
        self.has_backward = backward
        if backward:
            self.ws_b = alloc_workspace(workspace_size(OP_BATCHED_BACKWARD, A, B, 0, n), dev)
            self.dA = torch.empty(max(1, A.nnz), dtype=vdt, device=dev)
            self.dB = torch.empty(max(1, B.nnz), dtype=vdt, device=dev)
        self.graph = None

    @property
    def C(self) -> CSC:
        return CSC(self.A.nrows, self.B.ncols, self.colptr, self.rowidx[:self.nnz_c], self.values[:self.nnz_c])

    def forward(self, stream=None):
        _check(_lib.spgemm_batched_forward(ctypes.byref(desc(self.A)), ctypes.byref(desc(self.B)), self.nnz_c,
                                           _ptr(self.flops), _ptr(self.nnz), _ptr(self.colptr), _ptr(self.rowidx),
                                           _ptr(self.values), _ptr(self.ws), self.ws.numel(), _stream(stream)),
               "spgemm_batched_forward")

    def backward(self, dC: torch.Tensor, stream=None):
        Cp = CSC(self.A.nrows, self.B.ncols, self.colptr, self.rowidx[:self.nnz_c], None)
        cd = desc(Cp, F32)
        _check(_lib.spgemm_batched_backward(ctypes.byref(desc(self.A)), ctypes.byref(desc(self.B)), ctypes.byref(cd),
                                            _ptr(dC), _ptr(self.dA), _ptr(self.dB), _ptr(self.ws_b),
                                            self.ws_b.numel(), _stream(stream)), "spgemm_batched_backward")
        return self.dA[:self.A.nnz], self.dB[:self.B.nnz]

    def check(self, stream=None):
        check_ws(self.ws, "device-side check (batched forward)", stream)
        if self.has_backward:
            check_ws(self.ws_b, "device-side check (batched backward)", stream)

    # -- HIP graph ----------------------------------------------------------
    def capture(self, body):
        """Captures body() (library calls on the current stream) in a graph;
        replay() runs it again."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            body()  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            body()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()


def spgemm_batched(pairs, graph: bool = True, device="cuda"):
    """C_i = A_i B_i for a list of (A_i, B_i) pairs of device CSCs, as one
    packed product: one symbolic pass, one scan and one numeric pass over all
    instances.  With graph=True the forward is captured in a HIP graph and
    run by a replay.  Returns (list of C_i, rows local to each instance, the
    engine); the engine replays the product for new values of the same
    patterns (its packed A and B hold the values).  The C_i are views of the
    engine's output buffers: a replay rewrites them in place."""
    if not pairs:
        raise ValueError("no instances")
    As = [a for a, _ in pairs]
    Bs = [b for _, b in pairs]
    for i, (a, b) in enumerate(pairs):
        if int(a.ncols) != int(b.nrows):
            raise ValueError(f"instance {i}: A has {a.ncols} columns, B has {b.nrows} rows")
        if a.values is None or b.values is None or a.values.dtype != As[0].values.dtype or \
                b.values.dtype != As[0].values.dtype:
            raise ValueError(f"instance {i}: every operand needs values of one dtype")
    A, offA = batch_pack(As, device)
    B, offB = batch_pack(Bs, device)
    eng = BatchedEngine(A, B, device=device)
    if graph:
        eng.capture(eng.forward)
        eng.replay()
    else:
        eng.forward()
    eng.check()
    C = eng.C
    cp = C.colptr.cpu().numpy()
    out = []
    for i in range(len(pairs)):
        c0, c1 = int(offB[i, 1]), int(offB[i + 1, 1])
        e0, e1 = int(cp[c0]), int(cp[c1])
        out.append(CSC(int(As[i].nrows), int(Bs[i].ncols), C.colptr[c0:c1 + 1] - e0,
                       C.rowidx[e0:e1] - int(offA[i, 0]), C.values[e0:e1]))
    return out, eng


# ------------------------------------------------------------------ autotuner
def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_2010_08526_amd", "autotune.json")


def _candidates():
    """Threshold sets for the numeric kernels: the defaults (load factor up
    to 1/2), lighter tables (up to 3/8 and 1/4 full), and columns of more than
    256 or 128 rows moved from the 1024-slot wave tables to the workgroup
    tables."""
    out = [tuple(NUM_TABLE_CAP)]
    for lf in (0.375, 0.25):
        out.append(tuple(max(1, int(c * 2 * lf)) for c in NUM_TABLE_CAP))
    c = list(NUM_TABLE_CAP)
    for cap2 in (256, 128):
        out.append(tuple([c[0], min(c[1], cap2), cap2] + c[3:]))
    return out


def workload_key(A, B) -> str:
    dev = torch.cuda.get_device_properties(A.rowidx.device)
    arch = getattr(dev, "gcnArchName", dev.name)
    deg = max(1, A.nnz // max(1, A.ncols)) * max(1, B.nnz // max(1, B.ncols))
    cls = int(np.log2(deg)) if deg > 0 else 0
    return f"{arch}|{A.values.dtype}|flops_per_col_2^{cls}"


NUM_BPC = (8, 8, 4, 4, 1)  # workgroups per CU of the numeric bin kernels (library defaults)
SYM_BPC = (8, 8, 8, 8, 1)  # the same for the symbolic bin kernels


def _bpc_candidates(default):
    """Launch shapes of the five bin kernels: the defaults, half as many and
    twice as many workgroups per compute unit (at least 1, at most 32)."""
    half = tuple(max(1, x // 2) for x in default)
    double = tuple(min(32, 2 * x) for x in default)
    return [tuple(default), half, double]


def _apply(setting):
    set_bin_caps(1, setting["caps"])
    set_bin_caps(2, setting["num_bpc"])
    set_bin_caps(3, setting["sym_bpc"])


def autotune(eng: BatchedEngine, reps: int = 3, use_cache: bool = True, verbose: bool = False):
    """Times forward replays while it searches, one knob at a time, the
    numeric bin thresholds (hash-table load factor), then the workgroups per
    compute unit of the numeric bin kernels, then those of the symbolic bin
    kernels; keeps the fastest setting and records it per (arch, dtype,
    workload class).  Settings change speed, never results."""
    key = workload_key(eng.A, eng.B)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache and "num_bpc" in cache[key]:
        _apply(cache[key])
        return cache[key]

    def timed(setting):
        _apply(setting)
        eng.forward()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            eng.forward()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    best = {"caps": tuple(NUM_TABLE_CAP), "num_bpc": NUM_BPC, "sym_bpc": SYM_BPC}
    best_t = timed(best)
    results = [{**{k: list(v) for k, v in best.items()}, "ms": best_t * 1e3}]
    default_ms = best_t * 1e3
    for knob, cands in (("caps", _candidates()), ("num_bpc", _bpc_candidates(NUM_BPC)),
                        ("sym_bpc", _bpc_candidates(SYM_BPC))):
        for c in cands:
            if tuple(c) == tuple(best[knob]):
                continue
            trial = dict(best)
            trial[knob] = tuple(c)
            dt = timed(trial)
            results.append({**{k: list(v) for k, v in trial.items()}, "ms": dt * 1e3})
            if verbose:
                print(f"# autotune {knob}={c} {dt * 1e3:.3f} ms", flush=True)
            if dt < best_t:
                best, best_t = trial, dt
    _apply(best)
    entry = {**{k: list(v) for k, v in best.items()}, "ms": best_t * 1e3, "default_ms": default_ms,
             "tried": results}
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return entry
