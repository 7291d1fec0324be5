"""Python binding of libspgemm (the C ABI in include/spgemm.h).

Argument marshalling only: every step of the product runs in the library's
HIP kernels or its host-side planner.  torch supplies device memory and
streams.  torch is imported before the library is loaded so that both use
one HIP runtime.  There is no fallback: if the library is missing the
import fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libspgemm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_2010_08526_amd/build.py`")
_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
OK, E_INVAL, E_SHAPE, E_DTYPE, E_BUDGET, E_WORKSPACE, E_HIP, E_OVERFLOW, E_DEVICE = 0, -1, -2, -3, -4, -5, -6, -7, -8
F32, F64 = 0, 1
# semirings of the numeric pass and the merge (spgemm_semiring)
PLUS_TIMES, MIN_PLUS, OR_AND = 0, 1, 2
SEMIRINGS = {"plus_times": PLUS_TIMES, "min_plus": MIN_PLUS, "or_and": OR_AND}
(OP_SYMBOLIC, OP_NUMERIC, OP_MERGE, OP_COLPTR, OP_MASKED_XTY, OP_TRANSPOSE, OP_BATCHED_FORWARD, OP_BATCHED_BACKWARD,
 OP_PRUNE, OP_SORT) = range(10)
MAX_PARTS = 4096

_DTYPE = {torch.float32: F32, torch.float64: F64}


class spgemm_csc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("dtype", ctypes.c_int32)]


_P = ctypes.POINTER(spgemm_csc)
_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t

_lib.spgemm_workspace_size.argtypes = [ctypes.c_int, _P, _P, _i64, _i64, _i32, ctypes.POINTER(_sz)]
_lib.spgemm_symbolic.argtypes = [_P, _P, _i64, _i64, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.spgemm_plan_batches.argtypes = [_vp, _i64, _i32, _i32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _i32,
                                     _vp, ctypes.POINTER(_i32), _vp]
_lib.spgemm_colptr.argtypes = [_vp, _i64, _vp, _vp, _sz, _vp]
_lib.spgemm_numeric.argtypes = [_P, _P, _i64, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp]
_lib.spgemm_merge.argtypes = [_P, _i32, _vp, _vp, _vp, _i32, _vp, _sz, _vp]
_lib.spgemm_ws_status.argtypes = [_vp, _vp]
_lib.spgemm_ws_status_code.argtypes = [_vp, _vp, _vp]
_lib.spgemm_ws_invalidate.argtypes = [_vp, _vp]
_lib.spgemm_batched_forward.argtypes = [_P, _P, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.spgemm_batched_masked_xty.argtypes = [_P, _P, _P, _vp, _vp, _sz, _vp]
_lib.spgemm_batched_backward.argtypes = [_P, _P, _P, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.spgemm_set_bin_caps.argtypes = [_i32, _vp]
_lib.spgemm_batch_pack.argtypes = [_P, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.spgemm_debug_min_bin.argtypes = [_i32]
_lib.spgemm_profile_enable.argtypes = [_i32]
_lib.spgemm_profile_report.argtypes = [ctypes.c_char_p, _sz]


def profile_enable(on: bool = True):
    """Start (or stop) per-kernel HIP-event timing inside the library."""
    _check(_lib.spgemm_profile_enable(int(on)), "spgemm_profile_enable")


def profile_report() -> dict:
    """{kernel name: (total ms, launches)} since profile_enable(True)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.spgemm_profile_report(buf, len(buf)), "spgemm_profile_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, ms, cnt = line.split()
        out[name] = (float(ms), int(cnt))
    return out
_lib.spgemm_status_string.restype = ctypes.c_char_p
_lib.spgemm_status_string.argtypes = [ctypes.c_int]
_lib.spgemm_last_hip_error.restype = ctypes.c_int


class SpgemmError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = status_string(status)
        if status == E_HIP:
            msg += f" (hipError {int(_lib.spgemm_last_hip_error())})"
        super().__init__(f"{where}: {msg}" if where else msg)


def status_string(status: int) -> str:
    return _lib.spgemm_status_string(int(status)).decode()


def _check(rc: int, where: str):
    if rc != OK:
        raise SpgemmError(rc, where)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        return int(torch.cuda.current_stream().cuda_stream) if torch.cuda.is_available() else None
    return int(getattr(stream, "cuda_stream", stream))


@dataclass
class CSC:
    """A CSC matrix in torch tensors: colptr int64[ncols+1], rowidx int32[nnz],
    values float32/float64[nnz] (or None)."""

    nrows: int
    ncols: int
    colptr: torch.Tensor
    rowidx: torch.Tensor
    values: torch.Tensor | None

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())


def desc(M, dtype: int | None = None) -> spgemm_csc:
    """C descriptor of any object with nrows/ncols/colptr/rowidx/values."""
    v = M.values
    if dtype is None:
        dtype = _DTYPE.get(v.dtype, -1) if v is not None else F32
    return spgemm_csc(int(M.nrows), int(M.ncols), int(M.rowidx.numel()), _ptr(M.colptr), _ptr(M.rowidx), _ptr(v),
                      int(dtype))


# ------------------------------------------------------------ thin wrappers
def workspace_size(op: int, A=None, B=None, c0: int = 0, c1: int = 0, n_layers: int = 1) -> int:
    out = _sz(0)
    a = ctypes.byref(desc(A)) if A is not None else None
    b = ctypes.byref(desc(B)) if B is not None else None
    _check(_lib.spgemm_workspace_size(op, a, b, c0, c1, n_layers, ctypes.byref(out)), "spgemm_workspace_size")
    return int(out.value)


def alloc_workspace(nbytes: int, device=None) -> torch.Tensor:
    """A 256-byte aligned device buffer (torch's allocator aligns to 512)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")
    assert t.data_ptr() % 256 == 0
    t[:4096].zero_()  # header: no status recorded before the first call
    return t


def symbolic(A, B, c0: int, c1: int, n_layers: int, flops_out, nnz_out, ws: torch.Tensor, stream=None):
    _check(_lib.spgemm_symbolic(ctypes.byref(desc(A)), ctypes.byref(desc(B)), c0, c1, n_layers, _ptr(flops_out),
                                _ptr(nnz_out), _ptr(ws), ws.numel(), _stream(stream)), "spgemm_symbolic")


def plan_batches(nnz_host, ncols: int, n_layers: int, value_bytes: int, input_bytes: int, budget_bytes: int,
                 reserve_bytes: int = 0, max_batches: int = 1 << 16):
    """Returns (bounds: list[int], batch_nnz: np.ndarray[b, rows])."""
    nnz_host = np.ascontiguousarray(np.asarray(nnz_host, dtype=np.int64))
    rows = n_layers + 1 if n_layers > 1 else 1
    bounds = np.zeros(max_batches + 1, np.int64)
    tot = np.zeros(max_batches * rows, np.int64)
    nb = _i32(0)
    _check(_lib.spgemm_plan_batches(nnz_host.ctypes.data, ncols, n_layers, value_bytes, int(input_bytes),
                                    int(budget_bytes), int(reserve_bytes), max_batches, bounds.ctypes.data,
                                    ctypes.byref(nb), tot.ctypes.data), "spgemm_plan_batches")
    b = int(nb.value)
    return bounds[:b + 1].tolist(), tot[:b * rows].reshape(b, rows)


def colptr(counts: torch.Tensor, out: torch.Tensor, ws: torch.Tensor, stream=None):
    n = counts.numel()
    _check(_lib.spgemm_colptr(_ptr(counts), n, _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "spgemm_colptr")


def semiring_id(semiring) -> int:
    """spgemm_semiring value of a name ('plus_times', 'min_plus', 'or_and') or id."""
    if isinstance(semiring, str):
        if semiring not in SEMIRINGS:
            raise ValueError(f"unknown semiring {semiring!r}")
        return SEMIRINGS[semiring]
    return int(semiring)


def numeric(A, B, c0: int, c1: int, layer: int, n_layers: int, flops, c_colptr, c_rowidx, c_values,
            ws: torch.Tensor, stream=None, semiring=PLUS_TIMES):
    _check(_lib.spgemm_numeric(ctypes.byref(desc(A)), ctypes.byref(desc(B)), c0, c1, layer, n_layers, _ptr(flops),
                               _ptr(c_colptr), _ptr(c_rowidx), _ptr(c_values), semiring_id(semiring), _ptr(ws),
                               ws.numel(), _stream(stream)), "spgemm_numeric")


_lib.spgemm_numeric_sorted.argtypes = [_P, _P, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, _i32, _vp,
                                       _sz, _vp]

# Compression ratio up to which a column of at most 4096 product terms is
# formed in row order by expand-sort-compress rather than hashed and sorted.
ESC_CF_DEFAULT = 2.0


def numeric_sorted(A, B, c0: int, c1: int, flops, c_colptr, c_rowidx, c_values, tmp_rowidx, tmp_values,
                   ws: torch.Tensor, stream=None, semiring=PLUS_TIMES, esc_cf: float = ESC_CF_DEFAULT):
    """Columns [c0, c1) of A*B in row order: low-compression columns by
    expand-sort-compress, the others hashed into tmp_* and sorted."""
    _check(_lib.spgemm_numeric_sorted(ctypes.byref(desc(A)), ctypes.byref(desc(B)), c0, c1, _ptr(flops),
                                      _ptr(c_colptr), _ptr(c_rowidx), _ptr(c_values), _ptr(tmp_rowidx),
                                      _ptr(tmp_values), float(esc_cf), semiring_id(semiring), _ptr(ws), ws.numel(),
                                      _stream(stream)), "spgemm_numeric_sorted")


def merge(parts, c_colptr, c_rowidx, c_values, ws: torch.Tensor, stream=None, semiring=PLUS_TIMES):
    arr = (spgemm_csc * len(parts))(*[desc(p) for p in parts])
    _check(_lib.spgemm_merge(arr, len(parts), _ptr(c_colptr), _ptr(c_rowidx), _ptr(c_values), semiring_id(semiring),
                             _ptr(ws), ws.numel(), _stream(stream)), "spgemm_merge")


_lib.spgemm_sort_columns.argtypes = [_P, _vp, _vp, _vp, _sz, _vp]


def sort_columns(C, rowidx_out: torch.Tensor | None = None, values_out: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, stream=None) -> CSC:
    """C with every column's entries in row order (values moved with their
    rows), written to separate arrays; C's column pointers are shared."""
    dev = C.rowidx.device
    n = C.nnz
    if ws is None:
        ws = alloc_workspace(workspace_size(OP_SORT, C), dev)
    if rowidx_out is None:
        rowidx_out = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    if values_out is None:
        values_out = torch.empty(max(1, n), dtype=C.values.dtype, device=dev)
    _check(_lib.spgemm_sort_columns(ctypes.byref(desc(C)), _ptr(rowidx_out), _ptr(values_out), _ptr(ws), ws.numel(),
                                    _stream(stream)), "spgemm_sort_columns")
    return CSC(C.nrows, C.ncols, C.colptr, rowidx_out[:n], values_out[:n])


def ws_status(ws: torch.Tensor, stream=None) -> int:
    """Synchronizes and returns the device-side status of a workspace."""
    return int(_lib.spgemm_ws_status(_ptr(ws), _stream(stream)))


def ws_invalidate(ws: torch.Tensor, stream=None):
    """Drops what the workspace keeps between numeric calls (the slabbed copy of A)."""
    _check(_lib.spgemm_ws_invalidate(_ptr(ws), _stream(stream)), "spgemm_ws_invalidate")


def ws_status_code(ws: torch.Tensor, stream=None) -> tuple[int, int]:
    """(status, first device-side code) of a workspace; clears the code."""
    code = ctypes.c_int32(0)
    rc = int(_lib.spgemm_ws_status_code(_ptr(ws), _stream(stream), ctypes.byref(code)))
    return rc, int(code.value)


def check_ws(ws: torch.Tensor, where: str = "device check", stream=None):
    rc, code = ws_status_code(ws, stream)
    _check(rc, f"{where} (device code {code})" if code else where)


# -------------------------------------------------------------- batch loop
def layer_bounds(kdim: int, n_layers: int) -> list[tuple[int, int]]:
    """The inner-dimension ranges the library uses for n_layers layers."""
    w = -(-kdim // n_layers) if n_layers > 0 else kdim
    return [(min(kdim, l * w), min(kdim, l * w + w)) for l in range(n_layers)]


@dataclass
class Plan:
    """Result of the symbolic pass and the planner for one product."""

    flops: torch.Tensor  # int64 [n] per output column (device)
    nnz: torch.Tensor  # int64 [rows, n] (device)
    nnz_host: np.ndarray  # int64 [rows, n]
    bounds: list
    batch_nnz: np.ndarray  # [b, rows]
    n_layers: int
    budget_bytes: int
    input_bytes: int
    reserve_bytes: int

    @property
    def nbatches(self) -> int:
        return len(self.bounds) - 1

    @property
    def total_flops(self) -> int:
        return int(self.flops.sum())


class Engine:
    """Holds workspaces and output buffers for repeated products of one shape.

    run(A, B) performs: symbolic pass -> counts to host -> batch planner ->
    per batch (numeric per layer [-> merge]) -> consume(c0, c1, C_batch).
    """

    def __init__(self, A, B, n_layers: int = 1, budget_bytes: int | None = None, max_batches: int = 1 << 16,
                 device="cuda", semiring=PLUS_TIMES, sorted_output: bool = False, esc_cf: float = ESC_CF_DEFAULT):
        if A.ncols != B.nrows:
            raise SpgemmError(E_SHAPE, "Engine")
        self.A, self.B, self.L = A, B, int(n_layers)
        self.semiring = semiring_id(semiring)
        # row-sorted output columns: each batch is formed, then sorted into a
        # second buffer of the same size (counted by the planner); with one
        # layer, columns of compression ratio up to esc_cf (and at most 4096
        # terms) are formed in row order directly (0: every column hashed)
        self.sorted_output = bool(sorted_output)
        self.esc_cf = float(esc_cf)
        self.device = device
        self.max_batches = max_batches
        self.vbytes = 4 if A.values is None or A.values.dtype == torch.float32 else 8
        self.vdtype = torch.float32 if self.vbytes == 4 else torch.float64
        n = B.ncols
        self.ws_sym = alloc_workspace(workspace_size(OP_SYMBOLIC, A, B, 0, n, self.L), device)
        self.ws_num = alloc_workspace(workspace_size(OP_NUMERIC, A, B, 0, n, self.L), device)
        mparts = CSC(A.nrows, n, A.colptr, A.rowidx, A.values)
        self.ws_mrg = alloc_workspace(workspace_size(OP_MERGE, mparts, None, 0, 0, max(1, self.L)), device) \
            if self.L > 1 else None
        self.ws_scan = alloc_workspace(workspace_size(OP_COLPTR, None, None, 0, n + 1), device)
        self.ws_sort = alloc_workspace(workspace_size(OP_SORT, CSC(A.nrows, n, B.colptr, B.rowidx, B.values)), device) \
            if self.sorted_output and self.L > 1 else None
        rows = self.L + 1 if self.L > 1 else 1
        self.flops = torch.empty(n, dtype=torch.int64, device=device)
        self.nnz = torch.empty((rows, n), dtype=torch.int64, device=device)
        r = 4 + self.vbytes
        self.input_bytes = r * (A.nnz + B.nnz) + 8 * (A.ncols + B.ncols + 2)
        self.reserve_bytes = sum(int(w.numel()) for w in (self.ws_sym, self.ws_num, self.ws_mrg, self.ws_scan,
                                                          self.ws_sort) if w is not None) + 8 * 4 * (n + 1) * rows
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.9) + self.input_bytes + self.reserve_bytes
        self.budget_bytes = int(budget_bytes)
        self._bufs = None

    # -- passes --------------------------------------------------------------
    def plan(self, stream=None) -> Plan:
        A, B, n = self.A, self.B, self.B.ncols
        # a product starts from scratch: its batches share one slabbed copy of A
        ws_invalidate(self.ws_num, stream)
        symbolic(A, B, 0, n, self.L, self.flops, self.nnz, self.ws_sym, stream)
        nnz_host = self.nnz.cpu().numpy()
        counts = nnz_host
        if self.sorted_output:  # the merged batch is held twice: as formed and sorted
            counts = nnz_host.copy()
            counts[-1] *= 2
        bounds, tot = plan_batches(counts.reshape(-1), n, self.L, self.vbytes, self.input_bytes, self.budget_bytes,
                                   self.reserve_bytes, self.max_batches)
        if self.sorted_output:
            tot = np.stack([nnz_host[:, a:b].sum(1) for a, b in zip(bounds[:-1], bounds[1:])]) if len(bounds) > 1 \
                else tot
        return Plan(self.flops, self.nnz, nnz_host, bounds, tot, self.L, self.budget_bytes, self.input_bytes,
                    self.reserve_bytes)

    def _buffers(self, plan: Plan):
        widths = [b - a for a, b in zip(plan.bounds[:-1], plan.bounds[1:])]
        wmax = max(widths) if widths else 0
        L = self.L
        if L == 1:
            need = (wmax, int(plan.batch_nnz[:, 0].max()) if plan.nbatches else 0, 0)
        else:
            need = (wmax, int(plan.batch_nnz[:, L].max()), int(plan.batch_nnz[:, :L].sum(1).max()))
        if self._bufs is None or any(x > y for x, y in zip(need, self._bufs["need"])):
            dev = self.device
            bufs = {"need": need,
                    "ccp": torch.empty(need[0] + 1, dtype=torch.int64, device=dev),
                    "cri": torch.empty(max(1, need[1]), dtype=torch.int32, device=dev),
                    "cv": torch.empty(max(1, need[1]), dtype=self.vdtype, device=dev)}
            if self.sorted_output:
                bufs["sri"] = torch.empty(max(1, need[1]), dtype=torch.int32, device=dev)
                bufs["sv"] = torch.empty(max(1, need[1]), dtype=self.vdtype, device=dev)
            if L > 1:
                bufs["dcp"] = torch.empty((L, need[0] + 1), dtype=torch.int64, device=dev)
                bufs["dri"] = torch.empty(max(1, need[2]), dtype=torch.int32, device=dev)
                bufs["dv"] = torch.empty(max(1, need[2]), dtype=self.vdtype, device=dev)
            self._bufs = bufs
        return self._bufs

    def release_buffers(self):
        """Drops the output buffers (they are allocated again, at the size the next plan needs)."""
        self._bufs = None

    def run_batch(self, plan: Plan, i: int, stream=None, marks=None) -> CSC:
        """Forms batch i; the returned CSC views buffers reused by the next call.
        With ``marks`` (a list), (phase, start_event, end_event) tuples are
        appended for the numeric and merge phases (HIP events on the stream)."""
        A, B, L = self.A, self.B, self.L

        def mark():
            if marks is None:
                return None
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.current_stream())
            return e
        c0, c1 = plan.bounds[i], plan.bounds[i + 1]
        w = c1 - c0
        bufs = self._buffers(plan)
        ccp, cri, cv = bufs["ccp"][:w + 1], bufs["cri"], bufs["cv"]
        if L == 1:
            e0 = mark()
            colptr(self.nnz[0, c0:c1], ccp, self.ws_scan, stream)
            nnzc = int(plan.batch_nnz[i, 0])
            if self.sorted_output:  # formed in row order (hashed columns staged in cri / cv)
                numeric_sorted(A, B, c0, c1, self.flops[c0:c1], ccp, bufs["sri"], bufs["sv"], cri, cv, self.ws_num,
                               stream, self.semiring, self.esc_cf)
                if marks is not None:
                    marks.append(("numeric_sorted", e0, mark()))
                return CSC(A.nrows, w, ccp, bufs["sri"][:nnzc], bufs["sv"][:nnzc])
            numeric(A, B, c0, c1, 0, 1, self.flops[c0:c1], ccp, cri, cv, self.ws_num, stream, self.semiring)
            if marks is not None:
                marks.append(("numeric", e0, mark()))
        else:
            parts = []
            off = 0
            e0 = mark()
            for l in range(L):
                dcp = bufs["dcp"][l, :w + 1]
                colptr(self.nnz[l, c0:c1], dcp, self.ws_scan, stream)
                cnt = int(plan.batch_nnz[i, l])
                dri = bufs["dri"][off:off + cnt]
                dv = bufs["dv"][off:off + cnt]
                numeric(A, B, c0, c1, l, L, self.flops[c0:c1], dcp, dri, dv, self.ws_num, stream, self.semiring)
                parts.append(CSC(A.nrows, w, dcp, dri, dv))
                off += cnt
            e1 = mark()
            colptr(self.nnz[L, c0:c1], ccp, self.ws_scan, stream)
            merge(parts, ccp, cri, cv, self.ws_mrg, stream, self.semiring)
            if marks is not None:
                marks.append(("numeric", e0, e1))
                marks.append(("merge", e1, mark()))
            nnzc = int(plan.batch_nnz[i, L])
        if self.sorted_output:
            e0 = mark()
            Cs = sort_columns(CSC(A.nrows, w, ccp, cri[:nnzc], cv[:nnzc]), bufs["sri"], bufs["sv"], self.ws_sort, stream)
            if marks is not None:
                marks.append(("sort", e0, mark()))
            return Cs
        return CSC(A.nrows, w, ccp, cri[:nnzc], cv[:nnzc])

    def check(self, stream=None):
        for w in (self.ws_sym, self.ws_num, self.ws_mrg, self.ws_sort):
            if w is not None:
                check_ws(w, "device-side check", stream)

    def run(self, consume=None, stream=None):
        """All batches; consume(c0, c1, C_batch) per batch, or the whole C."""
        plan = self.plan(stream)
        out = [] if consume is None else None
        for i in range(plan.nbatches):
            Cb = self.run_batch(plan, i, stream)
            if consume is None:
                out.append(CSC(Cb.nrows, Cb.ncols, Cb.colptr.clone(), Cb.rowidx.clone(), Cb.values.clone()))
            else:
                consume(plan.bounds[i], plan.bounds[i + 1], Cb)
        self.check(stream)
        if consume is not None:
            return plan
        return _concat(out, self.A.nrows), plan


def _concat(batches, nrows):
    ncols = sum(b.ncols for b in batches)
    cps = []
    off = 0
    for b in batches:
        cps.append(b.colptr[:-1] + off)
        off += b.nnz
    dev = batches[0].rowidx.device if batches else "cuda"
    cps.append(torch.tensor([off], dtype=torch.int64, device=dev))
    return CSC(nrows, ncols, torch.cat(cps), torch.cat([b.rowidx for b in batches]),
               torch.cat([b.values for b in batches]))


def spgemm(A, B, *, layers: int = 1, budget_bytes: int | None = None, consume=None, stream=None,
           semiring=PLUS_TIMES, sorted_output: bool = False, esc_cf: float = ESC_CF_DEFAULT):
    """C = A B over ``semiring`` ('plus_times', 'min_plus', 'or_and'), rows of
    each column in hash-table order or, with ``sorted_output``, ascending.
    With ``consume`` the batches are handed to it and discarded; otherwise C
    is returned (all batches concatenated)."""
    eng = Engine(A, B, layers, budget_bytes, semiring=semiring, sorted_output=sorted_output, esc_cf=esc_cf)
    res = eng.run(consume, stream)
    return res if consume is not None else res[0]


# ------------------------------------------------------ consumer of a batch
_lib.spgemm_prune_topk.argtypes = [_P, ctypes.c_double, _i64, _vp, _vp, _vp, _i64, _vp, _sz, _vp]


def prune_bound(nnz: int, ncols: int, k: int) -> int:
    """Most entries a pruned matrix can hold: min(nnz, k * ncols), nnz for k < 0."""
    return nnz if k < 0 else min(nnz, k * ncols)


def prune_topk(C, threshold: float, k: int, ws: torch.Tensor | None = None, stream=None) -> CSC:
    """Per-column pruning of an output batch (the consumer an application
    runs on each batch): entries >= threshold, then at most the k largest of
    each column (k < 0: no limit), equal values going to the smaller row;
    kept entries stay in input order.  Reads the entry count back to the
    host and checks the workspace status."""
    if C.values is None:
        raise ValueError("prune_topk needs values")
    dev = C.rowidx.device
    if ws is None:
        ws = alloc_workspace(workspace_size(OP_PRUNE, C), dev)
    cap = prune_bound(C.nnz, C.ncols, int(k))
    cp = torch.empty(C.ncols + 1, dtype=torch.int64, device=dev)
    ri = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
    v = torch.empty(max(1, cap), dtype=C.values.dtype, device=dev)
    _check(_lib.spgemm_prune_topk(ctypes.byref(desc(C)), float(threshold), int(k), _ptr(cp), _ptr(ri), _ptr(v), cap,
                                  _ptr(ws), ws.numel(), _stream(stream)), "spgemm_prune_topk")
    check_ws(ws, "device-side check (prune)", stream)
    n = int(cp[-1])
    return CSC(C.nrows, C.ncols, cp, ri[:n], v[:n])


def spgemm_topk(A, B, threshold: float, k: int, *, layers: int = 1, budget_bytes: int | None = None,
                stream=None) -> CSC:
    """C = A B formed batch by batch, every batch pruned as it is formed
    (``prune_topk``: entries >= threshold, at most the k largest per column)
    and only the pruned batches kept, concatenated: the whole product never
    needs to fit in memory, only one batch of it."""
    eng = Engine(A, B, layers, budget_bytes)
    ws = {}
    kept = []

    def consume(c0, c1, Cb):
        need = workspace_size(OP_PRUNE, Cb)
        if "ws" not in ws or ws["ws"].numel() < need:
            ws["ws"] = alloc_workspace(need, Cb.rowidx.device)
        kept.append(prune_topk(Cb, threshold, k, ws=ws["ws"], stream=stream))

    eng.run(consume, stream)
    if not kept:  # no batches
        dev = A.rowidx.device
        return CSC(A.nrows, B.ncols, torch.zeros(B.ncols + 1, dtype=torch.int64, device=dev),
                   torch.zeros(0, dtype=torch.int32, device=dev), torch.zeros(0, dtype=A.values.dtype, device=dev))
    return _concat(kept, A.nrows)


# ------------------------------------------------------------ gradient support
_lib.spgemm_transpose.argtypes = [_P, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.spgemm_masked_xty.argtypes = [_P, _P, _P, _vp, _vp, _sz, _vp]
_lib.spgemm_permute.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _vp]


def transpose(X, ws: torch.Tensor | None = None, values: bool = True, perm: bool = True, stream=None):
    """X^T as a CSC (values optional) and the permutation perm with
    X^T.values[q] = X.values[perm[q]]."""
    dev = X.rowidx.device
    if ws is None:
        ws = alloc_workspace(workspace_size(OP_TRANSPOSE, X), dev)
    tcp = torch.empty(X.nrows + 1, dtype=torch.int64, device=dev)
    tri = torch.empty(max(1, X.nnz), dtype=torch.int32, device=dev)
    tv = torch.empty(max(1, X.nnz), dtype=X.values.dtype, device=dev) if (values and X.values is not None) else None
    pm = torch.empty(max(1, X.nnz), dtype=torch.int64, device=dev) if perm else None
    _check(_lib.spgemm_transpose(ctypes.byref(desc(X)), _ptr(tcp), _ptr(tri), _ptr(tv), _ptr(pm), _ptr(ws),
                                 ws.numel(), _stream(stream)), "spgemm_transpose")
    n = X.nnz
    T = CSC(X.ncols, X.nrows, tcp, tri[:n], None if tv is None else tv[:n])
    return T, (None if pm is None else pm[:n])


def masked_xty(X, Y, M, out: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """out(k,j) = sum_i X(i,k) Y(i,j) for each stored (k,j) of M, in M's order."""
    dev = Y.rowidx.device
    if ws is None:
        ws = alloc_workspace(workspace_size(OP_MASKED_XTY, X, Y, 0, Y.ncols), dev)
    if out is None:
        out = torch.empty(max(1, M.nnz), dtype=Y.values.dtype, device=dev)
    Md = desc(M, F32)
    Md.values = None
    _check(_lib.spgemm_masked_xty(ctypes.byref(desc(X)), ctypes.byref(desc(Y)), ctypes.byref(Md), _ptr(out), _ptr(ws),
                                  ws.numel(), _stream(stream)), "spgemm_masked_xty")
    return out[:M.nnz]


def permute(src: torch.Tensor, perm: torch.Tensor, scatter: bool = False, out: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
    """Gather out[i] = src[perm[i]] or scatter out[perm[i]] = src[i]."""
    n = perm.numel()
    if out is None:
        out = torch.empty(n, dtype=src.dtype, device=src.device)
    _check(_lib.spgemm_permute(_ptr(src), _ptr(perm), n, _DTYPE[src.dtype], int(scatter), _ptr(out), _stream(stream)),
           "spgemm_permute")
    return out


class Backward:
    """Gradients of a loss on P(C), C = A B, with respect to the stored values
    of A and B.  The transposes of A's and B's patterns and of C's pattern are
    formed once (per structure) and reused."""

    def __init__(self, A, B, C, stream=None):
        self.A, self.B, self.C = A, B, C
        dev = C.rowidx.device
        self.ws_tr = alloc_workspace(max(workspace_size(OP_TRANSPOSE, M) for M in (A, B, C)), dev)
        self.AT, self.permA = transpose(A, self.ws_tr, values=False, perm=True, stream=stream)
        self.CT, self.permC = transpose(C, self.ws_tr, values=False, perm=True, stream=stream)
        self.BT, self.permB = transpose(B, self.ws_tr, values=True, perm=True, stream=stream)
        self.ws_b = alloc_workspace(workspace_size(OP_MASKED_XTY, A, C, 0, C.ncols), dev)
        self.ws_a = alloc_workspace(workspace_size(OP_MASKED_XTY, self.BT, self.CT, 0, self.CT.ncols), dev)

    def refresh_values(self, B, stream=None):
        """New values of B (same pattern): B^T's values are re-gathered."""
        self.B = B
        permute(B.values, self.permB, False, self.BT.values, stream)

    def __call__(self, dC_values: torch.Tensor, stream=None):
        A, B, C = self.A, self.B, self.C
        Y = CSC(C.nrows, C.ncols, C.colptr, C.rowidx, dC_values)
        dB = masked_xty(A, Y, B, ws=self.ws_b, stream=stream)
        dCT = permute(dC_values, self.permC, False, stream=stream)
        YT = CSC(self.CT.nrows, self.CT.ncols, self.CT.colptr, self.CT.rowidx, dCT)
        dAT = masked_xty(self.BT, YT, self.AT, ws=self.ws_a, stream=stream)
        dA = permute(dAT, self.permA, True, stream=stream)
        return dA, dB

    def check(self, stream=None):
        for w in (self.ws_tr, self.ws_b, self.ws_a):
            check_ws(w, "device-side check (backward)", stream)


class SpGEMMFn(torch.autograd.Function):
    """C.values = (A B).values as a function of A's and B's stored values;
    C's pattern (colptr, rowidx) is returned as non-differentiable outputs.

        c_vals, c_colptr, c_rowidx = SpGEMMFn.apply(a_vals, b_vals, A, B)

    A and B give the patterns (their own values are ignored)."""

    @staticmethod
    def forward(ctx, a_vals, b_vals, A, B, layers=1, budget_bytes=None):
        Av = CSC(A.nrows, A.ncols, A.colptr, A.rowidx, a_vals)
        Bv = CSC(B.nrows, B.ncols, B.colptr, B.rowidx, b_vals)
        C, _ = Engine(Av, Bv, layers, budget_bytes).run()
        ctx.save_for_backward(a_vals, b_vals)
        ctx.A, ctx.B, ctx.C = A, B, CSC(C.nrows, C.ncols, C.colptr, C.rowidx, None)
        ctx.mark_non_differentiable(C.colptr, C.rowidx)
        return C.values, C.colptr, C.rowidx

    @staticmethod
    def backward(ctx, d_vals, _d_cp, _d_ri):
        a_vals, b_vals = ctx.saved_tensors
        A = CSC(ctx.A.nrows, ctx.A.ncols, ctx.A.colptr, ctx.A.rowidx, a_vals)
        B = CSC(ctx.B.nrows, ctx.B.ncols, ctx.B.colptr, ctx.B.rowidx, b_vals)
        bw = Backward(A, B, ctx.C)
        dA, dB = bw(d_vals.contiguous())
        bw.check()
        return dA, dB, None, None, None, None
