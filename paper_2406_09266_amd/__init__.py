"""Symmetric sparse tensor kernels on AMD Instinct MI355X (gfx950).

A thin Python binding over the C ABI of libsystec.so (include/systec.h).
Torch tensors supply device memory and the current HIP stream; the binding
only marshals arguments. Every step of the computation runs in the library's
HIP kernels; nothing here computes.

    import paper_2406_09266_amd as systec
    y = systec.ssymv(rowptr, col, val, x)          # y = A x, A symmetric (upper CSR)
    s = systec.syprd(rowptr, col, val, x)          # x^T A x (FP64 device scalar)
    C = systec.mttkrp([i1, i2, i3], val, B)        # symmetric MTTKRP, order 3..5

Symmetric operands are given by their canonical entries (ascending indices,
the upper triangle for a matrix), as in SySTeC (arXiv 2406.09266, Sec. 2.1).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import SYSTEC_BF16, SYSTEC_F32, SystecError, call, ptr_array

__all__ = [
    "SystecError", "ssymv", "syprd", "bellman_ford", "mttkrp", "ttm", "mttkrp_partial", "spmv_csr", "mttkrp_full", "expand_csr",
    "expand_coo", "expansion_stats", "validate_csr_upper", "validate_coo",
    "canonicalize_coo", "quantize_bf16", "KernelTimer", "version", "Tensor", "Server",
]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return SYSTEC_F32
    if t.dtype == torch.bfloat16:
        return SYSTEC_BF16
    raise TypeError(f"vector/factor dtype must be float32 or bfloat16, got {t.dtype}")


def _dev(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def version():
    return _lib.lib().systec_version().decode()


# ---------------------------------------------------------------- SSYMV ----

def ssymv(rowptr, col, val, x, out=None, stream=None):
    """y = A x, A symmetric given by its upper-triangle CSR (int32 rowptr/col,
    float32 val). x is float32 or bfloat16; y is float32."""
    torch = _torch()
    n = rowptr.numel() - 1
    _dev(rowptr, torch.int32, "rowptr"), _dev(col, torch.int32, "col")
    _dev(val, torch.float32, "val"), _dev(x, None, "x")
    if x.numel() != n:
        raise ValueError("x must have n elements")
    y = out if out is not None else torch.empty(n, dtype=torch.float32, device=x.device)
    _dev(y, torch.float32, "out")
    call("systec_ssymv", n, col.numel(), _p(rowptr), _p(col), _p(val), _p(x), _dtype_code(x),
         _p(y), _stream(stream))
    return y


def spmv_csr(rowptr, col, val, x, out=None, stream=None):
    """y = A x for a general (full) CSR matrix: the comparison kernel."""
    torch = _torch()
    n = rowptr.numel() - 1
    y = out if out is not None else torch.empty(n, dtype=torch.float32, device=x.device)
    call("systec_spmv_csr", n, col.numel(), _p(rowptr), _p(col), _p(val), _p(x),
         _dtype_code(x), _p(y), _stream(stream))
    return y


def syprd(rowptr, col, val, x, out=None, stream=None):
    """x^T A x (A symmetric, upper-triangle CSR) as a float64 device scalar."""
    torch = _torch()
    n = rowptr.numel() - 1
    s = out if out is not None else torch.empty(1, dtype=torch.float64, device=x.device)
    call("systec_syprd", n, col.numel(), _p(rowptr), _p(col), _p(val), _p(x), _dtype_code(x),
         _p(s), _stream(stream))
    return s


def bellman_ford(rowptr, col, val, d, out=None, stream=None):
    """y[i] = min_j (A[i,j] + d[j]) over the stored coordinates of the
    symmetric matrix A (upper-triangle CSR; float32 edge lengths and
    distances); +inf where row i stores nothing."""
    torch = _torch()
    n = rowptr.numel() - 1
    _dev(rowptr, torch.int32, "rowptr"), _dev(col, torch.int32, "col")
    _dev(val, torch.float32, "val"), _dev(d, torch.float32, "d")
    if d.numel() != n:
        raise ValueError("d must have n elements")
    y = out if out is not None else torch.empty(n, dtype=torch.float32, device=d.device)
    _dev(y, torch.float32, "out")
    call("systec_bellman_ford", n, col.numel(), _p(rowptr), _p(col), _p(val), _p(d), _p(y),
         _stream(stream))
    return y


# --------------------------------------------------------------- MTTKRP ----

def _idx_ptrs(idx, name="idx"):
    torch = _torch()
    for t in idx:
        _dev(t, torch.int32, name)
    return ptr_array([t.data_ptr() for t in idx])


MTTKRP_ALGOS = {"auto": 0, "atomic": 1, "lds": 2, "views": 3}


def _algo(name):
    if name not in MTTKRP_ALGOS:
        raise ValueError(f"algo must be one of {sorted(MTTKRP_ALGOS)}")
    return MTTKRP_ALGOS[name]


def mttkrp_choose(I, R, bf16, prepared):
    """Name of the algorithm "auto" runs for this shape ("atomic" for the
    one-shot call, "views" or "lds" for a prepared tensor)."""
    code = ctypes.c_int32(0)
    call("systec_mttkrp_choose", I, 1 if bf16 else 0, R, 1 if prepared else 0,
         ctypes.byref(code))
    return {v: k for k, v in MTTKRP_ALGOS.items()}[code.value]


def mttkrp(idx, val, B, out=None, stream=None, algo="auto"):
    """Symmetric MTTKRP: idx is a list of `order` (3..5) int32 index tensors of
    canonical COO (each tuple ascending, list sorted), val float32, B (I x R)
    float32 or bfloat16. Returns C (I x R) float32. algo: "auto" or "atomic"
    (the other algorithms need a prepared tensor, see Tensor.mttkrp)."""
    torch = _torch()
    order = len(idx)
    I, R = B.shape
    _dev(B, None, "B"), _dev(val, torch.float32, "val")
    if any(t.numel() != val.numel() for t in idx):
        raise ValueError("index arrays and values must have the same length")
    C = out if out is not None else torch.empty((I, R), dtype=torch.float32, device=B.device)
    _dev(C, torch.float32, "out")
    if tuple(C.shape) != (I, R):
        raise ValueError("out must be I x R")
    pp, keep = _idx_ptrs(idx)
    call("systec_mttkrp_ex", order, I, val.numel(), pp, _p(val), _p(B), _dtype_code(B), R, _p(C),
         _algo(algo), _stream(stream))
    del keep
    return C


def ttm(idx, val, B, out=None, mirror=True, stream=None):
    """TTM of a fully symmetric 3-index tensor (canonical COO: three int32
    index tensors, float32 val) with B (I x R, float32 or bfloat16):
    C[j, l, r] = sum_k T[k, j, l] B[k, r], an I x I x R float32 tensor,
    symmetric in (j, l). The canonical half j <= l is computed; mirror=False
    leaves the other half unwritten."""
    torch = _torch()
    if len(idx) != 3:
        raise ValueError("ttm needs a 3-index tensor")
    I, R = B.shape
    _dev(B, None, "B"), _dev(val, torch.float32, "val")
    C = out if out is not None else torch.empty((I, I, R), dtype=torch.float32, device=B.device)
    _dev(C, torch.float32, "out")
    if tuple(C.shape) != (I, I, R):
        raise ValueError("out must be I x I x R")
    pp, keep = _idx_ptrs(idx)
    call("systec_ttm", I, val.numel(), pp, _p(val), _p(B), _dtype_code(B), R, _p(C),
         1 if mirror else 0, _stream(stream))
    del keep
    return C


def mttkrp_partial(parts, idx, val, F, out=None, stream=None):
    """MTTKRP (output mode 1) of a tensor symmetric only inside consecutive
    parts of its slots: parts lists the part sizes (e.g. [2, 2]), idx the
    canonical COO (indices ascending inside each part), F one I x R factor
    per part (float32 or bfloat16, all of one dtype)."""
    import numpy as np
    torch = _torch()
    order = len(idx)
    if sum(parts) != order or len(F) != len(parts):
        raise ValueError("parts must sum to the order and give one factor per part")
    I, R = F[0].shape
    for f in F:
        _dev(f, F[0].dtype, "F")
        if tuple(f.shape) != (I, R):
            raise ValueError("every factor must be I x R")
    _dev(val, torch.float32, "val")
    C = out if out is not None else torch.empty((I, R), dtype=torch.float32, device=val.device)
    _dev(C, torch.float32, "out")
    sizes = np.ascontiguousarray(parts, dtype=np.int32)
    pp, keep = _idx_ptrs(idx)
    fp, fkeep = ptr_array([f.data_ptr() for f in F])
    call("systec_mttkrp_partial", order, len(parts), ctypes.c_void_p(sizes.ctypes.data), I,
         val.numel(), pp, _p(val), fp, _dtype_code(F[0]), R, _p(C), _stream(stream))
    del keep, fkeep
    return C


def mttkrp_full(idx, val, B, out=None, stream=None):
    """MTTKRP over listed (non-symmetric) entries grouped by idx[0]: the
    comparison kernel over an expanded tensor."""
    torch = _torch()
    order = len(idx)
    I, R = B.shape
    C = out if out is not None else torch.empty((I, R), dtype=torch.float32, device=B.device)
    pp, keep = _idx_ptrs(idx)
    call("systec_mttkrp_full", order, I, val.numel(), pp, _p(val), _p(B), _dtype_code(B), R,
         _p(C), _stream(stream))
    del keep
    return C


# ------------------------------------------------------------ expansion ----

def expand_csr(rowptr, col, val, stream=None):
    """Full CSR of A = U + U^T - diag(U) (setup for the comparison kernel)."""
    torch = _torch()
    n = rowptr.numel() - 1
    full = ctypes.c_int64()
    call("systec_expand_csr_size", n, col.numel(), _p(rowptr), _p(col), ctypes.byref(full),
         _stream(stream))
    frp = torch.empty(n + 1, dtype=torch.int32, device=rowptr.device)
    fcol = torch.empty(max(1, full.value), dtype=torch.int32, device=rowptr.device)
    fval = torch.empty(max(1, full.value), dtype=torch.float32, device=rowptr.device)
    call("systec_expand_csr", n, col.numel(), _p(rowptr), _p(col), _p(val), _p(frp), _p(fcol),
         _p(fval), _stream(stream))
    return frp, fcol[: full.value], fval[: full.value]


def expand_coo(idx, val, I, stream=None):
    """Every distinct permutation of every canonical entry, grouped by the
    first index (setup for the comparison kernel)."""
    torch = _torch()
    order = len(idx)
    pp, keep = _idx_ptrs(idx)
    full = ctypes.c_int64()
    call("systec_expand_coo_size", order, I, val.numel(), pp, ctypes.byref(full), _stream(stream))
    dev = val.device
    out = [torch.empty(max(1, full.value), dtype=torch.int32, device=dev) for _ in range(order)]
    oval = torch.empty(max(1, full.value), dtype=torch.float32, device=dev)
    op, okeep = ptr_array([t.data_ptr() for t in out])
    call("systec_expand_coo", order, I, val.numel(), pp, _p(val), op, _p(oval), _stream(stream))
    del keep, okeep
    return [t[: full.value] for t in out], oval[: full.value]


def expansion_stats(idx, I, stream=None):
    """(hist over equality patterns, effective nnz) computed on the device."""
    order = len(idx)
    pp, keep = _idx_ptrs(idx)
    hist = (ctypes.c_int64 * 16)()
    eff = ctypes.c_int64()
    n = idx[0].numel()
    call("systec_expansion_stats", order, I, n, pp, ctypes.cast(hist, _lib.PI64),
         ctypes.byref(eff), _stream(stream))
    del keep
    return [int(hist[m]) for m in range(1 << (order - 1))], int(eff.value)


# ----------------------------------------------------------- validation ----

def validate_csr_upper(rowptr, col, stream=None):
    """Raises SystecError (SYSTEC_ENONCANON) unless the CSR is a canonical upper triangle."""
    call("systec_validate_csr_upper", rowptr.numel() - 1, col.numel(), _p(rowptr), _p(col),
         _stream(stream))


def validate_coo(idx, I, stream=None):
    """Raises SystecError (SYSTEC_ENONCANON) unless the COO is canonical."""
    pp, keep = _idx_ptrs(idx)
    call("systec_validate_coo", len(idx), I, idx[0].numel(), pp, _stream(stream))
    del keep


def canonicalize_coo(idx, val):
    """Host helper: sort each tuple, sort the list, sum duplicates (numpy
    int32 index arrays and a float64 value array, modified in place).
    Returns the new length."""
    import numpy as np
    order = len(idx)
    for a in idx:
        if a.dtype != np.int32 or not a.flags.c_contiguous:
            raise TypeError("index arrays must be contiguous int32")
    if val.dtype != np.float64 or not val.flags.c_contiguous:
        raise TypeError("val must be contiguous float64")
    pp, keep = ptr_array([a.ctypes.data for a in idx])
    out = ctypes.c_int64()
    call("systec_canonicalize_coo", order, val.size, pp, ctypes.c_void_p(val.ctypes.data),
         ctypes.byref(out))
    del keep
    return int(out.value)


def quantize_bf16(x, out=None, stream=None):
    """FP32 -> BF16 (round to nearest even) on the device."""
    torch = _torch()
    _dev(x, torch.float32, "x")
    y = out if out is not None else torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    call("systec_quantize_bf16", _p(x), _p(y), x.numel(), _stream(stream))
    return y


class Tensor:
    """A prepared symmetric operand (library-owned device copy, rearranged
    once so that every output update is a segmented reduction).

        A = Tensor.from_csr(rowptr, col, val)     # upper-triangle CSR
        y = A.ssymv(x)
        T = Tensor.from_coo([i1, i2, i3], val, I)  # canonical COO, order 3..5
        C = T.mttkrp(B)
    """

    def __init__(self, handle):
        self._h = handle
        order, dim, nnz, eff, nbytes = (ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(),
                                        ctypes.c_int64(), ctypes.c_uint64())
        call("systec_tensor_info", self._h, ctypes.byref(order), ctypes.byref(dim),
             ctypes.byref(nnz), ctypes.byref(eff), ctypes.byref(nbytes))
        self.order, self.dim, self.nnz = order.value, dim.value, nnz.value
        self.effective_nnz, self.bytes = eff.value, nbytes.value

    @classmethod
    def from_csr(cls, rowptr, col, val, stream=None, relabel=False):
        """relabel: True stores the matrix with its vertices ordered by degree
        (each ssymv then permutes x in and y out; faster on power-law
        graphs), False keeps the order, None lets the library decide from the
        degree skew. A Server serves a relabeled matrix with two more
        n-element vectors per request (counted against its budget)."""
        torch = _torch()
        _dev(rowptr, torch.int32, "rowptr"), _dev(col, torch.int32, "col")
        _dev(val, torch.float32, "val")
        h = ctypes.c_void_p()
        code = -1 if relabel is None else (1 if relabel else 0)
        call("systec_tensor_create_csr_ex", rowptr.numel() - 1, col.numel(), _p(rowptr), _p(col),
             _p(val), code, _stream(stream), ctypes.byref(h))
        return cls(h)

    def vertex_order(self, stream=None):
        """None if the matrix is stored in the caller's vertex order, else
        perm (int32 on the device): perm[i] is the caller's vertex stored at
        position i."""
        torch = _torch()
        rel = ctypes.c_int()
        call("systec_tensor_vertex_order", self._h, ctypes.byref(rel), None, _stream(stream))
        if not rel.value:
            return None
        perm = torch.empty(self.dim, dtype=torch.int32, device="cuda")
        call("systec_tensor_vertex_order", self._h, None, _p(perm), _stream(stream))
        return perm

    @classmethod
    def from_coo(cls, idx, val, I, stream=None):
        torch = _torch()
        _dev(val, torch.float32, "val")
        pp, keep = _idx_ptrs(idx)
        h = ctypes.c_void_p()
        call("systec_tensor_create_coo", len(idx), I, val.numel(), pp, _p(val), _stream(stream),
             ctypes.byref(h))
        del keep
        return cls(h)

    def ssymv(self, x, out=None, stream=None, stored_order=False):
        """y = A x. stored_order: x and y are in the order the matrix is
        stored in (see vertex_order), so no permutation runs."""
        torch = _torch()
        _dev(x, None, "x")
        if self.order != 2 or x.numel() != self.dim or (out is not None and out.numel() != self.dim):
            raise ValueError("ssymv needs a prepared matrix and x, y of n elements")
        y = out if out is not None else torch.empty(self.dim, dtype=torch.float32, device=x.device)
        call("systec_ssymv_t_ex", self._h, _p(x), _dtype_code(x), _p(y), 1 if stored_order else 0,
             _stream(stream))
        return y

    def syprd(self, x, out=None, stream=None, stored_order=False):
        """x^T A x of the prepared matrix as a float64 device scalar
        (stored_order as for ssymv)."""
        torch = _torch()
        _dev(x, None, "x")
        if self.order != 2 or x.numel() != self.dim:
            raise ValueError("syprd needs a prepared matrix and x of n elements")
        s = out if out is not None else torch.empty(1, dtype=torch.float64, device=x.device)
        call("systec_syprd_t_ex", self._h, _p(x), _dtype_code(x), _p(s), 1 if stored_order else 0,
             _stream(stream))
        return s

    def bellman_ford(self, d, out=None, stream=None):
        """y[i] = min_j (A[i,j] + d[j]) for the prepared matrix (float32 d)."""
        torch = _torch()
        _dev(d, torch.float32, "d")
        if self.order != 2 or d.numel() != self.dim:
            raise ValueError("bellman_ford needs a prepared matrix and d of n elements")
        y = out if out is not None else torch.empty(self.dim, dtype=torch.float32, device=d.device)
        _dev(y, torch.float32, "out")
        call("systec_bellman_ford_t", self._h, _p(d), _p(y), _stream(stream))
        return y

    def mttkrp(self, B, out=None, stream=None, algo="auto"):
        """C = MTTKRP of the prepared tensor; algo: "auto", "views" (slot
        views), "lds" (slot views with B staged in LDS; small index spaces;
        the automatic choice where all of B fits) or "atomic" (the canonical
        list with device atomics)."""
        torch = _torch()
        _dev(B, None, "B")
        I, R = B.shape
        if I != self.dim or self.order < 3:
            raise ValueError("B must have one row per tensor index")
        C = out if out is not None else torch.empty((I, R), dtype=torch.float32, device=B.device)
        _dev(C, torch.float32, "out")
        if tuple(C.shape) != (I, R):
            raise ValueError("out must be I x R")
        call("systec_mttkrp_t_ex", self._h, _p(B), _dtype_code(B), R, _p(C), _algo(algo),
             _stream(stream))
        return C

    def cp_step(self, B, stream=None):
        """One symmetric CP-ALS step around this tensor's MTTKRP: returns
        (B_new, C, G, fit) with C = MTTKRP(T, B), G = B^T B, B_new = C
        (G^(N-1))^-1 and fit a float64 device tensor of ||T||^2,
        <T,[[B]]>, ||[[B]]||^2 and ||T - [[B]]||^2."""
        torch = _torch()
        _dev(B, None, "B")
        I, R = B.shape
        if I != self.dim or self.order < 3:
            raise ValueError("B must have one row per tensor index")
        C = torch.empty((I, R), dtype=torch.float32, device=B.device)
        B_new = torch.empty((I, R), dtype=torch.float32, device=B.device)
        G = torch.empty((R, R), dtype=torch.float32, device=B.device)
        fit = torch.empty(4, dtype=torch.float64, device=B.device)
        call("systec_cp_step", self._h, _p(B), _dtype_code(B), R, _p(C), _p(B_new), _p(G),
             _p(fit), _stream(stream))
        return B_new, C, G, fit

    def close(self):
        if self._h is not None and self._h.value:
            _lib.lib().systec_tensor_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over prepared operands resident in HBM.

        srv = Server(budget_bytes=200 << 30, max_slots=16)
        tid = srv.register(Tensor.from_csr(rowptr, col, val))   # ownership moves
        req = srv.submit(tid, x, y)        # y = A x, asynchronous
        srv.wait(req)
        srv.stats()                        # p50/p99 latency, throughput

    Input and output buffers are kept alive by the server object until the
    request has completed (wait() or poll() saw it finish)."""

    QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, budget_bytes=200 << 30, max_slots=32, step_work_nnz=1 << 27, device=None,
                 max_queue=0, max_inflight=0, streams=0, min_step_work_nnz=0):
        """step_work_nnz: entries per step; larger steps raise throughput
        (2^27 measured best at saturation on a mixed workload), smaller ones
        lower the latency of small requests that share steps with large ones.
        max_inflight: steps queued on the device at once (0: the default, 2).
        streams: 1 runs the kernel kinds of a step one after another on one
        stream; 0 gives each kind its own stream.
        min_step_work_nnz: step budget with one running request, growing
        linearly to step_work_nnz with max_slots running (0: fixed steps)."""
        torch = _torch()
        cfg = _lib.ServeConfig(budget_bytes, max_slots, step_work_nnz,
                               torch.cuda.current_device() if device is None else device,
                               max_queue, max_inflight, streams, min_step_work_nnz)
        self._h = ctypes.c_void_p()
        call("systec_serve_create", ctypes.byref(cfg), ctypes.byref(self._h))
        self._live = {}
        self._kind = {}

    @staticmethod
    def now_ns():
        return int(_lib.lib().systec_serve_now_ns())

    def register(self, tensor):
        tid = ctypes.c_int64()
        call("systec_serve_register", self._h, tensor._h, ctypes.byref(tid))
        tensor._h = None  # owned by the server now
        self._kind[tid.value] = (tensor.order, tensor.dim, tensor.effective_nnz)
        return tid.value

    def submit(self, tensor_id, inp, out, arrival_ns=0, stream=None):
        """Queues out = A inp (or C = MTTKRP(T, B)). The request's work on the
        device starts after the work enqueued so far on `stream` (default:
        the current stream), which wrote inp or last used out."""
        torch = _torch()
        _dev(inp, None, "input"), _dev(out, torch.float32, "output")
        R = 1 if inp.dim() == 1 else inp.shape[1]
        order, dim, _ = self._kind.get(tensor_id, (None, None, None))
        if order == 2:
            if inp.numel() != dim or out.numel() != dim:
                raise ValueError("x and y must have n elements")
        elif order is not None:
            if inp.dim() != 2 or inp.shape[0] != dim or tuple(out.shape) != (dim, R):
                raise ValueError("B must be I x R and C I x R")
        rid = ctypes.c_int64()
        call("systec_serve_submit_after", self._h, tensor_id, _p(inp), _dtype_code(inp), R,
             _p(out), int(arrival_ns), _stream(stream), ctypes.byref(rid))
        self._live[rid.value] = (inp, out)
        return rid.value

    def poll(self, req):
        st = ctypes.c_int()
        call("systec_serve_poll", self._h, req, ctypes.byref(st))
        if st.value in (self.DONE, self.FAILED):
            self._live.pop(req, None)
        return st.value

    def wait(self, req, timeout_us=-1):
        try:
            call("systec_serve_wait", self._h, req, int(timeout_us))
        except SystecError as e:
            if e.status_name != "SYSTEC_ETIMEOUT":
                self._live.pop(req, None)
            raise
        self._live.pop(req, None)

    def stats(self):
        st = _lib.ServeStats()
        call("systec_serve_get_stats", self._h, ctypes.byref(st))
        return {name: getattr(st, name) for name, _ in st._fields_}

    def reset_stats(self):
        call("systec_serve_reset_stats", self._h)

    def close(self):
        if self._h is not None and self._h.value:
            _lib.lib().systec_serve_destroy(self._h)
        self._h = None
        self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KernelTimer:
    """Times the library's hot-kernel launches with HIP events on their own
    stream:  with KernelTimer() as kt: ...;  kt.total_ms, kt.launches."""

    def __enter__(self):
        call("systec_kernel_timing", 1)
        self.read()  # discard anything recorded before
        return self

    def read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        call("systec_kernel_timing_read", ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    def __exit__(self, *exc):
        self.total_ms, self.launches = self.read()
        call("systec_kernel_timing", 0)
        return False
