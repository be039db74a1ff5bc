"""Sparse tensor-train decomposition on MI355X (gfx950): Python binding of libttsparse.

Method: arXiv 1908.02721, "Faster Tensor Train Decomposition for Sparse Data".
Every step runs in the library's HIP kernels; this module only marshals
arguments (PyTorch provides device memory and streams).

    tt = decompose(idx, val, dims, eps)          # idx int32 [nnz, d], val float64 [nnz] on cuda
    tt.ranks, tt.cores                            # cores [r_{k-1}, n_k, r_k]
    y = EvalEntries.apply(idx, *cores)            # TT entries at idx, differentiable
    mpo = decompose_matrix(rows, cols, val, row_dims, col_dims, eps)   # sparse matrix -> MPO
    mpo.mpo_cores()                               # [r_{k-1}, m_k, n_k, r_k]
    ftt = fasttt_decompose(idx, val, dims, eps, p=0)   # the paper's fiber-trie variant
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import STAGES, TTError

__all__ = ["decompose", "decompose_matrix", "matrix_to_tensor", "fasttt_decompose", "fasttt_select_p", "TT", "eval_entries", "eval_entries_backward",
           "EvalPlan", "EvalEntries", "TTError", "library_path"]

library_path = _lib.LIB_PATH


def _stream_handle(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _CAI:
    """A borrowed device buffer exposed through __cuda_array_interface__.  ``owner``
    (the result that holds the buffer) stays alive as long as this object, which a
    tensor made from it keeps."""

    def __init__(self, ptr: int, shape, typestr: str, owner=None):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(int(x) for x in shape),
                                         "typestr": typestr, "version": 2, "strides": None}
        self._owner = owner


_TYPESTR = {torch.float64: "<f8", torch.float32: "<f4", torch.int64: "<i8", torch.int32: "<i4"}


def _view_of_device(ptr: int, shape, dtype, owner) -> torch.Tensor:
    """Zero-copy torch view of a library-owned device buffer that keeps ``owner`` alive."""
    n = 1
    for x in shape:
        n *= int(x)
    if n == 0 or not ptr:
        return torch.empty(tuple(shape), dtype=dtype, device="cuda")
    return torch.as_tensor(_CAI(ptr, shape, _TYPESTR[dtype], owner), device="cuda")


def _copy_from_device(ptr: int, shape, dtype) -> torch.Tensor:
    """Owning torch copy of a library-owned device buffer."""
    n = 1
    for x in shape:
        n *= int(x)
    if n == 0 or not ptr:
        return torch.empty(tuple(shape), dtype=dtype, device="cuda")
    view = torch.as_tensor(_CAI(ptr, shape, _TYPESTR[dtype]), device="cuda")
    return view.clone()


class TT:
    """Result of ``decompose``: owns the library handle until garbage-collected."""

    def __init__(self, handle: ctypes.c_void_p, dims):
        self._h = handle
        self.dims = tuple(int(x) for x in dims)
        self.d = len(self.dims)
        L = _lib.load()
        r = (ctypes.c_int64 * (self.d + 1))()
        _lib.check(L.tt_get_ranks(self._h, r))
        self.ranks = [int(x) for x in r]
        info = (ctypes.c_int64 * 3)()
        nrm, dl = ctypes.c_double(), ctypes.c_double()
        _lib.check(L.tt_get_info(self._h, info, ctypes.byref(nrm), ctypes.byref(dl)))
        self.nnz, self.rounded = int(info[0]), bool(info[1])
        self.norm, self.delta = nrm.value, dl.value
        b = (ctypes.c_int64 * (self.d + 1))()
        q = (ctypes.c_int64 * (self.d + 1))()
        _lib.check(L.tt_get_sparse_ranks(self._h, b, q if self.rounded else None))
        self.betas = [int(x) for x in b]
        self.qr_ranks = [int(x) for x in q] if self.rounded else None
        t = (ctypes.c_double * _lib.NUM_STAGES)()
        _lib.check(L.tt_get_times(self._h, t))
        self.times_ms = dict(zip(STAGES, (float(x) for x in t)))
        self.row_dims = self.col_dims = None  # set for a matrix decomposed as an MPO

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().tt_free(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def cores(self):
        """The cores, [r_{k-1}, n_k, r_k] each: torch views of this result's device
        memory, made without a copy (ordered on the stream the decomposition ran on).
        Each view keeps the result alive; writing to one changes the result's core."""
        L = _lib.load()
        out = []
        for k in range(1, self.d + 1):
            p = ctypes.c_void_p()
            dt = ctypes.c_int32()
            _lib.check(L.tt_get_core(self._h, k, ctypes.byref(p), ctypes.byref(dt)))
            dtype = torch.float64 if dt.value == _lib.DTYPE_F64 else torch.float32
            shape = (self.ranks[k - 1], self.dims[k - 1], self.ranks[k])
            out.append(_view_of_device(p.value, shape, dtype, self))
        return out

    def sigma(self, b: int):
        """Singular values at bond b (1..d-1) and the discarded sum of squares."""
        L = _lib.load()
        cnt = ctypes.c_int64()
        ptr = ctypes.POINTER(ctypes.c_double)()
        tail = ctypes.c_double()
        _lib.check(L.tt_get_sigma(self._h, b, ctypes.byref(cnt), ctypes.byref(ptr), ctypes.byref(tail)))
        import numpy as np

        sig = np.ctypeslib.as_array(ptr, shape=(cnt.value,)).copy() if cnt.value else np.zeros(0)
        return sig, tail.value

    def mpo_cores(self):
        """Cores of a matrix decomposed by decompose_matrix, viewed as [r_{k-1}, m_k, n_k, r_k]."""
        if self.row_dims is None:
            raise ValueError("not a matrix decomposition (use decompose_matrix)")
        return [c.view(c.shape[0], m, n, c.shape[2]) for c, m, n in zip(self.cores, self.row_dims, self.col_dims)]

    def bond_delta(self, b: int) -> float:
        """Truncation threshold used at bond b (1..d-1)."""
        L = _lib.load()
        x = ctypes.c_double()
        _lib.check(L.tt_get_bond_delta(self._h, b, ctypes.byref(x)))
        return x.value

    def level_sizes(self):
        """Per level k = 1..d-1: (columns = nnz_{k+1}, beta_k, nnz(N_k))."""
        L = _lib.load()
        out = []
        for k in range(1, self.d):
            sz = (ctypes.c_int64 * 3)()
            _lib.check(L.tt_get_level_sizes(self._h, k, sz))
            out.append(tuple(int(x) for x in sz))
        return out

    def level(self, k: int):
        """Level k (1..d-1) of the sparse stage (needs keep_intermediates=True)."""
        L = _lib.load()
        ncols, beta = ctypes.c_int64(), ctypes.c_int64()
        ptrs = [ctypes.c_void_p() for _ in range(6)]
        _lib.check(L.tt_get_level(self._h, k, ctypes.byref(ncols), ctypes.byref(beta),
                                  *[ctypes.byref(p) for p in ptrs]))
        nc, bt = ncols.value, beta.value
        colptr = _copy_from_device(ptrs[3].value, (bt + 1,), torch.int64)
        nnz_n = int(colptr[-1].item()) if bt else 0
        return {
            "ncols": nc,
            "beta": bt,
            "col": _copy_from_device(ptrs[0].value, (nc,), torch.int64),
            "g": _copy_from_device(ptrs[1].value, (nc,), torch.int32),
            "s": _copy_from_device(ptrs[2].value, (nc,), torch.float64),
            "n_colptr": colptr,
            "n_row": _copy_from_device(ptrs[4].value, (nnz_n,), torch.int32),
            "n_val": _copy_from_device(ptrs[5].value, (nnz_n,), torch.float64),
        }


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def decompose(idx: torch.Tensor, val: torch.Tensor, dims, eps: float, precision: str = "fp64",
              max_rank: int = 0, keep_intermediates: bool = False, sparse_only: bool = False,
              device_mem_budget: int = 0, stream=None, allocator=None, dynamic_delta: bool = False,
              key_bits: int = 0) -> TT:
    """Sparse TT decomposition of the COO tensor (idx int32 [nnz, d], val float64 [nnz], on cuda).

    allocator: optional (alloc(nbytes) -> device pointer int, free(pointer int)) used for
    every device allocation of the call and of the result (the tt_options hooks); it
    must be ordered on `stream`, as torch's caching allocator is on the current stream.
    dynamic_delta: per-bond truncation thresholds from the remaining error budget
    (Algorithm 8) instead of eps ||A|| / sqrt(d-1) at every bond.
    key_bits: 0 for the exact parallel test; 1..52 rounds every canonical value to
    that many fraction bits before grouping (tolerant test for noisy parallel columns).
    """
    L = _lib.load()
    if not (idx.is_cuda and val.is_cuda):
        raise ValueError("idx and val must be cuda tensors")
    if idx.dtype != torch.int32 or val.dtype != torch.float64:
        raise TypeError("idx must be int32 and val float64")
    idx = idx.contiguous()
    val = val.contiguous()
    d = len(dims)
    nnz = int(val.numel())
    if idx.numel() != nnz * d:
        raise ValueError("idx must have shape [nnz, d]")
    opt = _lib.tt_options()
    L.tt_options_default(ctypes.byref(opt))
    opt.precision = _lib.PRECISION[precision]
    opt.max_rank = int(max_rank)
    opt.keep_intermediates = int(bool(keep_intermediates))
    opt.sparse_only = int(bool(sparse_only))
    opt.device_mem_budget = int(device_mem_budget)
    opt.dynamic_delta = int(bool(dynamic_delta))
    opt.key_bits = int(key_bits)
    hooks = None
    if allocator is not None:
        a_fn, f_fn = allocator
        hooks = (_ALLOC_T(lambda nbytes, ctx: int(a_fn(int(nbytes)) or 0)),
                 _FREE_T(lambda ptr, ctx: f_fn(int(ptr))))
        opt.alloc = ctypes.cast(hooks[0], ctypes.c_void_p)
        opt.free = ctypes.cast(hooks[1], ctypes.c_void_p)
    dims_a = (ctypes.c_int64 * d)(*[int(x) for x in dims])
    h = ctypes.c_void_p()
    st = L.tt_sparse_decompose(d, dims_a, nnz, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                               float(eps), ctypes.byref(opt), _stream_handle(stream), ctypes.byref(h))
    _lib.check(st)
    tt = TT(h, dims)
    tt._hooks = hooks  # the result frees through them in tt_free
    return tt


def _coo_args(idx, val, dims):
    if not (idx.is_cuda and val.is_cuda):
        raise ValueError("idx and val must be cuda tensors")
    if idx.dtype != torch.int32 or val.dtype != torch.float64:
        raise TypeError("idx must be int32 and val float64")
    idx = idx.contiguous()
    val = val.contiguous()
    d = len(dims)
    nnz = int(val.numel())
    if idx.numel() != nnz * d:
        raise ValueError("idx must have shape [nnz, d]")
    return idx, val, d, nnz, (ctypes.c_int64 * d)(*[int(x) for x in dims])


def fasttt_decompose(idx: torch.Tensor, val: torch.Tensor, dims, eps: float, p: int = 0, max_rank: int = 0,
                     sparse_only: bool = False, device_mem_budget: int = 0, stream=None,
                     dynamic_delta: bool = False, precision: str = "fp64") -> TT:
    """The paper's fiber-trie FastTT (Algorithm 7): exact TT of the nonzero p-fibers
    reduced by Algorithm 4, rounded from core p outwards (Algorithm 6).

    p = 0 chooses p by Algorithm 9.  The returned TT also has ``ftt_p`` (the p used)
    and ``fibers`` (R, the number of nonzero p-fibers); ``betas`` holds the exact
    ranks r~ of Algorithm 4.
    """
    L = _lib.load()
    idx, val, d, nnz, dims_a = _coo_args(idx, val, dims)
    opt = _lib.tt_options()
    L.tt_options_default(ctypes.byref(opt))
    opt.max_rank = int(max_rank)
    opt.sparse_only = int(bool(sparse_only))
    opt.device_mem_budget = int(device_mem_budget)
    opt.dynamic_delta = int(bool(dynamic_delta))
    opt.precision = _lib.PRECISION[precision]
    h = ctypes.c_void_p()
    _lib.check(L.tt_fasttt_decompose(d, dims_a, nnz, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                     float(eps), int(p), ctypes.byref(opt), _stream_handle(stream), ctypes.byref(h)))
    tt = TT(h, dims)
    pp, R = ctypes.c_int32(), ctypes.c_int64()
    _lib.check(L.tt_get_fasttt_info(h, ctypes.byref(pp), ctypes.byref(R)))
    tt.ftt_p, tt.fibers = int(pp.value), int(R.value)
    return tt


class GramSlice(TT):
    """Result of ``gram_slice``: the bond-2 Gram slice of the QR sweep (tt_sparse_gram_slice).

    Attributes: m (bond-1 rank), sigma1 (singular values of X_1, numpy), nblocks,
    npairs, wnorm2 (= trace of the Gram), gram_flops (algorithmic FP64 flops of the
    Gram), slice_ms (stage times).  q1() and r1() return owning copies; x2_view()
    and gram_view() return views of library memory, valid while this object lives.
    """

    def __init__(self, handle: ctypes.c_void_p, dims):
        super().__init__(handle, dims)
        import numpy as np

        L = _lib.load()
        m = ctypes.c_int64()
        q1, r1 = ctypes.c_void_p(), ctypes.c_void_p()
        sg = ctypes.POINTER(ctypes.c_double)()
        _lib.check(L.tt_get_slice_bond1(self._h, ctypes.byref(m), ctypes.byref(q1), ctypes.byref(r1), ctypes.byref(sg)))
        self.m = int(m.value)
        self._q1, self._r1 = q1.value, r1.value
        self.sigma1 = np.ctypeslib.as_array(sg, shape=(self.m,)).copy()
        nb = ctypes.c_int64()
        sp, bc, xv = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        dt = ctypes.c_int32()
        _lib.check(L.tt_get_slice_x2(self._h, ctypes.byref(nb), ctypes.byref(sp), ctypes.byref(bc), ctypes.byref(xv),
                                     ctypes.byref(dt)))
        self.nblocks = int(nb.value)
        self._slot_ptr, self._blk_col, self._x2 = sp.value, bc.value, xv.value
        self.x2_dtype = torch.float64 if dt.value == _lib.DTYPE_F64 else torch.float32
        g = ctypes.c_void_p()
        wn, fl = ctypes.c_double(), ctypes.c_double()
        npairs = ctypes.c_int64()
        ms = (ctypes.c_double * 5)()
        _lib.check(L.tt_get_slice_gram(self._h, ctypes.byref(g), ctypes.byref(wn), ctypes.byref(npairs),
                                       ctypes.byref(fl), ms))
        self._gram = g.value
        self.wnorm2, self.gram_flops, self.npairs = wn.value, fl.value, int(npairs.value)
        self.slice_ms = dict(zip(("bond1_qr", "x2", "pairs", "gram", "slice"), (float(x) for x in ms)))
        self.n2 = self.dims[1]

    def q1(self) -> torch.Tensor:
        """Q_1 as an owning [n_1, m] tensor."""
        return _copy_from_device(self._q1, (self.m, self.dims[0]), torch.float64).T

    def r1(self) -> torch.Tensor:
        """R_1 as an owning [m, beta_1] tensor."""
        return _copy_from_device(self._r1, (self.betas[1], self.m), torch.float64).T

    def slot_ptr(self) -> torch.Tensor:
        return _copy_from_device(self._slot_ptr, (self.n2 + 1,), torch.int64)

    def blk_col(self) -> torch.Tensor:
        return _copy_from_device(self._blk_col, (self.nblocks,), torch.int32)

    def x2_view(self) -> torch.Tensor:
        """The X_2 blocks [nblocks, m] (slot-major), a view of library memory."""
        return torch.as_tensor(_CAI(self._x2, (self.nblocks, self.m), _TYPESTR[self.x2_dtype]), device="cuda")

    def gram_view(self) -> torch.Tensor:
        """The packed upper blocks of the Gram (1-D), a view of library memory."""
        n = self.n2 * (self.n2 + 1) // 2 * self.m * self.m
        return torch.as_tensor(_CAI(self._gram, (n,), "<f8"), device="cuda")

    def gram_offset(self, q, q2):
        """Element offsets in gram_view() of Gamma[q, q2] (q = i m + a; arrays or ints, i <= i2 after swap)."""
        import numpy as np

        q = np.asarray(q, dtype=np.int64)
        q2 = np.asarray(q2, dtype=np.int64)
        lo, hi = np.minimum(q, q2), np.maximum(q, q2)
        swap = (q // self.m) > (q2 // self.m)
        a_row = np.where(swap, q2, q)
        a_col = np.where(swap, q, q2)
        i, a = a_row // self.m, a_row % self.m
        i2, a2 = a_col // self.m, a_col % self.m
        blk = i * self.n2 - i * (i - 1) // 2 + (i2 - i)
        del lo, hi
        return blk * self.m * self.m + a * self.m + a2


def gram_slice(idx: torch.Tensor, val: torch.Tensor, dims, precision: str = "fp64", keep_intermediates: bool = False,
               key_bits: int = 0, device_mem_budget: int = 0, stream=None) -> GramSlice:
    """Bond-2 Gram slice of the QR sweep (tt_sparse_gram_slice): bond-1 QR in the SVD
    gauge, X_2 = R_1 x_1 G^(2) (block-sparse, in the precision's operands) and the
    weighted FP64 Gram of bond 2."""
    L = _lib.load()
    idx, val, d, nnz, dims_a = _coo_args(idx, val, dims)
    opt = _lib.tt_options()
    L.tt_options_default(ctypes.byref(opt))
    opt.precision = _lib.PRECISION[precision]
    opt.keep_intermediates = int(bool(keep_intermediates))
    opt.key_bits = int(key_bits)
    opt.device_mem_budget = int(device_mem_budget)
    h = ctypes.c_void_p()
    _lib.check(L.tt_sparse_gram_slice(d, dims_a, nnz, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                      ctypes.byref(opt), _stream_handle(stream), ctypes.byref(h)))
    return GramSlice(h, dims)


def cache_trim() -> int:
    """Wait for the device and free every device block the library keeps cached; bytes freed."""
    L = _lib.load()
    b = ctypes.c_uint64()
    _lib.check(L.tt_cache_trim(ctypes.byref(b)))
    return int(b.value)


def fasttt_select_p(idx: torch.Tensor, val: torch.Tensor, dims, stream=None):
    """Algorithm 9: (p, estimated cost of every p = 1..d)."""
    L = _lib.load()
    idx, val, d, nnz, dims_a = _coo_args(idx, val, dims)
    costs = (ctypes.c_double * d)()
    pp = ctypes.c_int32()
    _lib.check(L.tt_fasttt_select_p(d, dims_a, nnz, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                    costs, ctypes.byref(pp), _stream_handle(stream)))
    return int(pp.value), [float(x) for x in costs]


def matrix_to_tensor(rows: torch.Tensor, cols: torch.Tensor, row_dims, col_dims, stream=None) -> torch.Tensor:
    """Tensor coordinates of matrix entries for the MPO front-end (tt_matrix_to_tensor).

    rows, cols: int64 [nnz] on cuda.  Returns int32 [nnz, d] with mode k index
    i_k * n_k + j_k, where (i_k) and (j_k) are the mixed-radix digits of the row
    and column index in (m_1..m_d) and (n_1..n_d), first digit most significant.
    """
    L = _lib.load()
    if not (rows.is_cuda and cols.is_cuda):
        raise ValueError("rows and cols must be cuda tensors")
    if rows.dtype != torch.int64 or cols.dtype != torch.int64:
        raise TypeError("rows and cols must be int64")
    rows = rows.contiguous()
    cols = cols.contiguous()
    d = len(row_dims)
    if len(col_dims) != d:
        raise ValueError("row_dims and col_dims must have the same length")
    nnz = int(rows.numel())
    if int(cols.numel()) != nnz:
        raise ValueError("rows and cols must have the same length")
    idx = torch.empty((nnz, d), dtype=torch.int32, device=rows.device)
    ra = (ctypes.c_int64 * d)(*[int(x) for x in row_dims])
    ca = (ctypes.c_int64 * d)(*[int(x) for x in col_dims])
    _lib.check(L.tt_matrix_to_tensor(d, ra, ca, nnz, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
                                     ctypes.c_void_p(idx.data_ptr()), _stream_handle(stream)))
    return idx


def decompose_matrix(rows: torch.Tensor, cols: torch.Tensor, val: torch.Tensor, row_dims, col_dims, eps: float,
                     stream=None, method: str = "cps", **kw) -> TT:
    """Matrix in TT format (MPO) of a sparse M x N matrix, M = prod(row_dims), N = prod(col_dims).

    The matrix becomes the tensor with modes m_k * n_k (matrix_to_tensor), which is
    decomposed by ``decompose`` (method "cps") or by the fiber-trie ``fasttt_decompose``
    (method "fasttt"), with that function's options; ``TT.mpo_cores()`` gives the
    cores as [r_{k-1}, m_k, n_k, r_k].
    """
    idx = matrix_to_tensor(rows, cols, row_dims, col_dims, stream=stream)
    dims = [int(m) * int(n) for m, n in zip(row_dims, col_dims)]
    if method == "fasttt":
        tt = fasttt_decompose(idx, val, dims, eps, stream=stream, **kw)
    elif method == "cps":
        tt = decompose(idx, val, dims, eps, stream=stream, **kw)
    else:
        raise ValueError("method must be 'cps' or 'fasttt'")
    tt.row_dims = tuple(int(x) for x in row_dims)
    tt.col_dims = tuple(int(x) for x in col_dims)
    return tt


def _core_args(cores):
    d = len(cores)
    dims = (ctypes.c_int64 * d)(*[int(c.shape[1]) for c in cores])
    ranks = (ctypes.c_int64 * (d + 1))(*([int(c.shape[0]) for c in cores] + [int(cores[-1].shape[2])]))
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    return d, dims, ranks, ptrs


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.DTYPE_F64
    if t.dtype == torch.float32:
        return _lib.DTYPE_F32
    raise TypeError("cores must be float32 or float64")


def eval_entries(cores, idx: torch.Tensor, stream=None) -> torch.Tensor:
    """y[n] = G1[0, i1, :] G2[:, i2, :] ... Gd[:, id, 0] for idx int32 [m, d] (cuda)."""
    L = _lib.load()
    cores = [c.contiguous() for c in cores]
    dt = _dtype_code(cores[0])
    if any(c.dtype != cores[0].dtype for c in cores):
        raise TypeError("all cores must share one dtype")
    idx = idx.contiguous()
    m = idx.shape[0]
    y = torch.empty(m, dtype=cores[0].dtype, device=cores[0].device)
    d, dims, ranks, ptrs = _core_args(cores)
    _lib.check(L.tt_eval_entries(d, dims, ranks, ptrs, dt, m, ctypes.c_void_p(idx.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), _stream_handle(stream)))
    return y


def eval_entries_backward(cores, idx: torch.Tensor, grad_y: torch.Tensor, stream=None):
    """Gradients of sum_n grad_y[n] * y_n with respect to every core."""
    L = _lib.load()
    cores = [c.contiguous() for c in cores]
    dt = _dtype_code(cores[0])
    idx = idx.contiguous()
    grad_y = grad_y.contiguous().to(cores[0].dtype)
    grads = [torch.empty_like(c) for c in cores]
    d, dims, ranks, ptrs = _core_args(cores)
    gptrs = (ctypes.c_void_p * d)(*[g.data_ptr() for g in grads])
    _lib.check(L.tt_eval_entries_backward(d, dims, ranks, ptrs, dt, idx.shape[0], ctypes.c_void_p(idx.data_ptr()),
                                          ctypes.c_void_p(grad_y.data_ptr()), gptrs, _stream_handle(stream)))
    return grads


class EvalPlan:
    """Sorted coordinates and their prefix trie, built once for idx int32 [m, d] (cuda).

    forward(cores, save=False) -> y; backward(cores, grad_y, use_saved=False) -> grads.
    With save, the forward keeps its left partial products; a backward with
    use_saved reuses them (same ranks and dtype, unchanged core values).
    """

    def __init__(self, idx: torch.Tensor, dims, stream=None):
        L = _lib.load()
        idx = idx.contiguous()
        if idx.dtype != torch.int32 or idx.dim() != 2:
            raise TypeError("idx must be an int32 [m, d] tensor")
        self.dims = [int(n) for n in dims]
        self.m = int(idx.shape[0])
        self.device = idx.device
        d = len(self.dims)
        a = (ctypes.c_int64 * d)(*self.dims)
        h = ctypes.c_void_p()
        _lib.check(L.tt_eval_plan_create(d, a, self.m, ctypes.c_void_p(idx.data_ptr()), _stream_handle(stream),
                                         ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().tt_eval_plan_free(h)
            except Exception:
                pass
            self._h = None

    def _cores(self, cores):
        cores = [c.contiguous() for c in cores]
        if [int(c.shape[1]) for c in cores] != self.dims:
            raise ValueError("core mode sizes differ from the plan's dims")
        if any(c.dtype != cores[0].dtype for c in cores):
            raise TypeError("all cores must share one dtype")
        return cores

    def forward(self, cores, save: bool = False, stream=None) -> torch.Tensor:
        L = _lib.load()
        cores = self._cores(cores)
        dt = _dtype_code(cores[0])
        y = torch.empty(self.m, dtype=cores[0].dtype, device=cores[0].device)
        _, _, ranks, ptrs = _core_args(cores)
        _lib.check(L.tt_eval_plan_forward(self._h, ranks, ptrs, dt, ctypes.c_void_p(y.data_ptr()), int(bool(save)),
                                          _stream_handle(stream)))
        return y

    def backward(self, cores, grad_y: torch.Tensor, use_saved: bool = False, stream=None):
        L = _lib.load()
        cores = self._cores(cores)
        dt = _dtype_code(cores[0])
        grad_y = grad_y.contiguous().to(cores[0].dtype)
        grads = [torch.empty_like(c) for c in cores]
        d, _, ranks, ptrs = _core_args(cores)
        gptrs = (ctypes.c_void_p * d)(*[g.data_ptr() for g in grads])
        _lib.check(L.tt_eval_plan_backward(self._h, ranks, ptrs, dt, ctypes.c_void_p(grad_y.data_ptr()), gptrs,
                                           int(bool(use_saved)), _stream_handle(stream)))
        return grads


class EvalEntries(torch.autograd.Function):
    """Differentiable sampled-entry evaluation: EvalEntries.apply(idx, *cores) -> y.

    The forward builds an EvalPlan and keeps its left partial products; the backward
    reuses both.  The cores are saved for backward, so autograd rejects an in-place
    change of them in between.
    """

    @staticmethod
    def forward(ctx, idx, *cores):
        plan = EvalPlan(idx, [int(c.shape[1]) for c in cores])
        y = plan.forward(cores, save=True)
        ctx.plan = plan
        ctx.save_for_backward(*cores)
        return y

    @staticmethod
    def backward(ctx, grad_y):
        cores = ctx.saved_tensors
        grads = ctx.plan.backward(cores, grad_y, use_saved=True)
        return (None, *grads)
