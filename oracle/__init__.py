"""CPU oracle for the sparse TT decomposition: test infrastructure only.

A plain, single-threaded FP64 C++ implementation written from the paper
(arXiv 1908.02721).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP path; the product library never loads it.

Parity status per function (see the pins in ``tests/test_oracle_*.py``):
  decompose (sparse stage)  -- pinned: literal pairwise Deparallelisation with exact
                               integer arithmetic, closed forms (rank-1, disjoint
                               sums, diagonal, single entry), exact reconstruction.
  decompose (rounding)      -- pinned: dense TT-SVD ranks and spectra computed with
                               LAPACK on tiny tensors, error bound, Pythagorean
                               error identity, orthonormality, known QTT ranks of
                               the 2D Laplacian, FDM matrix ranks printed in the paper.
  decompose (dynamic delta) -- pinned: a worked case with closed-form singular
                               values, dense TT-SVD with the same thresholds, the
                               bound of Algorithm 8's correctness theorem.
  decompose (key_bits)      -- pinned: the rounding equals NumPy's binary32 and
                               binary16 conversions at 23 and 10 bits; snapped
                               grouping of noisy parallel columns equals the exact
                               grouping of the noise-free tensor; per-entry error
                               bound of the reconstruction.
  matrix_coords (MPO)       -- pinned: dense reshape/transpose of tiny matrices,
                               the quantized Laplacian and FDM layouts built from
                               grid coordinates, MPO matrix-vector products.
  eval / eval_grad          -- pinned: dense reconstruction, rank-1 closed form,
                               central finite differences.
  tt_diff_norm              -- pinned: dense subtraction on tiny tensors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ttoracle.cpp")
# TTORACLE_LIB names another build of the same source (the sanitizer test loads an
# ASan/UBSan build this way); the default is the in-tree library built by build().
_LIB = os.environ.get("TTORACLE_LIB") or os.path.join(_HERE, "libttoracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "OK", 1: "ARG", 2: "INDEX", 3: "DUPLICATE", 4: "NONFINITE", 5: "EMPTY", 6: "TOO_LARGE"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code} ({STATUS.get(code, '?')})")
        self.code = code
        self.name = STATUS.get(code, "?")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, single-threaded, strict IEEE)."""
    if os.environ.get("TTORACLE_LIB"):
        return _LIB  # a prebuilt variant (see above): never rebuilt here
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", _LIB, _SRC]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            i32, i64, f64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
            lib.orc_decompose.argtypes = [i32, P(i64), i64, P(ctypes.c_int32), P(f64), f64, i32, i32, i32, i32, P(vp)]
            lib.orc_snap.argtypes = [P(f64), i64, i32, P(f64)]
            lib.orc_decompose.restype = ctypes.c_int
            lib.orc_free.argtypes = [vp]
            lib.orc_summary.argtypes = [vp, P(i64), P(f64), P(f64)]
            lib.orc_times.argtypes = [vp, P(f64)]
            lib.orc_level_sizes.argtypes = [vp, i32, P(i64)]
            lib.orc_level.argtypes = [vp, i32, P(i64), P(i32), P(f64), P(i64), P(i64), P(f64)]
            lib.orc_last_exact.argtypes = [vp, P(f64)]
            lib.orc_ranks.argtypes = [vp, P(i64)]
            lib.orc_qr_ranks.argtypes = [vp, P(i64)]
            lib.orc_core.argtypes = [vp, i32, P(f64)]
            lib.orc_sigma_count.argtypes = [vp, i32]
            lib.orc_sigma_count.restype = i64
            lib.orc_sigma.argtypes = [vp, i32, P(f64), P(f64)]
            lib.orc_bond_delta.argtypes = [vp, i32]
            lib.orc_bond_delta.restype = f64
            lib.orc_eval.argtypes = [i32, P(i64), P(i64), P(P(f64)), i64, P(i32), P(f64)]
            lib.orc_eval.restype = ctypes.c_int
            lib.orc_eval_grad.argtypes = [i32, P(i64), P(i64), P(P(f64)), i64, P(i32), P(f64), P(P(f64))]
            lib.orc_eval_grad.restype = ctypes.c_int
            lib.orc_tt_diff_norm.argtypes = [i32, P(i64), P(i64), P(P(f64)), P(i64), P(P(f64))]
            lib.orc_tt_diff_norm.restype = f64
            _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class Level:
    col: np.ndarray      # int64 row-major suffix index per column (row-major column order)
    g: np.ndarray        # int32 group per column
    s: np.ndarray        # float64 prefactor per column
    beta: int
    n_colptr: np.ndarray
    n_row: np.ndarray
    n_val: np.ndarray


@dataclass
class OracleResult:
    dims: tuple
    nnz: int
    norm: float
    delta: float
    levels: list = field(default_factory=list)       # levels[k-1], k = 1..d-1
    last_exact: np.ndarray = None                     # beta_{d-1} x n_d
    ranks: list = None
    qr_ranks: list = None
    cores: list = None                                # dense [r_{k-1}, n_k, r_k]
    sigma: list = None                                # sigma[b-1]
    tail: list = None
    bond_delta: list = None                           # threshold used at bond b-1
    times: tuple = None

    @property
    def betas(self):
        return [1] + [L.beta for L in self.levels] + [1]

    def exact_cores(self):
        """Dense cores of the exact TT from the sparse stage."""
        d = len(self.dims)
        b = self.betas
        cores = []
        for k in range(1, d):
            L = self.levels[k - 1]
            G = np.zeros((b[k - 1] * self.dims[k - 1], b[k]))
            for c in range(L.beta):
                for e in range(L.n_colptr[c], L.n_colptr[c + 1]):
                    G[L.n_row[e], c] = L.n_val[e]
            cores.append(G.reshape(b[k - 1], self.dims[k - 1], b[k]))
        cores.append(self.last_exact.reshape(b[d - 1], self.dims[d - 1], 1))
        return cores


def decompose(idx, val, dims, eps, max_rank: int = 0, do_round: bool = True,
              dynamic_delta: bool = False, key_bits: int = 0) -> OracleResult:
    lib = _load()
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    d = len(dims)
    dims_a = np.asarray(dims, dtype=np.int64)
    nnz = val.shape[0]
    if idx.size != nnz * d:
        raise ValueError("idx must be [nnz, d]")
    h = ctypes.c_void_p()
    st = lib.orc_decompose(d, _p(dims_a, ctypes.c_int64), nnz, _p(idx, ctypes.c_int32), _p(val, ctypes.c_double),
                           float(eps), int(max_rank), int(bool(do_round)), int(bool(dynamic_delta)), int(key_bits),
                           ctypes.byref(h))
    if st != 0:
        raise OracleError(st)
    try:
        info = np.zeros(2, dtype=np.int64)
        nrm = ctypes.c_double()
        dl = ctypes.c_double()
        lib.orc_summary(h, _p(info, ctypes.c_int64), ctypes.byref(nrm), ctypes.byref(dl))
        t4 = np.zeros(4)
        lib.orc_times(h, _p(t4, ctypes.c_double))
        res = OracleResult(dims=tuple(int(x) for x in dims), nnz=int(info[0]), norm=nrm.value, delta=dl.value,
                           times=tuple(t4))
        for k in range(1, d):
            sz = np.zeros(3, dtype=np.int64)
            lib.orc_level_sizes(h, k, _p(sz, ctypes.c_int64))
            ncol, beta, nn = (int(x) for x in sz)
            col = np.zeros(ncol, dtype=np.int64)
            g = np.zeros(ncol, dtype=np.int32)
            s = np.zeros(ncol)
            cp = np.zeros(beta + 1, dtype=np.int64)
            rw = np.zeros(nn, dtype=np.int64)
            vl = np.zeros(nn)
            lib.orc_level(h, k, _p(col, ctypes.c_int64), _p(g, ctypes.c_int32), _p(s, ctypes.c_double),
                          _p(cp, ctypes.c_int64), _p(rw, ctypes.c_int64), _p(vl, ctypes.c_double))
            res.levels.append(Level(col, g, s, beta, cp, rw, vl))
        res.last_exact = np.zeros(res.levels[-1].beta * dims[-1])
        lib.orc_last_exact(h, _p(res.last_exact, ctypes.c_double))
        if info[1]:
            rk = np.zeros(d + 1, dtype=np.int64)
            lib.orc_ranks(h, _p(rk, ctypes.c_int64))
            res.ranks = [int(x) for x in rk]
            lib.orc_qr_ranks(h, _p(rk, ctypes.c_int64))
            res.qr_ranks = [int(x) for x in rk]
            res.cores = []
            for k in range(1, d + 1):
                c = np.zeros(res.ranks[k - 1] * dims[k - 1] * res.ranks[k])
                lib.orc_core(h, k, _p(c, ctypes.c_double))
                res.cores.append(c.reshape(res.ranks[k - 1], dims[k - 1], res.ranks[k]))
            res.sigma, res.tail = [], []
            res.bond_delta = [lib.orc_bond_delta(h, b) for b in range(1, d)]
            for b in range(1, d):
                cnt = lib.orc_sigma_count(h, b)
                sg = np.zeros(cnt)
                tl = ctypes.c_double()
                lib.orc_sigma(h, b, _p(sg, ctypes.c_double), ctypes.byref(tl))
                res.sigma.append(sg)
                res.tail.append(tl.value)
        return res
    finally:
        lib.orc_free(h)


def _core_ptrs(cores):
    arrs = [np.ascontiguousarray(c, dtype=np.float64) for c in cores]
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_p(a, ctypes.c_double) for a in arrs])
    return arrs, ptrs


def _ranks_of(cores):
    return np.asarray([c.shape[0] for c in cores] + [cores[-1].shape[2]], dtype=np.int64)


def eval_entries(cores, idx) -> np.ndarray:
    """TT entries at coordinates idx [m, d] (FP64)."""
    lib = _load()
    d = len(cores)
    dims = np.asarray([c.shape[1] for c in cores], dtype=np.int64)
    ranks = _ranks_of(cores)
    arrs, ptrs = _core_ptrs(cores)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, d)
    y = np.zeros(idx.shape[0])
    st = lib.orc_eval(d, _p(dims, ctypes.c_int64), _p(ranks, ctypes.c_int64), ptrs, idx.shape[0],
                      _p(idx, ctypes.c_int32), _p(y, ctypes.c_double))
    if st != 0:
        raise OracleError(st)
    return y


def eval_grad(cores, idx, gy) -> list:
    """Gradient of sum_n gy[n] * TT(idx_n) with respect to every core (FP64)."""
    lib = _load()
    d = len(cores)
    dims = np.asarray([c.shape[1] for c in cores], dtype=np.int64)
    ranks = _ranks_of(cores)
    arrs, ptrs = _core_ptrs(cores)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, d)
    gy = np.ascontiguousarray(gy, dtype=np.float64)
    grads = [np.zeros_like(a) for a in arrs]
    gptrs = (ctypes.POINTER(ctypes.c_double) * d)(*[_p(g, ctypes.c_double) for g in grads])
    st = lib.orc_eval_grad(d, _p(dims, ctypes.c_int64), _p(ranks, ctypes.c_int64), ptrs, idx.shape[0],
                           _p(idx, ctypes.c_int32), _p(gy, ctypes.c_double), gptrs)
    if st != 0:
        raise OracleError(st)
    return grads


def tt_diff_norm(cores_a, cores_b) -> float:
    """||A - B||_F of two TTs with equal mode sizes (stable: TT sum + QR sweep)."""
    lib = _load()
    d = len(cores_a)
    dims = np.asarray([c.shape[1] for c in cores_a], dtype=np.int64)
    ra, rb = _ranks_of(cores_a), _ranks_of(cores_b)
    aa, pa = _core_ptrs(cores_a)
    ab, pb = _core_ptrs(cores_b)
    return float(lib.orc_tt_diff_norm(d, _p(dims, ctypes.c_int64), _p(ra, ctypes.c_int64), pa,
                                      _p(rb, ctypes.c_int64), pb))


def matrix_coords(rows, cols, row_dims, col_dims) -> np.ndarray:
    """Tensor coordinates of matrix entries (matrix in TT format, Sec. 3.4).

    The M x N matrix, M = m_1...m_d, N = n_1...n_d, is the tensor of order 2d with
    indices (i_1, j_1, ..., i_d, j_d): (i_k) are the digits of the row index in the
    radix (m_1..m_d), (j_k) those of the column index in (n_1..n_d), first digit most
    significant.  Mode k of the d-way tensor merges (i_k, j_k) into i_k n_k + j_k.
    Returns int32 [nnz, d]; raises IndexError for an index outside the matrix.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    m = [int(x) for x in row_dims]
    n = [int(x) for x in col_dims]
    M = int(np.prod(np.array(m, dtype=object)))
    N = int(np.prod(np.array(n, dtype=object)))
    if rows.size and (rows.min() < 0 or int(rows.max()) >= M or cols.min() < 0 or int(cols.max()) >= N):
        raise IndexError("row or column index outside the matrix")
    d = len(m)
    out = np.empty((rows.size, d), dtype=np.int64)
    # digits from the least significant (mode d) to the most significant (mode 1)
    I = rows.astype(object) if M >= 2 ** 62 else rows.copy()
    J = cols.astype(object) if N >= 2 ** 62 else cols.copy()
    for k in range(d - 1, -1, -1):
        ik, I = I % m[k], I // m[k]
        jk, J = J % n[k], J // n[k]
        out[:, k] = np.asarray(ik, dtype=np.int64) * n[k] + np.asarray(jk, dtype=np.int64)
    return out.astype(np.int32)


def snap(x, key_bits: int) -> np.ndarray:
    """The oracle's rounding of canonical values to key_bits fraction bits."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib.orc_snap(_p(x, ctypes.c_double), x.size, int(key_bits), _p(out, ctypes.c_double))
    return out


@dataclass
class KnifeEdge:
    """How far each bond's rank decision sits from flipping (rank rule of Alg 2, Sec. 2.4).

    margin_rel[b]: min over r of |tail_r - delta^2| / ||A||_F^2, tail_r the sum of the
                   squared singular values beyond r; a rank decision that rounding could
                   flip has this near the unit roundoff.
    kept_over_delta[b]: the smallest kept singular value over delta (inf for rank 0).
    dropped_over_delta[b]: the largest discarded singular value over delta (0 if none).
    """
    margin_rel: list
    kept_over_delta: list
    dropped_over_delta: list


def knife_edge(res: OracleResult) -> KnifeEdge:
    """Distances of the oracle's rank decisions from the truncation threshold.

    Uses only the singular values each bond met and the threshold it used, so the
    same report can be made for any result carrying those (the GPU path's too).
    """
    margins, kept, dropped = [], [], []
    norm2 = res.norm * res.norm
    for b, sig in enumerate(res.sigma):
        delta = res.bond_delta[b]
        s = np.asarray(sig, dtype=np.float64)
        tails = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])  # tails[r] = sum_{i>=r} s_i^2
        margins.append(float(np.min(np.abs(tails[1:] - delta * delta))) / norm2)
        r = res.ranks[b + 1]
        kept.append(float(s[r - 1] / delta) if r >= 1 and delta > 0 else float("inf"))
        dropped.append(float(s[r] / delta) if r < len(s) and delta > 0 else 0.0)
    return KnifeEdge(margins, kept, dropped)
