"""CPU oracle for the bond-2 Gram slice of the left-to-right QR sweep: test infrastructure only.

Plain NumPy, FP64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; it shares no code with the HIP path.

The slice is the start of TT-rounding's orthogonalisation sweep (Alg 2, Sec. 2.4,
run left to right) on the exact sparse TT of the parallel-vector rounding, carried
as far as one device can when the second bond is too wide to factor:

  * bond 1: X_1 = unfold_2(G^(1)) (n_1 x beta_1; r_0 = 1) = Q_1 R_1, an economic
    QR with m = min(#nonzero rows, beta_1).  A wide X_1 of full row rank leaves Q_1
    free up to an orthogonal factor, so the slice fixes the gauge by the SVD:
    Q_1 = the first m left singular vectors (singular values non-ascending, the
    entry of largest magnitude of each column positive, lowest index on ties) and
    R_1 = Q_1^T X_1 (= Sigma V^T).  core 1 := Q_1; R_1 moves into core 2.
  * the contraction X_2 = unfold_2(R_1 x_1 G^(2)) ((m n_2) x beta_2): with N_2's
    entries (rho = g n_2 + i, column j, value c),
        X_2[(a, i), j] = sum over entries of column j with rho mod n_2 = i of
                         c * R_1[a, rho div n_2].
  * the right-part weights w_2: the rows of the right part P_2 (beta_2 x n_3...n_d,
    the product of the exact cores 3..d) are mutually orthogonal in the exact TT
    (each transfer-matrix column has one nonzero), with squared norms
        w_{d-1}[g] = sum_i G^(d)[g, i]^2,
        w_k[g]     = sum over entries (rho, b, c) of N_{k+1} with rho div n_{k+1} = g
                     of c^2 w_{k+1}[b].
  * the weighted Gram Gamma = X_2 diag(w_2) X_2^T.  Up to the orthogonal Q_1 (x) I it
    is the Gram matrix of the bond-2 unfolding of A, so its eigenvalues are that
    unfolding's squared singular values and its trace is ||A||_F^2.  Rows and columns
    are indexed slot-major, q = i * m + a (i = i_2, a = the bond-1 index).

Parity status: pinned (tests/test_oracle_slice.py) by dense reshapes and matrix
products of the exact TT on small tensors (X_1, X_2, P_2), orthonormality and the
gauge of Q_1, the eigenvalues of Gamma against LAPACK singular values of the dense
bond-2 unfolding of A, and trace(Gamma) = ||A||_F^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Bond1:
    Q1: np.ndarray       # n_1 x m, orthonormal columns (SVD gauge)
    R1: np.ndarray       # m x beta_1
    sigma: np.ndarray    # m singular values of X_1, non-ascending
    X1: np.ndarray       # n_1 x beta_1 (the exact core 1 unfolded)


def _csc_dense(L, nrows):
    """Dense nrows x beta matrix of a level's N_k (CSC)."""
    M = np.zeros((nrows, L.beta))
    cols = np.repeat(np.arange(L.beta), np.diff(L.n_colptr))
    M[np.asarray(L.n_row, dtype=np.int64), cols] = L.n_val
    return M


def bond1_qr(res) -> Bond1:
    """Economic QR of X_1 in the SVD gauge (module docstring).  res: oracle.decompose(..., do_round=False)."""
    n1 = res.dims[0]
    X1 = _csc_dense(res.levels[0], n1)
    U, s, _ = np.linalg.svd(X1, full_matrices=False)
    m = min(int(np.count_nonzero(np.any(X1 != 0.0, axis=1))), X1.shape[1])
    Q1 = U[:, :m].copy()
    for j in range(m):
        p = int(np.argmax(np.abs(Q1[:, j])))  # first index of the largest magnitude
        if Q1[p, j] < 0.0:
            Q1[:, j] = -Q1[:, j]
    R1 = Q1.T @ X1
    return Bond1(Q1=Q1, R1=R1, sigma=s[:m].copy(), X1=X1)


def right_weights(res, k: int) -> np.ndarray:
    """w_k (length beta_k), the squared row norms of the right part of bond k (1 <= k <= d-1)."""
    d = len(res.dims)
    G = np.asarray(res.last_exact).reshape(res.levels[d - 2].beta, res.dims[d - 1])
    w = np.sum(G * G, axis=1)
    for lev in range(d - 2, k - 1, -1):  # N_{lev+1} = res.levels[lev]
        L = res.levels[lev]
        nk = res.dims[lev]
        cols = np.repeat(np.arange(L.beta), np.diff(L.n_colptr))
        g = np.asarray(L.n_row, dtype=np.int64) // nk
        wn = np.zeros(res.levels[lev - 1].beta)
        np.add.at(wn, g, L.n_val * L.n_val * w[cols])
        w = wn
    return w


class Slice:
    """X_2 and the weighted Gram of bond 2, evaluated at requested positions.

    Entries of N_2 are grouped by slot i = rho mod n_2 and, within a slot, by column j,
    so that a row (a, i) of X_2 is available as values over the slot's columns.
    """

    def __init__(self, res, b1: Bond1 | None = None):
        if len(res.dims) < 3:
            raise ValueError("the bond-2 slice needs d >= 3")
        self.res = res
        self.b1 = b1 if b1 is not None else bond1_qr(res)
        self.n2 = res.dims[1]
        self.m = self.b1.R1.shape[0]
        L2 = res.levels[1]
        self.beta2 = L2.beta
        col = np.repeat(np.arange(L2.beta), np.diff(L2.n_colptr))
        rho = np.asarray(L2.n_row, dtype=np.int64)
        slot = rho % self.n2
        g = rho // self.n2
        order = np.lexsort((col, slot))      # slot-major, then column
        self.e_slot = slot[order]
        self.e_col = col[order]
        self.e_g = g[order]
        self.e_c = np.asarray(L2.n_val)[order]
        self.slot_start = np.searchsorted(self.e_slot, np.arange(self.n2 + 1))
        self.w2 = right_weights(res, 2)
        self._cols = {}

    def _slot_cols(self, i):
        """Distinct columns of slot i (ascending) and the entry-run starts for reduceat."""
        if i not in self._cols:
            lo, hi = self.slot_start[i], self.slot_start[i + 1]
            c = self.e_col[lo:hi]
            starts = np.flatnonzero(np.concatenate([[True], c[1:] != c[:-1]])) if hi > lo else np.zeros(0, np.int64)
            self._cols[i] = (c[starts], starts)
        return self._cols[i]

    def row(self, a, i):
        """X_2[(a, i), j] over the slot's distinct columns j (ascending): (cols, values)."""
        lo, hi = self.slot_start[i], self.slot_start[i + 1]
        cols, starts = self._slot_cols(i)
        if hi == lo:
            return cols, np.zeros(0)
        v = self.e_c[lo:hi] * self.b1.R1[a, self.e_g[lo:hi]]
        return cols, np.add.reduceat(v, starts)

    def x2(self, a, i, j):
        """X_2[(a, i), j]."""
        cols, vals = self.row(int(a), int(i))
        p = np.searchsorted(cols, j)
        return float(vals[p]) if p < cols.size and cols[p] == j else 0.0

    def gram(self, q, q2):
        """Gamma[q, q2], q = i * m + a (slot-major)."""
        i, a = divmod(int(q), self.m)
        i2, a2 = divmod(int(q2), self.m)
        c1, v1 = self.row(a, i)
        c2, v2 = self.row(a2, i2)
        common, p1, p2 = np.intersect1d(c1, c2, assume_unique=True, return_indices=True)
        return float(np.sum(self.w2[common] * v1[p1] * v2[p2]))

    def dense_x2(self):
        """X_2 as a dense (n_2 m) x beta_2 array with slot-major rows q = i m + a (small sizes only)."""
        X = np.zeros((self.n2 * self.m, self.beta2))
        for i in range(self.n2):
            lo, hi = self.slot_start[i], self.slot_start[i + 1]
            if hi == lo:
                continue
            cols, starts = self._slot_cols(i)
            V = self.e_c[lo:hi, None] * self.b1.R1[:, self.e_g[lo:hi]].T
            X[i * self.m:(i + 1) * self.m, cols] = np.add.reduceat(V, starts, axis=0).T
        return X

    def dense_gram(self):
        """Gamma = X_2 diag(w_2) X_2^T, dense, slot-major (small sizes only)."""
        X = self.dense_x2()
        return (X * self.w2[None, :]) @ X.T

    def block_trace(self, i):
        """trace of the diagonal block (i, i) of Gamma: sum_a Gamma[(i, a), (i, a)]."""
        return float(sum(self.gram(i * self.m + a, i * self.m + a) for a in range(self.m)))

    def block_traces(self, chunk=200_000):
        """trace of every diagonal block (i, i) of Gamma, i.e. sum over the blocks (j, i)
        of X_2 of w_2[j] ||X_2[(:, i), j]||^2; their sum is trace(Gamma)."""
        # blocks (j, i) in column-major order; each block is the sum of its entries'
        # scaled columns of R_1
        order = np.lexsort((self.e_slot, self.e_col))
        col, slot, g, c = self.e_col[order], self.e_slot[order], self.e_g[order], self.e_c[order]
        n = col.size
        newblk = np.concatenate([[True], (col[1:] != col[:-1]) | (slot[1:] != slot[:-1])])
        out = np.zeros(self.n2)
        lo = 0
        while lo < n:
            hi = min(n, lo + chunk)
            while hi < n and not newblk[hi]:  # do not split a block between chunks
                hi += 1
            V = c[lo:hi, None] * self.b1.R1[:, g[lo:hi]].T
            starts = np.flatnonzero(newblk[lo:hi])
            B = np.add.reduceat(V, starts, axis=0)
            np.add.at(out, slot[lo:hi][starts], self.w2[col[lo:hi][starts]] * np.sum(B * B, axis=1))
            lo = hi
        return out

    def weighted_norm2(self, chunk=200_000):
        """sum_j w_2[j] ||X_2[:, j]||^2 (= trace(Gamma))."""
        return float(np.sum(self.block_traces(chunk)))
