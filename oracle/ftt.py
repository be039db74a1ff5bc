"""CPU oracle for the fiber-trie FastTT (Algorithms 4-7 and 9): test infrastructure only.

Plain NumPy, FP64.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; it shares no code with the HIP path.

What it computes (0-based modes; p is 1-based as in the paper):

  * exact_tt(idx, val, dims, p) -- Algorithm 4 with Algorithm 5 as Depar.  The rank-R
    TT of the nonzero p-fibers (Theorem on the rank-R TT) is reduced by
    Deparallelisation of quasi-permutation matrices from the left edge up to core p
    and from the right edge down to core p.  For a quasi-permutation matrix Algorithm 5
    keeps each nonzero row once, numbered by increasing row index, so:
      - for k < p, the bond-k index of a fiber is the rank of its prefix (i_1..i_k)
        among the distinct prefixes of the fibers, in lexicographic order (the row of
        spl_2(G^(k)) is (prefix id of i_1..i_{k-1}) * n_k + i_k);
        G^(k)[a, i, b] = 1 when prefix b extends prefix a by i;
      - for k > p, the bond-(k-1) index is the rank of the suffix (i_k..i_d) among the
        distinct suffixes, lexicographic with i_k most significant (the row of
        spl_1^T(G^(k)) is i_k * r_k + (suffix id of i_{k+1}..i_d));
        G^(k)[a, i, b] = 1 when suffix a is i followed by suffix b;
      - the middle core holds the values: G^(p)[prefix id, i_p, suffix id] = a_i.
  * round_tt(cores, p, eps, norm, max_rank, dynamic) -- Algorithm 6: a delta-truncated
    SVD sweep from core p to the right, a QR sweep back to core p, and a
    delta-truncated SVD sweep from core p to the left, delta = eps ||A||_F /
    (sqrt(p-1) + sqrt(d-p)) (the static thresholds).  With dynamic, Algorithm 8: the
    budgets delta_right = sqrt(d-p)/(sqrt(d-p)+sqrt(p-1)) eps ||A||_F and delta_left
    = sqrt(p-1)/(...) eps ||A||_F; bond k of the first sweep gets
    delta_right/sqrt(d-k), bond k-1 of the second delta_left/sqrt(k-1), and each
    budget then loses the bond's discarded sum of sigma^2.  rank_delta = the smallest
    r >= 1 whose discarded sum of sigma^2 is <= delta^2; fixed-rank truncation keeps
    min(max_rank, #nonzero sigma).
  * flop_estimate / select_p -- the cost model of the complexity analysis (Sec. 3.6)
    with f_SVD(m, n) = m n min(m, n) and the rank bounds of Algorithm 4 (the upper
    bounds r_bar), and Algorithm 9: the p of least estimated cost (lowest p on ties).

Parity status: pinned (tests/test_oracle_ftt.py) by exact reconstruction of dense
tiny tensors, the rank bounds, orthonormality of the indicator cores (corollary on
left/right orthonormality), the paper's FDM numbers R and r~ (Table 2), dense
TT-SVD ranks at eps -> 0, the error bound of Algorithm 6's correctness theorem,
the paper's worked FLOP examples, and for Algorithm 8 its correctness theorem, the
per-sweep budget invariants and dense TT-SVD ranks with the same thresholds at p = d.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FttExact:
    cores: list          # dense [r_{k-1}, n_k, r_k]
    ranks: list          # r~_0..r~_d
    R: int               # number of nonzero p-fibers
    norm: float


@dataclass
class FttResult:
    cores: list
    ranks: list
    exact_ranks: list
    R: int
    p: int
    norm: float
    delta: float
    sigma: list          # sigma[b-1] at bond b, sorted non-ascending
    tail: list           # discarded sum of sigma^2 at bond b
    bond_delta: list = None  # threshold used at bond b


def _validate(idx, val, dims):
    idx = np.asarray(idx, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    d = len(dims)
    if idx.ndim != 2 or idx.shape[1] != d or idx.shape[0] != val.size:
        raise ValueError("idx must be [nnz, d] with one value per row")
    if np.any(idx < 0) or np.any(idx >= np.asarray(dims, dtype=np.int64)[None, :]):
        raise IndexError("index out of range")
    if not np.all(np.isfinite(val)):
        raise ValueError("non-finite value")
    keep = val != 0.0
    idx, val = idx[keep], val[keep]
    if idx.shape[0] == 0:
        raise ValueError("no nonzero")
    if np.unique(idx, axis=0).shape[0] != idx.shape[0]:
        raise ValueError("duplicate coordinate")
    return idx, val


def _rank_ids(keys):
    """Rank of each row of `keys` among the distinct rows, lexicographic (column 0 first)."""
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    return inv.reshape(-1), uniq.shape[0]


def exact_tt(idx, val, dims, p: int) -> FttExact:
    idx, val = _validate(idx, val, dims)
    d = len(dims)
    if not 1 <= p <= d:
        raise ValueError("p must be in 1..d")
    nnz = idx.shape[0]
    ranks = [1] * (d + 1)
    # prefix ids per entry, k = 1..p-1 (the entries' prefixes are the fibers' prefixes)
    pid = [np.zeros(nnz, dtype=np.int64)]
    for k in range(1, p):
        ids, cnt = _rank_ids(idx[:, :k])
        pid.append(ids)
        ranks[k] = cnt
    # suffix ids per entry, k = d..p+1 (sid[k] indexes the suffix (i_k..i_d), 1-based k)
    sid = {d + 1: np.zeros(nnz, dtype=np.int64)}
    for k in range(d, p, -1):
        ids, cnt = _rank_ids(idx[:, k - 1:])
        sid[k] = ids
        ranks[k - 1] = cnt
    cores = []
    for k in range(1, d + 1):
        G = np.zeros((ranks[k - 1], dims[k - 1], ranks[k]))
        i = idx[:, k - 1]
        if k < p:
            G[pid[k - 1], i, pid[k]] = 1.0
        elif k > p:
            G[sid[k], i, sid[k + 1]] = 1.0
        else:
            G[pid[p - 1], i, sid[p + 1]] = val
        cores.append(G)
    # nonzero p-fibers: distinct (i_1..i_{p-1}, i_{p+1}..i_d)
    rest = np.delete(idx, p - 1, axis=1)
    R = np.unique(rest, axis=0).shape[0] if rest.shape[1] else 1
    return FttExact(cores=cores, ranks=ranks, R=int(R), norm=float(np.sqrt(np.sum(val * val))))


def _rank_rule(s, delta, max_rank):
    if max_rank > 0:
        return max(1, min(int(max_rank), int(np.sum(s > 0))))
    tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
    return next(r for r in range(1, s.size + 1) if tail[r] <= delta * delta)


def _sign_fix(U, VS):
    """Entry of largest magnitude of each kept left singular vector made positive."""
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] *= -1
            VS[:, j] *= -1
    return U, VS


def round_tt(cores, p: int, eps: float, norm: float, max_rank: int = 0, dynamic: bool = False):
    """Algorithm 6 (Algorithm 8 with dynamic) on dense cores;
    returns (cores, ranks, sigma, tail, delta, bond_delta)."""
    G = [c.copy() for c in cores]
    d = len(G)
    den = np.sqrt(p - 1) + np.sqrt(d - p)
    delta = eps * norm / den if d > 1 else 0.0
    right2 = (np.sqrt(d - p) / den * eps * norm) ** 2   # delta_right^2
    left2 = (np.sqrt(p - 1) / den * eps * norm) ** 2    # delta_left^2
    sigma = [None] * (d - 1)
    tail = [0.0] * (d - 1)
    bond_delta = [delta] * (d - 1)
    # first SVD sweep: k = p..d-1, G = spl_2(G^(k)) = U S V^T, core k := U, G^(k+1) := (S V^T) G^(k+1)
    for k in range(p, d):
        r0, n, r1 = G[k - 1].shape
        M = G[k - 1].reshape(r0 * n, r1)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        dk = np.sqrt(right2 / (d - k)) if dynamic else delta
        bond_delta[k - 1] = dk
        r = _rank_rule(s, dk, max_rank)
        sigma[k - 1] = s
        tail[k - 1] = float(np.sum(s[r:] ** 2))
        right2 = max(0.0, right2 - tail[k - 1])
        Uk = U[:, :r].copy()
        VS = (Vt[:r].T * s[:r]).copy()
        Uk, VS = _sign_fix(Uk, VS)
        G[k - 1] = Uk.reshape(r0, n, r)
        G[k] = np.tensordot(VS.T, G[k], axes=([1], [0]))
    # QR sweep: k = d..p+1, spl_1^T(G^(k)) = Q R, core k := Q^T, G^(k-1) := G^(k-1) x_3 R^T
    for k in range(d, p, -1):
        r0, n, r1 = G[k - 1].shape
        M = G[k - 1].reshape(r0, n * r1).T
        Q, Rm = np.linalg.qr(M, mode="reduced")
        G[k - 1] = Q.T.reshape(Q.shape[1], n, r1)
        G[k - 2] = np.tensordot(G[k - 2], Rm.T, axes=([2], [0]))
    # second SVD sweep: k = p..2, spl_1^T(G^(k)) = U S V^T, core k := U^T, G^(k-1) := G^(k-1) x_3 (V S)
    for k in range(p, 1, -1):
        r0, n, r1 = G[k - 1].shape
        M = G[k - 1].reshape(r0, n * r1).T
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        dk = np.sqrt(left2 / (k - 1)) if dynamic else delta
        bond_delta[k - 2] = dk
        r = _rank_rule(s, dk, max_rank)
        sigma[k - 2] = s
        tail[k - 2] = float(np.sum(s[r:] ** 2))
        left2 = max(0.0, left2 - tail[k - 2])
        Uk = U[:, :r].copy()
        VS = (Vt[:r].T * s[:r]).copy()
        Uk, VS = _sign_fix(Uk, VS)
        G[k - 1] = Uk.T.reshape(r, n, r1)
        G[k - 2] = np.tensordot(G[k - 2], VS, axes=([2], [0]))
    ranks = [1] + [int(g.shape[2]) for g in G]
    return G, ranks, sigma, tail, delta, bond_delta


def fiber_count(idx, dims, p: int) -> int:
    idx = np.asarray(idx, dtype=np.int64)
    rest = np.delete(idx, p - 1, axis=1)
    return int(np.unique(rest, axis=0).shape[0]) if rest.shape[1] else 1


def rank_bounds(dims, p: int, R: int):
    """The upper bounds r_bar_k (k = 0..d) of Algorithm 4's ranks."""
    d = len(dims)
    rb = [1] * (d + 1)
    for k in range(1, d):
        if k < p:
            rb[k] = int(min(R, np.prod([int(x) for x in dims[:k]], dtype=object)))
        else:
            rb[k] = int(min(R, np.prod([int(x) for x in dims[k:]], dtype=object)))
    return rb


def f_svd(m, n) -> float:
    return float(m) * float(n) * float(min(m, n))


def flop_estimate(dims, p: int, rt, r) -> float:
    """Estimated FLOP count of Algorithm 6 (Sec. 3.6): ranks rt before, r after (k = 0..d)."""
    d = len(dims)
    n = [int(x) for x in dims]
    f = f_svd(rt[p - 1] * n[p - 1], rt[p])
    for i in range(p + 1, d):
        f += f_svd(r[i - 1] * n[i - 1], rt[i])
    for i in range(2, p + 1):
        f += f_svd(rt[i - 1], n[i - 1] * r[i])
    return f


def select_p(idx, dims):
    """Algorithm 9 with the bounds r_bar for both rank sets: (p, costs by p)."""
    d = len(dims)
    costs = []
    for p in range(1, d + 1):
        R = fiber_count(idx, dims, p)
        rb = rank_bounds(dims, p, R)
        costs.append(flop_estimate(dims, p, rb, rb))
    return int(np.argmin(costs)) + 1, costs


def decompose(idx, val, dims, eps: float, p: int = 0, max_rank: int = 0, dynamic_delta: bool = False) -> FttResult:
    """Algorithm 7 (FastTT): exact rank-reduced TT, then Algorithm 6 (Algorithm 8 with
    dynamic_delta).  p = 0: Algorithm 9."""
    if p == 0:
        idx_v, _ = _validate(idx, val, dims)
        p, _ = select_p(idx_v, dims)
    ex = exact_tt(idx, val, dims, p)
    cores, ranks, sigma, tail, delta, bd = round_tt(ex.cores, p, eps, ex.norm, max_rank, dynamic_delta)
    return FttResult(cores=cores, ranks=ranks, exact_ranks=ex.ranks, R=ex.R, p=p, norm=ex.norm, delta=delta,
                     sigma=sigma, tail=tail, bond_delta=bd)
