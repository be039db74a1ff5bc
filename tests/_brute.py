"""Independent brute-force references used to pin the oracle (pure Python / NumPy).

Nothing here is shared with the oracle or the HIP path.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _lin(coords, dims):
    x = 0
    for c, n in zip(coords, dims):
        x = x * n + int(c)
    return x


def _unlin(x, dims):
    out = []
    for n in reversed(dims):
        out.append(x % n)
        x //= n
    return tuple(reversed(out))


def depar_exact(M: dict, ncols: int):
    """Deparallelisation (Algorithm 3) of a matrix given as {(row, col): Fraction}.

    Columns are scanned in order 0..ncols-1.  A column is compared against every kept
    column with the exact pairwise test (same support, u_i w_f == w_i u_f for all i,
    exact rational arithmetic); the first parallel kept column receives the prefactor,
    a column parallel to none is kept.  All-zero columns are skipped (they are the
    zero multiple of any column).  The kept columns are then rescaled so that their
    first nonzero is 1 (the transfer rows scaled inversely), which leaves M = N T.

    Returns (N list of {row: Fraction}, col -> (group, prefactor)).
    """
    cols = {}
    for (r, c), v in M.items():
        if v != 0:
            cols.setdefault(c, {})[r] = v
    kept = []        # first-seen columns, unnormalised
    T = {}           # col -> (kept index, prefactor w.r.t. kept column)
    for j in range(ncols):
        u = cols.get(j)
        if not u:
            continue
        hit = None
        for i, w in enumerate(kept):
            if set(u) != set(w):
                continue
            f = min(u)
            if all(u[x] * w[f] == w[x] * u[f] for x in u):
                hit = i
                T[j] = (i, u[f] / w[f])
                break
        if hit is None:
            kept.append(u)
            T[j] = (len(kept) - 1, Fraction(1))
    N = []
    for i, w in enumerate(kept):
        f = min(w)
        N.append({x: w[x] / w[f] for x in w})
    out = {}
    for j, (i, pf) in T.items():
        f = min(kept[i])
        out[j] = (i, pf * kept[i][f])
    return N, out


def cps_exact(idx, val, dims):
    """Algorithm 1 with every truncated SVD replaced by exact Deparallelisation.

    Works on tiny tensors (dense unfoldings enumerated in exact rationals).
    Returns per level k (1..d-1): dict(beta, N, T) with T: col -> (group, prefactor),
    plus the last core as {(g, i_d): Fraction}.
    """
    dims = tuple(int(n) for n in dims)
    d = len(dims)
    A = {}
    for c, v in zip(np.asarray(idx), np.asarray(val)):
        if v != 0:
            A[tuple(int(x) for x in c)] = Fraction(float(v))
    C = {}
    for c, v in A.items():
        C[(c[0], _lin(c[1:], dims[1:]))] = v
    levels = []
    last = None
    for k in range(1, d):
        ncols = int(np.prod(dims[k:]))
        N, T = depar_exact(C, ncols)
        levels.append(dict(beta=len(N), N=N, T=T))
        if k < d - 1:
            nk1 = dims[k]
            rest = dims[k + 1:]
            C = {}
            for j, (g, pf) in T.items():
                suf = _unlin(j, dims[k:])
                C[(g * nk1 + suf[0], _lin(suf[1:], rest))] = pf
        else:
            last = {(g, j): pf for j, (g, pf) in T.items()}
    return levels, last


def dense_tensor(idx, val, dims):
    A = np.zeros(tuple(int(n) for n in dims))
    for c, v in zip(np.asarray(idx), np.asarray(val)):
        A[tuple(int(x) for x in c)] += v
    return A


def tt_full(cores):
    """Dense tensor of a TT given as cores [r_{k-1}, n_k, r_k]."""
    X = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    for G in cores[1:]:
        X = np.tensordot(X, G, axes=([X.ndim - 1], [0]))
    return X.reshape(X.shape[:-1] if X.shape[-1] == 1 else X.shape)


def tt_svd_right_to_left(A, eps=None, ranks_fixed=None, dynamic=False):
    """Dense TT-SVD (Algorithm 1) run from the last mode to the first, LAPACK SVDs.

    dynamic: thresholds of Algorithm 8 (Sec. 3.5) instead of one fixed threshold:
    the budget (eps ||A||)^2, less what earlier bonds discarded, shared evenly by
    the bonds still to come.
    Returns (ranks [1, r_1, ..., r_{d-1}, 1], sigma per bond b = 1..d-1).
    """
    d = A.ndim
    n = A.shape
    nrm = np.linalg.norm(A.reshape(-1))
    delta = 0.0 if eps is None else eps * nrm / np.sqrt(d - 1)
    budget = 0.0 if eps is None else (eps * nrm) ** 2
    ranks = [1] * (d + 1)
    sig = [None] * (d - 1)
    C = A.reshape(-1)
    r_right = 1
    for k in range(d, 1, -1):
        C = C.reshape(int(np.prod(n[: k - 1])), n[k - 1] * r_right)
        U, S, Vt = np.linalg.svd(C, full_matrices=False)
        if ranks_fixed is not None:
            r = max(1, min(int(ranks_fixed), int(np.sum(S > 0))))
        else:
            tail = np.concatenate([np.cumsum((S * S)[::-1])[::-1], [0.0]])
            thr2 = budget / (k - 1) if dynamic else delta * delta
            r = next(rr for rr in range(1, S.size + 1) if tail[rr] <= thr2)
            budget = max(0.0, budget - tail[r])
        sig[k - 2] = S
        ranks[k - 1] = r
        C = U[:, :r] * S[:r]
        r_right = r
    return ranks, sig
