"""Seeded synthetic sparse tensors (COO) shaped like the workloads of the method.

This module only builds inputs: coordinates, values and mode sizes.  It holds none
of the decomposition's arithmetic, so both the HIP path and the CPU oracle may use
it.  Every generator is deterministic for a given seed (NumPy PCG64) and returns

    idx  : int32 [nnz, d]  0-based coordinates, row-major (last mode fastest)
    val  : float64 [nnz]   nonzero values
    dims : tuple of d ints

Workloads (sizes are those of the sparse-tensor experiments the method targets):

* ``random_sparse``  -- uniform random distinct coordinates, N(0,1) values.
* ``kronecker_sum``  -- sum of K sparse rank-1 (Kronecker) terms; every mode factor
  has ``q`` nonzeros drawn from the dyadic grid {16..48}/32, so products of d <= 8
  factors and their sums are exact in binary64 and parallel columns stay exactly
  parallel (heavy parallel-column structure).
* ``orthogonal_terms`` -- rank-1 terms with disjoint supports and geometrically
  spaced weights: every unfolding has a known spectrum of a chosen condition number.
* ``laplacian_qtt``  -- the 2D Dirichlet 5-point Laplacian on a 2^L x 2^L grid as a
  2L-way tensor with modes of size 4 (quantized TT / matrix-in-TT layout: row and
  column bits interleaved, x bits first, most significant bit first).
* ``fdm3d_mpo``      -- the 3D 7-point finite-difference matrix on an n^3 grid as a
  3-way tensor with modes of size n^2 (matrix-in-TT layout, modes (x,x'), (y,y'),
  (z,z')), with constant ("pattern") or random coefficients.
"""
from __future__ import annotations

import hashlib

import numpy as np

__all__ = [
    "random_sparse",
    "kronecker_sum",
    "noisy_kronecker",
    "orthogonal_terms",
    "laplacian_matrix",
    "laplacian_qtt",
    "fdm3d_matrix",
    "fdm3d_mpo",
    "unravel",
    "checksum",
    "workload",
    "WORKLOADS",
]


def unravel(lin: np.ndarray, dims) -> np.ndarray:
    """Row-major (last index fastest) linear indices -> int32 [nnz, d] coordinates."""
    lin = np.asarray(lin, dtype=np.int64)
    out = np.empty((lin.size, len(dims)), dtype=np.int32)
    rem = lin.copy()
    for k in range(len(dims) - 1, -1, -1):
        out[:, k] = rem % dims[k]
        rem //= dims[k]
    return out


def _ravel(idx: np.ndarray, dims) -> np.ndarray:
    lin = np.zeros(idx.shape[0], dtype=np.int64)
    for k, n in enumerate(dims):
        lin = lin * int(n) + idx[:, k].astype(np.int64)
    return lin


def random_sparse(dims, nnz: int, seed: int):
    """Distinct uniform-random coordinates (drawn as linear indices), N(0,1) values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = int(np.prod(np.asarray(dims, dtype=np.float64)))
    lin = rng.choice(total, int(nnz), replace=False)
    val = rng.standard_normal(int(nnz))
    return unravel(lin, dims), val.astype(np.float64), tuple(int(n) for n in dims)


def kronecker_sum(d: int, n: int, terms: int, q: int, seed: int, continuous: bool = False):
    """Sum of ``terms`` sparse rank-1 terms; each mode factor has ``q`` nonzeros.

    Values are integers 16..48 over 32 (dyadic, exact in binary64).  With
    ``continuous=True`` they are U[0.5, 1.5) instead (a robustness variant in which
    parallel columns are no longer exactly parallel after rounding).
    Overlapping coordinates of different terms are summed (exactly, in the dyadic
    case: all values are positive so nothing cancels).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = (n,) * d
    lin_parts, val_parts = [], []
    for _t in range(terms):
        pos, vals = [], []
        for _k in range(d):
            pos.append(rng.choice(n, q, replace=False).astype(np.int64))
            if continuous:
                vals.append(rng.uniform(0.5, 1.5, q))
            else:
                vals.append(rng.integers(16, 49, q).astype(np.float64) / 32.0)
        lin = np.zeros(1, dtype=np.int64)
        v = np.ones(1, dtype=np.float64)
        for k in range(d):
            lin = (lin[:, None] * n + pos[k][None, :]).reshape(-1)
            v = (v[:, None] * vals[k][None, :]).reshape(-1)
        lin_parts.append(lin)
        val_parts.append(v)
    lin = np.concatenate(lin_parts)
    v = np.concatenate(val_parts)
    uniq, inv = np.unique(lin, return_inverse=True)
    acc = np.zeros(uniq.size, dtype=np.float64)
    np.add.at(acc, inv, v)
    return unravel(uniq, dims), acc, dims


def orthogonal_terms(d: int, terms: int, q: int, kappa: float, seed: int):
    """Sum of ``terms`` rank-1 terms with pairwise disjoint supports in every mode.

    Mode size ``terms * q``; each factor is ``q`` ones on its own block of indices
    (blocks scattered by a random permutation per mode); term t carries the weight
    w_t = kappa^(t / (terms - 1)), the weights shuffled over the terms.  Every
    unfolding then has exactly the singular values w_t q^(d/2) (the terms are
    orthogonal in every unfolding), so its condition number is ``kappa``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = terms * q
    dims = (n,) * d
    perms = [rng.permutation(n) for _ in range(d)]
    w = kappa ** (np.arange(terms) / max(terms - 1, 1))
    w = w[rng.permutation(terms)]
    local = np.stack(np.meshgrid(*([np.arange(q)] * d), indexing="ij"), -1).reshape(-1, d)
    idx = np.concatenate([_perms_apply(perms, t * q + local) for t in range(terms)]).astype(np.int32)
    val = np.repeat(w, q ** d).astype(np.float64)
    return idx, val, dims


def _perms_apply(perms, idx):
    return np.stack([perms[k][idx[:, k]] for k in range(idx.shape[1])], 1)


def noisy_kronecker(seed: int, noise: float, d: int = 4, n: int = 6, terms: int = 5, q: int = 3):
    """Sum of rank-1 terms with factor values in {1, 2, 3}, and a noisy copy.

    Returns (idx, clean, noisy, dims): ``noisy`` is every entry times (1 + eta),
    eta ~ U(-noise, noise), so parallel columns of ``clean`` stay parallel in
    ``noisy`` only up to that perturbation.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    acc = {}
    for _ in range(terms):
        pos = [rng.choice(n, q, replace=False) for _ in range(d)]
        vals = [rng.integers(1, 4, q).astype(np.float64) for _ in range(d)]
        for a in np.ndindex(*(q,) * d):
            key = tuple(int(pos[k][a[k]]) for k in range(d))
            acc[key] = acc.get(key, 0.0) + float(np.prod([vals[k][a[k]] for k in range(d)]))
    idx = np.array(list(acc.keys()), dtype=np.int32)
    clean = np.array(list(acc.values()))
    noisy = clean * (1 + rng.uniform(-noise, noise, clean.size))
    return idx, clean, noisy, (n,) * d


def laplacian_matrix(L: int):
    """2D Dirichlet 5-point Laplacian on a 2^L x 2^L grid as a sparse matrix.

    Matrix index I = x * 2^L + y.  Entries: 4 on the diagonal, -1 between grid
    neighbours.  Returns (rows int64, cols int64, vals, row_dims, col_dims) with
    row_dims = col_dims = (2,) * 2L (the binary digits of the index, the quantized
    layout).  nnz = 5 * 4^L - 4 * 2^L.
    """
    side = 1 << L
    x, y = np.meshgrid(np.arange(side, dtype=np.int64), np.arange(side, dtype=np.int64), indexing="ij")
    x = x.reshape(-1)
    y = y.reshape(-1)
    I = x * side + y
    rows, cols, vals = [I], [I], [np.full(I.size, 4.0)]
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        xn, yn = x + dx, y + dy
        ok = (xn >= 0) & (xn < side) & (yn >= 0) & (yn < side)
        rows.append(I[ok])
        cols.append(xn[ok] * side + yn[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals).astype(np.float64)
    return r, c, v, (2,) * (2 * L), (2,) * (2 * L)


def laplacian_qtt(L: int):
    """The matrix of ``laplacian_matrix(L)`` in quantized-TT layout.

    The tensor has 2L modes of size 4; mode k (1-based) holds
    2 * bit_{2L-k}(I) + bit_{2L-k}(J), i.e. x bits first, most significant first.
    """
    r, c, v, _, _ = laplacian_matrix(L)
    d = 2 * L
    idx = np.empty((r.size, d), dtype=np.int32)
    for k in range(1, d + 1):
        b = d - k
        idx[:, k - 1] = (2 * ((r >> b) & 1) + ((c >> b) & 1)).astype(np.int32)
    return idx, v.astype(np.float64), (4,) * d


def _fdm3d_stencil(n: int, coeff: str, seed: int):
    """Grid coordinates of both ends of every stored entry, and its value."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(n, dtype=np.int64)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = x.reshape(-1), y.reshape(-1), z.reshape(-1)
    src = [(x, y, z, x, y, z, np.full(x.size, 6.0))]
    for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        xn, yn, zn = x + dx, y + dy, z + dz
        ok = (xn >= 0) & (xn < n) & (yn >= 0) & (yn < n) & (zn >= 0) & (zn < n)
        src.append((x[ok], y[ok], z[ok], xn[ok], yn[ok], zn[ok], np.full(int(ok.sum()), -1.0)))
    cols = [np.concatenate([s[i] for s in src]) for i in range(7)]
    xa, ya, za, xb, yb, zb, v = cols
    if coeff == "random":
        v = rng.standard_normal(v.size)
    elif coeff != "pattern":
        raise ValueError("coeff must be 'pattern' or 'random'")
    return xa, ya, za, xb, yb, zb, v.astype(np.float64)


def fdm3d_matrix(n: int, coeff: str = "pattern", seed: int = 0):
    """3D 7-point finite-difference matrix on an n x n x n grid as a sparse matrix.

    Grid point p = (x, y, z), matrix index I = (x * n + y) * n + z.  ``pattern``:
    6 on the diagonal and -1 for each neighbour; ``random``: every stored entry
    N(0,1).  Returns (rows int64, cols int64, vals, row_dims, col_dims) with
    row_dims = col_dims = (n, n, n).  nnz = n^3 + 6 n^2 (n - 1).
    """
    xa, ya, za, xb, yb, zb, v = _fdm3d_stencil(n, coeff, seed)
    return (xa * n + ya) * n + za, (xb * n + yb) * n + zb, v, (n,) * 3, (n,) * 3


def fdm3d_mpo(n: int, coeff: str = "pattern", seed: int = 0):
    """The matrix of ``fdm3d_matrix`` as a 3-way tensor.

    The tensor modes are (x, x'), (y, y'), (z, z'), each of size n^2 with index
    a * n + a'.
    """
    xa, ya, za, xb, yb, zb, v = _fdm3d_stencil(n, coeff, seed)
    idx = np.stack([xa * n + xb, ya * n + yb, za * n + zb], axis=1).astype(np.int32)
    return idx, v, (n * n,) * 3


def checksum(idx: np.ndarray, val: np.ndarray, dims) -> str:
    """SHA-256 over (dims, coordinates and value bits in row-major coordinate order)."""
    lin = _ravel(np.asarray(idx), dims)
    order = np.argsort(lin, kind="stable")
    h = hashlib.sha256()
    h.update(np.asarray(dims, dtype=np.int64).tobytes())
    h.update(lin[order].tobytes())
    h.update(np.asarray(val, dtype=np.float64)[order].tobytes())
    return h.hexdigest()


# Named workloads.  eps is the relative Frobenius tolerance the workload is run at.
WORKLOADS = {
    # 4-way 20^4, 1000 random nonzeros, N(0,1), eps 1e-12 (no effective truncation).
    "random4d_n20_nnz1k": dict(kind="random", dims=(20,) * 4, nnz=1000, seed=1, eps=1e-12),
    # 8-way 32^8, 64 Kronecker terms with 4 nonzeros per mode factor (~4.19M nnz), eps 1e-8.
    "kron8d_n32_t64": dict(kind="kron", d=8, n=32, terms=64, q=4, seed=2, eps=1e-8),
    # The same with continuous U[0.5, 1.5) factor values: parallel columns only up to
    # rounding, so it needs the tolerant parallel test (key_bits).
    "kron8d_n32_t64_cont": dict(kind="kron", d=8, n=32, terms=64, q=4, seed=2, eps=1e-8, continuous=True),
    # 2D 5-point Laplacian, 1024 x 1024 grid, as a 20-way QTT tensor (5,238,784 nnz), eps 1e-10.
    "laplace2d_qtt_L10": dict(kind="laplace", L=10, eps=1e-10),
    # 3D 7-point FDM matrix on a 40^3 grid, random coefficients, as a 3-way tensor
    # with modes of size 1600 (438,400 nnz), eps 1e-14: the largest case of the FDM
    # table, for the fiber-trie variant.
    "fdm3d_n40_random": dict(kind="fdm", n=40, coeff="random", seed=1, eps=1e-14),
    # the other FDM cases of the same table
    "fdm3d_n20_pattern": dict(kind="fdm", n=20, coeff="pattern", seed=1, eps=1e-14),
    "fdm3d_n30_pattern": dict(kind="fdm", n=30, coeff="pattern", seed=1, eps=1e-14),
    "fdm3d_n20_random": dict(kind="fdm", n=20, coeff="random", seed=1, eps=1e-14),
    "fdm3d_n30_random": dict(kind="fdm", n=30, coeff="random", seed=1, eps=1e-14),
    # 5-way 200^5 with 10M random nonzeros, N(0,1), eps 1e-2.
    "random5d_n200_nnz10m": dict(kind="random", dims=(200,) * 5, nnz=10_000_000, seed=4, eps=1e-2),
}


def workload(name: str):
    """Build a named workload: returns (idx, val, dims, eps)."""
    w = WORKLOADS[name]
    if w["kind"] == "random":
        idx, val, dims = random_sparse(w["dims"], w["nnz"], w["seed"])
    elif w["kind"] == "kron":
        idx, val, dims = kronecker_sum(w["d"], w["n"], w["terms"], w["q"], w["seed"], w.get("continuous", False))
    elif w["kind"] == "laplace":
        idx, val, dims = laplacian_qtt(w["L"])
    elif w["kind"] == "fdm":
        idx, val, dims = fdm3d_mpo(w["n"], w["coeff"], w["seed"])
    else:  # pragma: no cover
        raise KeyError(name)
    return idx, val, dims, w["eps"]
