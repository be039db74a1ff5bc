// CPU oracle for the sparse tensor-train decomposition (test infrastructure only).
//
// Plain, single-threaded, FP64.  Written from arXiv 1908.02721, "Faster Tensor
// Train Decomposition for Sparse Data".  Only the test-suite, the smoke check and
// the benchmark's CPU-baseline leg may load this library; it shares no code with
// the HIP path.
//
// What it computes, step by step (paper notation, 0-based indices, row-major
// linearisation with the last index fastest as in the vectorisation definition of
// Sec. 2.2):
//
//  1. Input: COO coordinates and values.  Explicit zeros are dropped; an index out
//     of range, a non-finite value or a repeated coordinate is an error.
//  2. ||A||_F summed in row-major coordinate order; delta = eps*||A||_F/sqrt(d-1)
//     (Algorithm 1, first step).
//  3. Parallel-vector rounding applied level by level to sparse unfoldings: this is
//     the TT-SVD sweep (Algorithm 1) with every delta-truncated SVD replaced by
//     Deparallelisation (Algorithm 3), as Sec. 2.4 describes parallel-vector
//     rounding.  At level k the matrix is the reshape of Algorithm 1 (rows
//     rho = g_{k-1}*n_k + i_k, columns = suffixes (i_{k+1},...,i_d) in row-major
//     order).  Deparallelisation, read as: scan the columns in order; a column is
//     "parallel" to a kept column iff their canonical forms (every entry divided by
//     the entry of smallest row, IEEE binary64 division) are bitwise identical; a
//     column parallel to no kept column starts a new group (numbered in scan
//     order); the transfer-matrix entry of a column is the prefactor s = value at
//     its smallest row.  The kept (canonical) columns form N_k and the core is
//     reshape(N_k, [beta_{k-1}, n_k, beta_k]) (Algorithm 1, core step); the
//     transfer matrix becomes the next level (C := T in place of C := Sigma V^T).
//     At the last level the transfer matrix is the last core.
//     Tolerant parallel test (optional, key_bits = b in 1..52): every canonical
//     value is rounded to b fraction bits before it is keyed and stored, by
//     round-half-to-even on the magnitude's bit pattern (a carry may move into the
//     exponent; a rounding that would reach the infinity/NaN exponent truncates
//     instead).  Columns parallel up to a relative perturbation well below 2^-b
//     then share one key; each stored entry moves by at most 2^-(b+1) relative.
//  4. TT-rounding (Algorithm 2, run mirrored): a left-to-right Householder QR sweep
//     (all-zero rows are left out of each QR, m = min(non-zero rows, columns),
//     diag(R) >= 0) followed by a right-to-left sweep of delta-truncated SVDs of
//     unfold_1^T of each core (one-sided Jacobi), rank_delta = the smallest r >= 1
//     whose discarded sum of sigma^2 is <= delta^2, merging V*Sigma into the left
//     neighbour (the product of Algorithm 6's merge step).  Fixed-rank truncation
//     (Sec. 3.4) keeps min(max_rank, #nonzero sigma) instead.  In each kept left
//     singular vector the entry of largest magnitude (lowest index on ties) is made
//     positive.
//     Dynamic truncation (Algorithm 8, Sec. 3.5), read for this sweep direction:
//     the whole budget eps*||A||_F is spent by the one SVD sweep (Algorithm 8 with
//     p = d has an empty first loop, so delta_left = eps*||A||_F).  With j bonds
//     still to truncate, the bond's threshold is rem/sqrt(j); after the bond, rem^2
//     loses the discarded sum of sigma^2.
//  5. Entry evaluation a_i = G1[i1] G2[i2] ... Gd[id] (Sec. 2.3) and its gradient by
//     the product rule, with explicit left and right partial products.

#include "ttoracle.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <numeric>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

// Canonical value rounded to b fraction bits (b = 0: unchanged).
double snap_value(double x, int32_t b) {
  if (b <= 0 || b >= 52) return x;
  uint64_t u;
  std::memcpy(&u, &x, sizeof(u));
  const uint64_t sign = u & (uint64_t(1) << 63);
  const uint64_t mag = u & ~sign;
  const int drop = 52 - b;
  const uint64_t kept = mag >> drop;            // bits that stay, as an integer
  const uint64_t rest = mag & ((uint64_t(1) << drop) - 1);
  const uint64_t half = uint64_t(1) << (drop - 1);
  uint64_t up = kept;
  if (rest > half || (rest == half && (kept & 1))) up = kept + 1;
  uint64_t r = up << drop;
  if ((r >> 52) >= 0x7FF) r = kept << drop;     // would reach inf/NaN: truncate
  r |= sign;
  double y;
  std::memcpy(&y, &r, sizeof(y));
  return y;
}

struct LevelOut {
  std::vector<int64_t> col;   // row-major linear index of each column's suffix
  std::vector<int32_t> g;     // group of each column (transfer-matrix row)
  std::vector<double> s;      // prefactor of each column (transfer-matrix value)
  int64_t beta = 0;           // number of groups (rank after the level)
  std::vector<int64_t> colptr, row;  // N_k, CSC
  std::vector<double> val;
};

// One entry of a level's sparse unfolding.  The column it belongs to is the suffix
// of the coordinates of a representative input nonzero `rep`.
struct Entry {
  int64_t rep;
  int64_t rho;
  double v;
};

uint64_t bits_of(double x) {
  uint64_t b;
  std::memcpy(&b, &x, sizeof b);
  return b;
}

// ---------------------------------------------------------------------------
// Dense linear algebra (plain loops).
// ---------------------------------------------------------------------------

// Householder QR of the column-major m x n matrix `a` (destroyed).
// Returns p = min(m, n); Q is m x p column-major with orthonormal columns, R is
// p x n row-major, upper trapezoidal, A = Q R.  Reflector j maps column j's
// trailing part x to alpha*e_1 with alpha = -sign(x_0)*||x|| (sign(0) = +1).
int64_t householder_qr(int64_t m, int64_t n, std::vector<double>& a, std::vector<double>* Q,
                       std::vector<double>& R) {
  const int64_t p = std::min(m, n);
  std::vector<double> vs(static_cast<size_t>(m * p), 0.0);
  std::vector<double> tau(static_cast<size_t>(p), 0.0);
  R.assign(static_cast<size_t>(p * n), 0.0);
  for (int64_t j = 0; j < p; ++j) {
    double* x = &a[j * m];
    double nrm2 = 0.0;
    for (int64_t i = j; i < m; ++i) nrm2 += x[i] * x[i];
    const double nrm = std::sqrt(nrm2);
    double alpha = 0.0;
    if (nrm > 0.0) {
      alpha = (x[j] >= 0.0) ? -nrm : nrm;
      double* v = &vs[j * m];
      for (int64_t i = j; i < m; ++i) v[i] = x[i];
      v[j] -= alpha;
      double vtv = 0.0;
      for (int64_t i = j; i < m; ++i) vtv += v[i] * v[i];
      tau[j] = (vtv > 0.0) ? 2.0 / vtv : 0.0;
      for (int64_t c = j + 1; c < n; ++c) {
        double* y = &a[c * m];
        double w = 0.0;
        for (int64_t i = j; i < m; ++i) w += v[i] * y[i];
        w *= tau[j];
        for (int64_t i = j; i < m; ++i) y[i] -= w * v[i];
      }
    }
    R[j * n + j] = alpha;
    for (int64_t c = j + 1; c < n; ++c) R[j * n + c] = a[c * m + j];
  }
  if (Q) {
    Q->assign(static_cast<size_t>(m * p), 0.0);
    for (int64_t c = 0; c < p; ++c) (*Q)[c * m + c] = 1.0;
    for (int64_t j = p - 1; j >= 0; --j) {
      if (tau[j] == 0.0) continue;
      const double* v = &vs[j * m];
      for (int64_t c = 0; c < p; ++c) {
        double* y = &(*Q)[c * m];
        double w = 0.0;
        for (int64_t i = j; i < m; ++i) w += v[i] * y[i];
        w *= tau[j];
        for (int64_t i = j; i < m; ++i) y[i] -= w * v[i];
      }
    }
  }
  return p;
}

// One-sided (Hestenes) Jacobi SVD of the column-major m x n matrix `g` (overwritten
// by G V).  V is n x n column-major.  On return column j of g is u_j * sigma_j.
void jacobi_svd(int64_t m, int64_t n, std::vector<double>& g, std::vector<double>& V) {
  V.assign(static_cast<size_t>(n * n), 0.0);
  for (int64_t j = 0; j < n; ++j) V[j * n + j] = 1.0;
  const double tol = std::sqrt(static_cast<double>(std::max<int64_t>(m, 1))) *
                     std::numeric_limits<double>::epsilon();
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int64_t p = 0; p + 1 < n; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        double* gp = &g[p * m];
        double* gq = &g[q * m];
        double a = 0.0, b = 0.0, c = 0.0;
        for (int64_t i = 0; i < m; ++i) {
          a += gp[i] * gp[i];
          b += gq[i] * gq[i];
          c += gp[i] * gq[i];
        }
        if (a == 0.0 || b == 0.0) continue;
        if (std::fabs(c) <= tol * std::sqrt(a) * std::sqrt(b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::hypot(1.0, zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = cs * t;
        for (int64_t i = 0; i < m; ++i) {
          const double x = gp[i], y = gq[i];
          gp[i] = cs * x - sn * y;
          gq[i] = sn * x + cs * y;
        }
        double* vp = &V[p * n];
        double* vq = &V[q * n];
        for (int64_t i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = cs * x - sn * y;
          vq[i] = sn * x + cs * y;
        }
      }
    }
    if (!rotated) break;
  }
}

// new = R x_1 core, i.e. unfold_1(new) = R * unfold_1(core).
// R is rn x r0 row-major; core is r0 x rest row-major; result rn x rest.
std::vector<double> mode1_product(const std::vector<double>& R, int64_t rn, int64_t r0,
                                  const std::vector<double>& core, int64_t rest) {
  std::vector<double> out(static_cast<size_t>(rn * rest), 0.0);
  for (int64_t a = 0; a < rn; ++a) {
    for (int64_t al = 0; al < r0; ++al) {
      const double rv = R[a * r0 + al];
      if (rv == 0.0) continue;
      const double* src = &core[al * rest];
      double* dst = &out[a * rest];
      for (int64_t x = 0; x < rest; ++x) dst[x] += rv * src[x];
    }
  }
  return out;
}

// new = core x_3 W, i.e. unfold_2(new) = unfold_2(core) * W.
// core is rows x r1 row-major, W is r1 x rn row-major; result rows x rn.
std::vector<double> mode3_product(const std::vector<double>& core, int64_t rows, int64_t r1,
                                  const std::vector<double>& W, int64_t rn) {
  std::vector<double> out(static_cast<size_t>(rows * rn), 0.0);
  for (int64_t x = 0; x < rows; ++x) {
    for (int64_t al = 0; al < r1; ++al) {
      const double cv = core[x * r1 + al];
      if (cv == 0.0) continue;
      for (int64_t j = 0; j < rn; ++j) out[x * rn + j] += cv * W[al * rn + j];
    }
  }
  return out;
}

}  // namespace

struct orc_result_s {
  int32_t d = 0;
  std::vector<int64_t> n;
  int64_t nnz = 0;
  double norm = 0.0, delta = 0.0;
  int32_t rounded = 0;
  double t[4] = {0, 0, 0, 0};
  std::vector<LevelOut> lev;            // lev[k-1], k = 1..d-1
  std::vector<double> last_exact;       // beta_{d-1} x n_d
  std::vector<int64_t> ranks, qr_ranks;
  std::vector<std::vector<double>> cores;
  std::vector<std::vector<double>> sigma;  // sigma[b-1], bond b = 1..d-1
  std::vector<double> tail;
  std::vector<double> bond_delta;          // threshold used at bond b = 1..d-1
};

extern "C" {

int orc_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx,
                  const double* val, double eps, int32_t max_rank, int32_t do_round,
                  int32_t dynamic_delta, int32_t key_bits, orc_result** out) {
  if (!out) return ORC_ERR_ARG;
  *out = nullptr;
  if (d < 2 || !dims || nnz < 0 || (nnz > 0 && (!idx || !val))) return ORC_ERR_ARG;
  if (!(eps >= 0.0 && eps < 1.0) || max_rank < 0 || key_bits < 0 || key_bits > 52) return ORC_ERR_ARG;
  for (int32_t k = 0; k < d; ++k)
    if (dims[k] <= 0 || dims[k] > std::numeric_limits<int32_t>::max()) return ORC_ERR_ARG;

  auto res = new orc_result_s();
  res->d = d;
  res->n.assign(dims, dims + d);
  const std::vector<int64_t>& n = res->n;
  auto t0 = Clock::now();

  // 1. Validate and drop explicit zeros.  Errors are reported in the order:
  //    index out of range, then non-finite value, then repeated coordinate.
  for (int64_t e = 0; e < nnz; ++e)
    for (int32_t k = 0; k < d; ++k)
      if (idx[e * d + k] < 0 || idx[e * d + k] >= n[k]) { delete res; return ORC_ERR_INDEX; }
  for (int64_t e = 0; e < nnz; ++e)
    if (!std::isfinite(val[e])) { delete res; return ORC_ERR_NONFINITE; }
  std::vector<int64_t> kept;
  for (int64_t e = 0; e < nnz; ++e)
    if (val[e] != 0.0) kept.push_back(e);
  auto coord_less = [&](int64_t a, int64_t b) {
    for (int32_t k = 0; k < d; ++k) {
      if (idx[a * d + k] != idx[b * d + k]) return idx[a * d + k] < idx[b * d + k];
    }
    return false;
  };
  std::sort(kept.begin(), kept.end(), [&](int64_t a, int64_t b) {
    if (coord_less(a, b)) return true;
    if (coord_less(b, a)) return false;
    return a < b;
  });
  for (size_t e = 1; e < kept.size(); ++e)
    if (!coord_less(kept[e - 1], kept[e])) { delete res; return ORC_ERR_DUPLICATE; }
  if (kept.empty()) { delete res; return ORC_ERR_EMPTY; }
  res->nnz = static_cast<int64_t>(kept.size());

  // 2. Norm and per-bond threshold.
  double ss = 0.0;
  for (int64_t e : kept) ss += val[e] * val[e];
  res->norm = std::sqrt(ss);
  res->delta = eps * res->norm / std::sqrt(static_cast<double>(d - 1));
  res->t[0] = seconds_since(t0);

  // 3. Parallel-vector rounding on the sparse unfoldings, k = 1..d-1.
  t0 = Clock::now();
  std::vector<Entry> E;
  E.reserve(kept.size());
  for (int64_t e : kept) E.push_back(Entry{e, idx[e * d + 0], val[e]});
  res->lev.resize(d - 1);
  for (int32_t k = 1; k <= d - 1; ++k) {
    // Columns are suffixes (modes k..d-1, 0-based); row-major column order, then rows.
    auto suffix_less = [&](const Entry& a, const Entry& b) {
      for (int32_t j = k; j < d; ++j) {
        const int32_t x = idx[a.rep * d + j], y = idx[b.rep * d + j];
        if (x != y) return x < y;
      }
      return false;
    };
    std::sort(E.begin(), E.end(), [&](const Entry& a, const Entry& b) {
      if (suffix_less(a, b)) return true;
      if (suffix_less(b, a)) return false;
      return a.rho < b.rho;
    });
    LevelOut& L = res->lev[k - 1];
    std::map<std::vector<uint64_t>, int32_t> groups;
    std::vector<Entry> next;
    L.colptr.push_back(0);
    if (k == d - 1) res->last_exact.clear();
    std::vector<std::pair<int32_t, std::pair<int64_t, double>>> last_entries;
    size_t a = 0;
    while (a < E.size()) {
      size_t b = a + 1;
      while (b < E.size() && !suffix_less(E[a], E[b])) ++b;
      // Column E[a..b): rows strictly increasing (distinct by construction).
      const int64_t m = static_cast<int64_t>(b - a);
      const double s = E[a].v;
      std::vector<uint64_t> key;
      key.reserve(1 + 2 * m);
      key.push_back(static_cast<uint64_t>(m));
      std::vector<double> c(static_cast<size_t>(m));
      for (int64_t j = 0; j < m; ++j) {
        if (j > 0 && E[a + j].rho <= E[a + j - 1].rho) { delete res; return ORC_ERR_ARG; }
        key.push_back(static_cast<uint64_t>(E[a + j].rho));
      }
      for (int64_t j = 0; j < m; ++j) {
        c[j] = snap_value(E[a + j].v / s, key_bits);
        key.push_back(bits_of(c[j]));
      }
      auto it = groups.find(key);
      int32_t g;
      if (it == groups.end()) {
        g = static_cast<int32_t>(groups.size());
        groups.emplace(std::move(key), g);
        for (int64_t j = 0; j < m; ++j) {
          L.row.push_back(E[a + j].rho);
          L.val.push_back(c[j]);
        }
        L.colptr.push_back(static_cast<int64_t>(L.row.size()));
      } else {
        g = it->second;
      }
      const int64_t rep = E[a].rep;
      int64_t lin = 0;
      for (int32_t j = k; j < d; ++j) lin = lin * n[j] + idx[rep * d + j];
      L.col.push_back(lin);
      L.g.push_back(g);
      L.s.push_back(s);
      const int64_t inext = idx[rep * d + k];  // i_{k+1}
      if (k < d - 1) {
        next.push_back(Entry{rep, static_cast<int64_t>(g) * n[k] + inext, s});
      } else {
        last_entries.push_back({g, {inext, s}});
      }
      a = b;
    }
    L.beta = static_cast<int64_t>(groups.size());
    if (k == d - 1) {
      res->last_exact.assign(static_cast<size_t>(L.beta * n[d - 1]), 0.0);
      for (auto& x : last_entries) res->last_exact[x.first * n[d - 1] + x.second.first] = x.second.second;
    }
    E.swap(next);
  }
  res->t[1] = seconds_since(t0);

  if (!do_round) {
    *out = res;
    return ORC_OK;
  }

  // Exact cores (dense), ranks beta.
  std::vector<int64_t> r(d + 1, 1);
  for (int32_t k = 1; k <= d - 1; ++k) r[k] = res->lev[k - 1].beta;
  for (int32_t k = 1; k <= d; ++k) {
    const double sz = static_cast<double>(r[k - 1]) * n[k - 1] * r[k];
    if (sz > 4.0e8) { delete res; return ORC_ERR_TOO_LARGE; }
  }
  std::vector<std::vector<double>> G(d);
  for (int32_t k = 1; k <= d - 1; ++k) {
    const LevelOut& L = res->lev[k - 1];
    G[k - 1].assign(static_cast<size_t>(r[k - 1] * n[k - 1] * r[k]), 0.0);
    for (int64_t col = 0; col < L.beta; ++col)
      for (int64_t e = L.colptr[col]; e < L.colptr[col + 1]; ++e)
        G[k - 1][L.row[e] * r[k] + col] = L.val[e];
  }
  G[d - 1] = res->last_exact;

  // 4a. Left-to-right QR sweep.
  t0 = Clock::now();
  for (int32_t k = 1; k <= d - 1; ++k) {
    const int64_t rows = r[k - 1] * n[k - 1], cols = r[k];
    const std::vector<double>& X = G[k - 1];  // unfold_2, row-major rows x cols
    std::vector<int64_t> nzr;
    for (int64_t i = 0; i < rows; ++i) {
      bool nz = false;
      for (int64_t j = 0; j < cols && !nz; ++j) nz = (X[i * cols + j] != 0.0);
      if (nz) nzr.push_back(i);
    }
    const int64_t mr = static_cast<int64_t>(nzr.size());
    std::vector<double> a(static_cast<size_t>(mr * cols));
    for (int64_t j = 0; j < cols; ++j)
      for (int64_t i = 0; i < mr; ++i) a[j * mr + i] = X[nzr[i] * cols + j];
    std::vector<double> Q, R;
    const int64_t p = householder_qr(mr, cols, a, &Q, R);
    for (int64_t j = 0; j < p; ++j) {
      if (R[j * cols + j] < 0.0) {
        for (int64_t c = 0; c < cols; ++c) R[j * cols + c] = -R[j * cols + c];
        for (int64_t i = 0; i < mr; ++i) Q[j * mr + i] = -Q[j * mr + i];
      }
    }
    std::vector<double> core(static_cast<size_t>(rows * p), 0.0);
    for (int64_t j = 0; j < p; ++j)
      for (int64_t i = 0; i < mr; ++i) core[nzr[i] * p + j] = Q[j * mr + i];
    G[k - 1].swap(core);
    const int64_t rest = n[k] * r[k + 1];
    G[k] = mode1_product(R, p, cols, G[k], rest);
    r[k] = p;
  }
  res->qr_ranks = r;
  res->t[2] = seconds_since(t0);

  // 4b. Right-to-left truncated SVD sweep.
  t0 = Clock::now();
  res->sigma.assign(d - 1, {});
  res->tail.assign(d - 1, 0.0);
  const double delta_static2 = res->delta * res->delta;
  // remaining budget of Algorithm 8 (squared): eps^2 ||A||_F^2 before the first bond
  double rem2 = (eps * res->norm) * (eps * res->norm);
  res->bond_delta.assign(d - 1, 0.0);
  for (int32_t k = d; k >= 2; --k) {
    const int64_t rl = r[k - 1], nk = n[k - 1], rr = r[k];
    const int64_t m = nk * rr;  // rows of unfold_1^T
    // bonds k-1, k-2, ..., 1 are still to be truncated: k-1 of them
    const double delta2 = dynamic_delta ? rem2 / static_cast<double>(k - 1) : delta_static2;
    res->bond_delta[k - 2] = std::sqrt(delta2);
    // gmat: column-major m x rl, column alpha = row alpha of unfold_1.
    std::vector<double> gmat(G[k - 1]);
    std::vector<double> V;
    jacobi_svd(m, rl, gmat, V);
    std::vector<double> sig(static_cast<size_t>(rl));
    for (int64_t j = 0; j < rl; ++j) {
      double s2 = 0.0;
      for (int64_t i = 0; i < m; ++i) s2 += gmat[j * m + i] * gmat[j * m + i];
      sig[j] = std::sqrt(s2);
    }
    std::vector<int64_t> perm(static_cast<size_t>(rl));
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return sig[x] > sig[y]; });
    std::vector<double> ss_sorted(static_cast<size_t>(rl));
    for (int64_t j = 0; j < rl; ++j) ss_sorted[j] = sig[perm[j]];
    // tail[r] = sum_{i >= r} sigma_i^2, accumulated from the smallest.
    std::vector<double> tailsum(static_cast<size_t>(rl + 1), 0.0);
    for (int64_t j = rl - 1; j >= 0; --j) tailsum[j] = tailsum[j + 1] + ss_sorted[j] * ss_sorted[j];
    int64_t rk;
    if (max_rank > 0) {
      int64_t nzs = 0;
      for (int64_t j = 0; j < rl; ++j) nzs += (ss_sorted[j] > 0.0);
      rk = std::max<int64_t>(1, std::min<int64_t>(max_rank, nzs));
    } else {
      rk = rl;
      for (int64_t cand = 1; cand <= rl; ++cand)
        if (tailsum[cand] <= delta2) { rk = cand; break; }
    }
    res->sigma[k - 2] = ss_sorted;
    res->tail[k - 2] = tailsum[rk];
    rem2 = std::max(0.0, rem2 - tailsum[rk]);
    // U (m x rk) and V*Sigma (rl x rk) with the sign rule.
    std::vector<double> U(static_cast<size_t>(m * rk)), VS(static_cast<size_t>(rl * rk));
    for (int64_t j = 0; j < rk; ++j) {
      const int64_t src = perm[j];
      const double s = sig[src];
      for (int64_t i = 0; i < m; ++i) U[j * m + i] = gmat[src * m + i] / s;
      int64_t imax = 0;
      for (int64_t i = 1; i < m; ++i)
        if (std::fabs(U[j * m + i]) > std::fabs(U[j * m + imax])) imax = i;
      const double sgn = (U[j * m + imax] < 0.0) ? -1.0 : 1.0;
      for (int64_t i = 0; i < m; ++i) U[j * m + i] *= sgn;
      for (int64_t a2 = 0; a2 < rl; ++a2) VS[a2 * rk + j] = sgn * V[src * rl + a2] * s;
    }
    // New core k: [rk][nk][rr] with G[j][(i,beta)] = U[(i,beta), j].
    G[k - 1] = U;  // column-major m x rk == row-major rk x m
    const int64_t rows_left = r[k - 2] * n[k - 2];
    G[k - 2] = mode3_product(G[k - 2], rows_left, rl, VS, rk);
    r[k - 1] = rk;
  }
  res->t[3] = seconds_since(t0);
  res->ranks = r;
  res->cores = std::move(G);
  res->rounded = 1;
  *out = res;
  return ORC_OK;
}

void orc_free(orc_result* r) { delete r; }

void orc_summary(const orc_result* r, int64_t* info, double* norm, double* delta) {
  info[0] = r->nnz;
  info[1] = r->rounded;
  *norm = r->norm;
  *delta = r->delta;
}

void orc_times(const orc_result* r, double* t4) {
  for (int i = 0; i < 4; ++i) t4[i] = r->t[i];
}

void orc_level_sizes(const orc_result* r, int32_t k, int64_t* sizes) {
  const LevelOut& L = r->lev[k - 1];
  sizes[0] = static_cast<int64_t>(L.col.size());
  sizes[1] = L.beta;
  sizes[2] = static_cast<int64_t>(L.row.size());
}

void orc_level(const orc_result* r, int32_t k, int64_t* col, int32_t* g, double* s,
               int64_t* n_colptr, int64_t* n_row, double* n_val) {
  const LevelOut& L = r->lev[k - 1];
  std::copy(L.col.begin(), L.col.end(), col);
  std::copy(L.g.begin(), L.g.end(), g);
  std::copy(L.s.begin(), L.s.end(), s);
  std::copy(L.colptr.begin(), L.colptr.end(), n_colptr);
  std::copy(L.row.begin(), L.row.end(), n_row);
  std::copy(L.val.begin(), L.val.end(), n_val);
}

void orc_last_exact(const orc_result* r, double* out) {
  std::copy(r->last_exact.begin(), r->last_exact.end(), out);
}

void orc_ranks(const orc_result* r, int64_t* ranks) {
  std::copy(r->ranks.begin(), r->ranks.end(), ranks);
}

void orc_qr_ranks(const orc_result* r, int64_t* ranks) {
  std::copy(r->qr_ranks.begin(), r->qr_ranks.end(), ranks);
}

void orc_core(const orc_result* r, int32_t k, double* out) {
  std::copy(r->cores[k - 1].begin(), r->cores[k - 1].end(), out);
}

int64_t orc_sigma_count(const orc_result* r, int32_t b) {
  return static_cast<int64_t>(r->sigma[b - 1].size());
}

void orc_sigma(const orc_result* r, int32_t b, double* sig, double* tail) {
  std::copy(r->sigma[b - 1].begin(), r->sigma[b - 1].end(), sig);
  *tail = r->tail[b - 1];
}

double orc_bond_delta(const orc_result* r, int32_t b) { return r->bond_delta[b - 1]; }

void orc_snap(const double* x, int64_t n, int32_t key_bits, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = snap_value(x[i], key_bits);
}

int orc_eval(int32_t d, const int64_t* dims, const int64_t* ranks, const double* const* cores,
             int64_t m, const int32_t* idx, double* y) {
  if (d < 1 || !dims || !ranks || !cores || m < 0 || (m > 0 && (!idx || !y))) return ORC_ERR_ARG;
  if (ranks[0] != 1 || ranks[d] != 1) return ORC_ERR_ARG;
  for (int64_t e = 0; e < m; ++e) {
    for (int32_t k = 0; k < d; ++k)
      if (idx[e * d + k] < 0 || idx[e * d + k] >= dims[k]) return ORC_ERR_INDEX;
    std::vector<double> left(1, 1.0);
    for (int32_t k = 0; k < d; ++k) {
      const int64_t r0 = ranks[k], r1 = ranks[k + 1], nk = dims[k], i = idx[e * d + k];
      std::vector<double> nxt(static_cast<size_t>(r1), 0.0);
      for (int64_t a = 0; a < r0; ++a)
        for (int64_t b = 0; b < r1; ++b) nxt[b] += left[a] * cores[k][(a * nk + i) * r1 + b];
      left.swap(nxt);
    }
    y[e] = left[0];
  }
  return ORC_OK;
}

int orc_eval_grad(int32_t d, const int64_t* dims, const int64_t* ranks,
                  const double* const* cores, int64_t m, const int32_t* idx, const double* gy,
                  double* const* gcores) {
  if (d < 1 || !dims || !ranks || !cores || !gcores || m < 0 || (m > 0 && (!idx || !gy)))
    return ORC_ERR_ARG;
  if (ranks[0] != 1 || ranks[d] != 1) return ORC_ERR_ARG;
  for (int32_t k = 0; k < d; ++k)
    std::fill(gcores[k], gcores[k] + ranks[k] * dims[k] * ranks[k + 1], 0.0);
  for (int64_t e = 0; e < m; ++e) {
    for (int32_t k = 0; k < d; ++k)
      if (idx[e * d + k] < 0 || idx[e * d + k] >= dims[k]) return ORC_ERR_INDEX;
    // left[k] : row vector of length ranks[k] = G1[i1]...Gk[ik]   (left[0] = [1])
    // right[k]: column vector of length ranks[k] = G_{k+1}[i_{k+1}]...Gd[id] (right[d] = [1])
    std::vector<std::vector<double>> left(d + 1), right(d + 1);
    left[0].assign(1, 1.0);
    for (int32_t k = 0; k < d; ++k) {
      const int64_t r0 = ranks[k], r1 = ranks[k + 1], nk = dims[k], i = idx[e * d + k];
      left[k + 1].assign(static_cast<size_t>(r1), 0.0);
      for (int64_t a = 0; a < r0; ++a)
        for (int64_t b = 0; b < r1; ++b) left[k + 1][b] += left[k][a] * cores[k][(a * nk + i) * r1 + b];
    }
    right[d].assign(1, 1.0);
    for (int32_t k = d - 1; k >= 0; --k) {
      const int64_t r0 = ranks[k], r1 = ranks[k + 1], nk = dims[k], i = idx[e * d + k];
      right[k].assign(static_cast<size_t>(r0), 0.0);
      for (int64_t a = 0; a < r0; ++a)
        for (int64_t b = 0; b < r1; ++b) right[k][a] += cores[k][(a * nk + i) * r1 + b] * right[k + 1][b];
    }
    for (int32_t k = 0; k < d; ++k) {
      const int64_t r0 = ranks[k], r1 = ranks[k + 1], nk = dims[k], i = idx[e * d + k];
      for (int64_t a = 0; a < r0; ++a)
        for (int64_t b = 0; b < r1; ++b)
          gcores[k][(a * nk + i) * r1 + b] += gy[e] * left[k][a] * right[k + 1][b];
    }
  }
  return ORC_OK;
}

double orc_tt_diff_norm(int32_t d, const int64_t* dims, const int64_t* ranks_a,
                        const double* const* cores_a, const int64_t* ranks_b,
                        const double* const* cores_b) {
  // TT of A - B by the TT sum lemma: C1 = [A1, -B1], Ck = diag(Ak, Bk), Cd = [Ad; Bd].
  std::vector<int64_t> r(d + 1);
  for (int32_t k = 0; k <= d; ++k) r[k] = (k == 0 || k == d) ? 1 : ranks_a[k] + ranks_b[k];
  std::vector<std::vector<double>> C(d);
  for (int32_t k = 0; k < d; ++k) {
    const int64_t nk = dims[k];
    const int64_t ra0 = ranks_a[k], ra1 = ranks_a[k + 1], rb0 = ranks_b[k], rb1 = ranks_b[k + 1];
    C[k].assign(static_cast<size_t>(r[k] * nk * r[k + 1]), 0.0);
    const int64_t offa0 = 0, offb0 = (k == 0) ? 0 : ra0;
    const int64_t offa1 = 0, offb1 = (k == d - 1) ? 0 : ra1;
    const double sb = (k == 0) ? -1.0 : 1.0;
    for (int64_t a = 0; a < ra0; ++a)
      for (int64_t i = 0; i < nk; ++i)
        for (int64_t b = 0; b < ra1; ++b)
          C[k][((offa0 + a) * nk + i) * r[k + 1] + offa1 + b] = cores_a[k][(a * nk + i) * ra1 + b];
    for (int64_t a = 0; a < rb0; ++a)
      for (int64_t i = 0; i < nk; ++i)
        for (int64_t b = 0; b < rb1; ++b)
          C[k][((offb0 + a) * nk + i) * r[k + 1] + offb1 + b] += sb * cores_b[k][(a * nk + i) * rb1 + b];
  }
  for (int32_t k = 0; k < d - 1; ++k) {
    const int64_t rows = r[k] * dims[k], cols = r[k + 1];
    std::vector<double> a(static_cast<size_t>(rows * cols));
    for (int64_t j = 0; j < cols; ++j)
      for (int64_t i = 0; i < rows; ++i) a[j * rows + i] = C[k][i * cols + j];
    std::vector<double> R;
    const int64_t p = householder_qr(rows, cols, a, nullptr, R);
    C[k + 1] = mode1_product(R, p, cols, C[k + 1], dims[k + 1] * r[k + 2]);
    r[k + 1] = p;
  }
  double s2 = 0.0;
  for (double x : C[d - 1]) s2 += x * x;
  return std::sqrt(s2);
}

}  // extern "C"
