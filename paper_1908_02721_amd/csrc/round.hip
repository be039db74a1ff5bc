// TT-rounding of the exact sparse TT: a left-to-right orthogonalisation (QR) sweep,
// then a right-to-left delta-truncated SVD sweep (Algorithm 2 run mirrored; at
// p = d the second sweep is Algorithm 6's right-to-left SVD sweep).
//
// Structure used by the left-to-right sweep.  In the exact TT built by
// parallel-vector rounding, every column of a transfer matrix T_k (one column per
// suffix (i_{k+1},...,i_d)) has exactly one nonzero -- the prefactor of that
// column in its group -- and the product of the later cores reproduces T_k
// structurally.  Hence T_k T_k^T = diag(w_k) with w_k[g] the squared norm of row g,
// and T_k = D_k Theta_k with D_k = diag(sqrt(w_k)) and Theta_k row-orthonormal.
// With the left part already orthonormal, the bond-k unfolding of A is
// (orthonormal) * (X_k D_k) * (orthonormal), X_k = W_{k-1} x_1 N_k.  So an
// orthonormal basis Q_k of X_k D_k that leaves a residual ||X_k D_k - Q Q^T X_k D_k||_F
// <= tau changes the represented tensor by exactly that residual.  The sweep uses
// this to drop directions whose whole weight is below tau (numerically zero
// directions of rank-deficient unfoldings) with a certified, exactly accounted
// error, so the later sweep works on the numerical ranks instead of the larger
// ranks of the exact sparse TT.  The basis comes from a pivoted Cholesky of the
// Gram matrix of X_k D_k and two CholeskyQR passes over the pivot columns; when the
// residual check fails (or tau = 0) the sweep falls back to an exact Householder QR.
//
// The truncated-SVD sweep orthogonalises unfold_1^T of each core (CholeskyQR2, or
// Householder when the Gram factor is ill-conditioned), takes a one-sided Jacobi
// SVD of the small R factor, keeps the smallest rank whose discarded sum of
// sigma^2 is <= delta^2 (or max_rank), makes the largest entry of every kept left
// singular vector positive and merges V*Sigma into the left neighbour.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "dense.hpp"
#include "linalg.hpp"

namespace tts {

namespace {

constexpr double kTheta = 1e-12;   // pivot threshold relative to the largest Gram diagonal
constexpr double kTauRel = 1e-13;  // per-bond deflation budget relative to ||A||_F
constexpr double kUnitRoundoff = 0x1p-53;
// largest condition number of a bond factor for which one CholeskyQR pass is kept
// (orthogonality of Q about u kOnePassCond^2 = 2e-13)
constexpr double kOnePassCond = 30.0;

__global__ void k_set_f64(double* p, double v) { *p = v; }
__global__ void k_set_i32(int32_t* p, int n, int32_t v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}


// perm[rank(j)] = j for the stable non-ascending order of s[0..n): rank(j) = number of
// i with s_i > s_j, or s_i == s_j and i < j.
// perm[r] = the index of the r-th largest sv (stable), and inv_sq[r] = 1 / sv^2 of it
// (when given)
__global__ __launch_bounds__(256) void k_rank_desc(const double* __restrict__ sv, int n, int32_t* __restrict__ perm,
                                                   double* __restrict__ inv_sq) {
  for (int j = threadIdx.x; j < n; j += 256) {
    const double x = sv[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double y = sv[i];
      r += (y > x || (y == x && i < j)) ? 1 : 0;
    }
    perm[r] = j;
    if (inv_sq) inv_sq[r] = 1.0 / (x * x);
  }
}

// A library-owned stream per device (default priority) for work off the critical
// path; ordered against the caller's stream with events only.
hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  TTS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  TTS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  streams.emplace(dev, st);
  return st;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    TTS_HIP(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    TTS_HIP(hipEventCreateWithFlags(&b, hipEventDisableTiming));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

void svd_check(const int32_t info[4], const double* sigma, int n, int rows) {
  double f2 = 0.0;
  for (int j = 0; j < n; ++j) {
    if (!std::isfinite(sigma[j])) fail(TT_ERR_NONFINITE, "a singular value of a bond factor is not finite");
    f2 += sigma[j] * sigma[j];
  }
  if (info[1]) return;
  // Stopped by the sweep cap.  Columns at the round-off floor can keep meeting the
  // relative test |a^T b| > tol ||a|| ||b||; the factors are still accurate when
  // every product rotated in the last sweep is at round-off relative to ||A||_F^2.
  double gmax;
  std::memcpy(&gmax, info + 2, sizeof(double));
  const double floor2 = static_cast<double>(std::max(rows, 16)) * 0x1p-52 * f2;
  if (gmax <= floor2) return;
  fail(TT_ERR_DEVICE, "one-sided Jacobi SVD did not converge within " + std::to_string(info[0]) +
                          " sweeps (largest rotated |a^T b| " + std::to_string(gmax / std::max(f2, 1e-300)) +
                          " of ||A||_F^2)");
}

// CholeskyQR2 of the column-major m x c matrix G: Q (m x c), R (c x c upper).
// ok[0..3] (device) are set to 0 when a Cholesky factor breaks down or is too
// ill-conditioned; nothing is read back here.  cholqr_async with passes = 1 stops
// after the first pass: Q is then orthonormal only to about u kappa(G)^2.
void cholqr2_async(Allocator* al, const double* G, int m, int c, double* Q, double* R, int32_t* ok, hipStream_t s) {
  cholqr_async(al, G, m, c, Q, R, ok, 2, s);
}

void cholqr_async(Allocator* al, const double* G, int m, int c, double* Q, double* R, int32_t* ok, int passes,
                  hipStream_t s) {
  k_set_i32<<<1, 64, 0, s>>>(ok, 4, 1);
  TTS_LAUNCH_CHECK();
  if (passes == 1) {  // R = chol(G^T G), and Q = G R^{-1} straight into Q when given
    gemm(al, true, false, c, c, m, 1.0, G, m, G, m, 0.0, R, c, s);
    cholesky_upper(R, c, c, 1e7, ok + 0, s);
    if (Q) trsm_right_upper(G, m, c, m, R, c, Q, m, ok + 1, s, al);
    return;
  }
  DBuf<double> g1(al, static_cast<size_t>(c) * c), q1(al, static_cast<size_t>(m) * c),
      g2(al, static_cast<size_t>(c) * c);
  gemm(al, true, false, c, c, m, 1.0, G, m, G, m, 0.0, g1.get(), c, s);
  cholesky_upper(g1.get(), c, c, 1e7, ok + 0, s);
  trsm_right_upper(G, m, c, m, g1.get(), c, q1.get(), m, ok + 1, s, al);
  gemm(al, true, false, c, c, m, 1.0, q1.get(), m, q1.get(), m, 0.0, g2.get(), c, s);
  cholesky_upper(g2.get(), c, c, 10.0, ok + 2, s);
  trsm_right_upper(q1.get(), m, c, m, g2.get(), c, Q, m, ok + 3, s, al);
  gemm(al, false, false, c, c, c, 1.0, g2.get(), c, g1.get(), c, 0.0, R, c, s);
}

// Truncated SVD of the column-major m x c matrix G (read only): G = Q R (m >= c) or G
// itself; one-sided Jacobi then runs on the transpose, Bt = R^T or G^T (c x cB):
// Bt U_R = V_R Sigma, so the accumulated rotations are the left singular vectors of
// R (resp. G) and the rotated columns are V Sigma, both without a division by sigma.
// (Jacobi on R^T rather than R also needs far fewer sweeps: the triangular factor
// acts as a preconditioner.)  One read-back: the singular values together with
// CholeskyQR2's success flags; on a breakdown the QR is redone with Householder.
// Rank: the smallest r >= 1 with discarded sum of sigma^2 <= delta2, or with
// max_rank > 0 min(max_rank, #nonzero sigma).  U (m x rank) and VS (c x rank) follow
// the sign rule (largest-magnitude entry of each column of U positive).
void truncated_svd(Allocator* A, int prec, const double* G, int m, int c, double delta2, int max_rank, SvdPart& o,
                   hipStream_t s) {
  DBuf<double> Qb, Bt;
  bool haveQ = false;
  int cB = m;
  Bt.reset(A, static_cast<size_t>(c) * std::min(m, c));
  // a square G takes the QR too: the Jacobi on a triangular factor needs fewer sweeps
  // and, with the one-pass QR accepted, no rotations
  if (m >= c) {
    cB = c;
    haveQ = true;
    Qb.reset(A, static_cast<size_t>(m) * c);
  }
  DBuf<double> V(A, static_cast<size_t>(cB) * cB), sig(A, cB), isq(A, cB);
  DBuf<int32_t> dperm(A, cB), okq(A, 4), jinfo(A, 4);
  std::vector<double> sh(cB);
  alignas(8) int32_t hinfo[4] = {0, 0, 0, 0};
  Readback rb(s);
  bool last_tri = false, direct = false;
  auto svd_of_bt = [&](bool lower_tri, bool want_v = true) {
    last_tri = jacobi_svd(Bt.get(), c, cB, c, V.get(), cB, sig.get(), jinfo.get(), s, lower_tri, want_v) && want_v;
    ++o.jacobi_runs;
    k_rank_desc<<<1, 256, 0, s>>>(sig.get(), cB, dperm.get(), isq.get());
    TTS_LAUNCH_CHECK();
    rb.add(sh.data(), sig.get(), sizeof(double) * cB);
    rb.add(hinfo, jinfo.get(), sizeof(hinfo));
  };
  // Bt = R^T is lower triangular: the Jacobi may leave its rotations unaccumulated and
  // form them afterwards; it says so (info[1] = -1) when that would not be accurate
  auto svd_of_r = [&]() {
    if (hinfo[1] == -1) {
      svd_of_bt(false);
      rb.sync();
    }
  };
  if (haveQ) {
    DBuf<double> R(A, static_cast<size_t>(c) * c);
    // One CholeskyQR pass first, whose Q would be orthonormal to about u kappa(G)^2,
    // enough when kappa(G) <= kOnePassCond.  The singular values read back with the
    // Jacobi (those of R = those of G; written also when the Jacobi declined to form V)
    // decide; otherwise the bond is redone with CholeskyQR2, and beyond
    // kJacobiNoVCond its Jacobi accumulates the rotations at once.
    // In FP64 the accepted pass needs neither Q nor the rotations: with Bt = R^T and
    // Bt_final = U_t Sigma the Jacobi's rotated columns, G = (Q J) Sigma U_t^T gives
    // U = Q J = G R^{-1} J = G U_t Sigma^{-1} = G Bt_final Sigma^{-2}, one product
    // accurate to about kappa(G) u (the reduced modes keep their rounded Q J).
    const bool direct_ok = prec == TT_FP64;
    cholqr_async(A, G, m, c, direct_ok ? nullptr : Qb.get(), R.get(), okq.get(), 1, s);
    o.qr_passes = 1;
    transpose(R.get(), c, c, c, Bt.get(), c, s);
    svd_of_bt(true, !direct_ok);
    int32_t okh[4];
    rb.add(okh, okq.get(), sizeof(okh));
    rb.sync();
    double smax = 0.0, smin = HUGE_VAL;
    for (double x : sh) {
      smax = std::max(smax, x);
      smin = std::min(smin, x);
    }
    // false for non-finite values of a broken-down first pass
    const bool finite = okh[0] && okh[1] && smin > 0.0 && smax < HUGE_VAL;
    const bool two = !(finite && hinfo[1] == 1 && smax <= kOnePassCond * smin);
    direct = direct_ok && !two;
    if (two) {
      const bool tri = finite && smax <= kJacobiNoVCond * smin;
      cholqr_async(A, G, m, c, Qb.get(), R.get(), okq.get(), 2, s);
      o.qr_passes = 2;
      transpose(R.get(), c, c, c, Bt.get(), c, s);
      svd_of_bt(tri);
      rb.add(okh, okq.get(), sizeof(okh));
      rb.sync();
      if (!(okh[0] && okh[1] && okh[2] && okh[3])) {
        qr_explicit(A, G, m, c, m, Qb.get(), m, R.get(), c, s);
        o.qr_passes = 3;
        transpose(R.get(), c, c, c, Bt.get(), c, s);
        svd_of_bt(tri);
        rb.sync();
      }
    }
    if (!direct) svd_of_r();
  } else {
    transpose(G, m, c, m, Bt.get(), c, s);
    svd_of_bt(false);
    rb.sync();
  }
  svd_check(hinfo, sh.data(), cB, c);
  o.v_substituted = last_tri && hinfo[1] == 1;
  o.u_direct = direct;
  o.jacobi_sweeps = hinfo[0];
  // the same stable non-ascending order as k_rank_desc
  std::vector<int32_t> perm(cB);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) { return sh[x] > sh[y]; });
  // c singular values in all (the c - cB beyond the rank bound are zero)
  std::vector<double> ss(c, 0.0), tailsum(c + 1, 0.0);
  for (int j = 0; j < cB; ++j) ss[j] = sh[perm[j]];
  for (int j = c - 1; j >= 0; --j) tailsum[j] = tailsum[j + 1] + ss[j] * ss[j];
  int rk;
  if (max_rank > 0) {
    int nz = 0;
    for (double x : ss) nz += (x > 0.0);
    rk = std::max(1, std::min(max_rank, nz));
  } else {
    rk = c;
    for (int t = 1; t <= c; ++t)
      if (tailsum[t] <= delta2) {
        rk = t;
        break;
      }
  }
  rk = std::min(rk, cB);
  o.sigma = ss;
  o.tail = tailsum[rk];
  o.rank = rk;
  DBuf<double> UR(A, static_cast<size_t>(cB) * rk);
  o.VS.reset(A, static_cast<size_t>(c) * rk);
  // direct: UR = the rotated columns scaled by 1 / sigma^2, U = G UR; otherwise UR = J
  permute_cols(direct ? Bt.get() : V.get(), direct ? c : cB, direct ? c : cB, dperm.get(), direct ? isq.get() : nullptr,
               rk, UR.get(), cB, s);
  permute_cols(Bt.get(), c, c, dperm.get(), nullptr, rk, o.VS.get(), c, s);
  o.U.reset(A, sizeof(double) * static_cast<size_t>(m) * rk);
  double* U = reinterpret_cast<double*>(o.U.get());
  if (direct)
    gemm(A, false, false, m, rk, c, 1.0, G, m, UR.get(), c, 0.0, U, m, s);
  else if (haveQ)
    gemm_prec(A, prec, false, false, m, rk, c, 1.0, Qb.get(), m, UR.get(), c, 0.0, U, m, s);
  else
    copy_matrix(UR.get(), m, rk, m, U, m, s);
  sign_fix(U, m, rk, m, o.VS.get(), c, c, s);
}

void round_tt(Allocator& al, const RoundInput& in, RoundOutput& out, hipStream_t s, hipEvent_t mid) {
  const int prec = in.precision;
  if (prec != TT_FP64 && prec != TT_FP32 && prec != TT_BF16_FP32ACC) fail(TT_ERR_ARG, "unknown precision");
  const int d = in.d;
  std::vector<int> n(d), beta(d + 1);
  for (int k = 0; k < d; ++k) n[k] = static_cast<int>(in.dims[k]);
  for (int k = 0; k <= d; ++k) beta[k] = static_cast<int>(in.betas[k]);
  for (int k = 1; k <= d; ++k) {
    const double sz = static_cast<double>(beta[k - 1]) * n[k - 1] * beta[k];
    if (beta[k] > 16384 || static_cast<double>(beta[k - 1]) * n[k - 1] > 2.0e9 || sz > 4.0e9)
      fail(TT_ERR_TOO_LARGE, "exact sparse TT too large to round on one device (bond " + std::to_string(k) + ")");
  }
  Allocator* A = &al;

  // Row norms of the transfer matrices (right parts): w[k] for bonds k = 1..d-1.
  std::vector<DBuf<double>> w(d);
  w[d - 1].reset(A, beta[d - 1]);
  row_sumsq(in.last_core, beta[d - 1], n[d - 1], w[d - 1].get(), s);
  for (int k = d - 2; k >= 1; --k) {
    w[k].reset(A, beta[k]);
    right_weights(A, in.n_colptr[k], in.n_row[k], in.n_val[k], beta[k + 1], in.n_nnz[k], n[k], beta[k],
                  w[k + 1].get(), w[k].get(), s);
  }

  // Acceptance threshold of a deflated basis.  With the tolerant parallel test the
  // exact sparse TT itself carries up to snap_rel ||A||_F of rounding (its canonical
  // values are rounded to key_bits fraction bits), so directions at that level are
  // dropped too, still within 1% of the bond's truncation threshold.  The residual
  // measures what the basis leaves out, X - Q Q^T X.  The whole left-to-right sweep
  // runs in FP64 in every precision (the basis, Q^T X and the carried factor), so
  // the same threshold certifies the deflation in the reduced modes, whose FP32/BF16
  // contractions start with the truncated SVD sweep.
  const double tau = std::min(1e-2 * in.delta, std::max(kTauRel, 4.0 * in.snap_rel) * in.norm);
  // At very small eps, 1% of delta can lie below what the residual of any FP64 basis
  // reads, the exact QR's included: about sqrt(r) u ||A||_F for a basis of r columns
  // (rounding of Q^T X and Q W').  A basis of r columns is then also accepted at
  // min(4 sqrt(r) u ||A||_F, delta / 4), which drops at most 1/16 of the bond's
  // truncation budget delta^2, so that such bonds keep their numerical rank instead
  // of taking the exact QR's full rank into the SVD sweep.
  auto tau_for = [&](int rsel) {
    if (!(tau > 0.0)) return tau;
    const double fl = std::min(4.0 * std::sqrt(static_cast<double>(rsel)) * kUnitRoundoff * in.norm,
                                  0.25 * in.delta);
    return std::min(std::max(tau, fl), std::max(kTauRel, 4.0 * in.snap_rel) * in.norm);
  };
  std::vector<int64_t> r(d + 1, 1);
  std::vector<DBuf<char>> cores(d);

  // ---------------- left-to-right sweep ----------------
  // A deflated basis is accepted on a residual test whose outcome is read back
  // together with the next bond's pivot count (one read-back per bond).  Should the
  // test fail, that bond is redone with an exact Householder QR and the bond after
  // it is recomputed from the exact factor.
  DBuf<double> W(A, 1);
  k_set_f64<<<1, 1, 0, s>>>(W.get(), 1.0);
  TTS_LAUNCH_CHECK();
  int rp = 1;
  // exact Householder QR of the bond-kb input Xb (rows x cols)
  auto exact_bond = [&](int kb, const DBuf<double>& Xb, int rows, int cols) {
    const int p = std::min(rows, cols);
    DBuf<double> Q(A, static_cast<size_t>(rows) * p), Wn(A, static_cast<size_t>(p) * cols);
    qr_explicit(A, Xb.get(), rows, cols, rows, Q.get(), rows, Wn.get(), p, s);
    cores[kb - 1].reset(A, sizeof(double) * static_cast<size_t>(rows) * p);
    transpose(Q.get(), rows, p, rows, reinterpret_cast<double*>(cores[kb - 1].get()), p, s);
    W = std::move(Wn);
    rp = p;
    r[kb] = p;
  };
  // The deflation residual of a bond is only read together with the next bond's
  // pivot count, so it runs on a side stream next to the next bond's work (the
  // single-workgroup pivoted Cholesky leaves the chip nearly idle).  Its inputs stay
  // alive in `pend` until that read, which waits for it.  With caller allocator hooks
  // (not stream-ordered) everything stays on the caller's stream.
  const bool side = !A->hook_alloc;
  const hipStream_t s2 = side ? side_stream() : s;
  Allocator al2;
  al2.stream = s2;
  al2.budget = A->budget;
  Allocator* A2 = side ? &al2 : A;
  EventPair ev;  // a: the basis and W' are ready; b: the residual is done
  struct Pending {
    bool active = false;
    int k = 0, rows = 0, cols = 0;
    double tau = 0.0;  // acceptance threshold of its basis
    DBuf<double> X, Q, e2;
    DBuf<int32_t> ok;
  } pend;
  int32_t pok[4];
  double pe2 = 0.0;
  auto pending_accepted = [&]() { return pok[1] && pok[2] && pok[3] && pe2 <= pend.tau * pend.tau; };
  int k = 1;
  double t_bond = host_ms();
  while (k <= d - 1) {
    const int nk = n[k - 1];
    const int rows = rp * nk, cols = beta[k];
    DBuf<double> X(A, static_cast<size_t>(rows) * cols);
    TTS_HIP(hipMemsetAsync(X.get(), 0, sizeof(double) * rows * cols, s));
    spmm_left(W.get(), rp, rp, in.n_colptr[k - 1], in.n_row[k - 1], in.n_val[k - 1], cols, nk, X.get(), rows, s);
    const int rmax = std::min(rows, cols);
    DBuf<double> L;
    DBuf<int32_t> piv, cnt;
    int32_t rsel = 0;
    Readback rb(s);
    if (tau > 0.0) {
      DBuf<double> Y(A, static_cast<size_t>(rows) * cols), G(A, static_cast<size_t>(cols) * cols);
      scale_cols_sqrt(X.get(), rows, cols, rows, w[k].get(), Y.get(), rows, s);
      gemm(A, true, false, cols, cols, rows, 1.0, Y.get(), rows, Y.get(), rows, 0.0, G.get(), cols, s);
      L.reset(A, static_cast<size_t>(cols) * rmax);
      piv.reset(A, rmax);
      cnt.reset(A, 1);
      pivoted_cholesky(G.get(), cols, cols, rmax, kTheta, L.get(), piv.get(), cnt.get(), s);
      rb.add(&rsel, cnt.get(), sizeof(int32_t));
    }
    if (pend.active) {
      if (side) TTS_HIP(hipStreamWaitEvent(s, ev.b, 0));
      rb.add(pok, pend.ok.get(), sizeof(pok));
      rb.add(&pe2, pend.e2.get(), sizeof(double));
    }
    if (tau > 0.0 || pend.active) rb.sync();
    if (pend.active) {
      pend.active = false;
      logf("QR bond %d: deflation to rank %lld %s (residual %.3e ||A||, threshold %.3e ||A||)", pend.k,
           static_cast<long long>(r[pend.k]), pending_accepted() ? "accepted" : "rejected, exact QR",
           std::sqrt(pe2) / in.norm, pend.tau / in.norm);
      if (!pending_accepted()) {
        exact_bond(pend.k, pend.X, pend.rows, pend.cols);
        k = pend.k + 1;  // this bond again, from the exact factor
        continue;
      }
    }
    logf("QR bond %d: %d x %d, %.3f ms (host)", k, rows, cols, host_ms() - t_bond);
    t_bond = host_ms();
    // fixed-rank truncation keeps min(max_rank, #nonzero sigma): deflating below
    // max_rank would drop numerically tiny but nonzero directions it keeps
    const bool rank_ok = in.max_rank <= 0 || rsel >= in.max_rank;
    if (tau > 0.0 && rsel > 0 && rank_ok) {
      DBuf<double> Ys(A, static_cast<size_t>(rows) * rsel), U1(A, static_cast<size_t>(rsel) * rsel),
          Q1(A, static_cast<size_t>(rows) * rsel), G2(A, static_cast<size_t>(rsel) * rsel),
          Q(A, static_cast<size_t>(rows) * rsel), Wn(A, static_cast<size_t>(rsel) * cols);
      DBuf<int32_t> ok(A, 4);
      DBuf<double> e2(A, 1);
      k_set_i32<<<1, 64, 0, s>>>(ok.get(), 4, 1);
      TTS_LAUNCH_CHECK();
      gather_cols(X.get(), rows, rows, piv.get(), rsel, w[k].get(), Ys.get(), rows, s);
      pivot_factor(L.get(), cols, piv.get(), rsel, U1.get(), s);
      trsm_right_upper(Ys.get(), rows, rsel, rows, U1.get(), rsel, Q1.get(), rows, ok.get() + 1, s, A);
      gemm(A, true, false, rsel, rsel, rows, 1.0, Q1.get(), rows, Q1.get(), rows, 0.0, G2.get(), rsel, s);
      cholesky_upper(G2.get(), rsel, rsel, 10.0, ok.get() + 2, s);
      trsm_right_upper(Q1.get(), rows, rsel, rows, G2.get(), rsel, Q.get(), rows, ok.get() + 3, s, A);
      // W' = Q^T X in FP64 in every precision: it is carried into the next bond, and a
      // rounded W' would give the next unfolding full numerical rank at the rounding
      // level, so that no deflation below that level could be certified
      gemm(A, true, false, rsel, cols, rows, 1.0, Q.get(), rows, X.get(), rows, 0.0, Wn.get(), rsel, s);
      const double* Wres = Wn.get();
      // residual of the basis, weighted by the right-part row norms (side stream)
      if (side) {
        TTS_HIP(hipEventRecord(ev.a, s));
        TTS_HIP(hipStreamWaitEvent(s2, ev.a, 0));
      }
      {
        DBuf<double> E(A2, static_cast<size_t>(rows) * cols);
        copy_matrix(X.get(), rows, cols, rows, E.get(), rows, s2);
        gemm(A2, false, false, rows, cols, rsel, -1.0, Q.get(), rows, Wres, rsel, 1.0, E.get(), rows, s2);
        weighted_sumsq(A2, E.get(), rows, cols, rows, w[k].get(), e2.get(), s2);
      }
      if (side) TTS_HIP(hipEventRecord(ev.b, s2));
      // core k = Q reshaped to [r_{k-1}][n_k][r_k] (row-major) = Q^T column-major
      cores[k - 1].reset(A, sizeof(double) * static_cast<size_t>(rows) * rsel);
      transpose(Q.get(), rows, rsel, rows, reinterpret_cast<double*>(cores[k - 1].get()), rsel, s);
      W = std::move(Wn);
      rp = rsel;
      r[k] = rsel;
      pend.active = true;
      pend.k = k;
      pend.tau = tau_for(rsel);
      pend.rows = rows;
      pend.cols = cols;
      pend.X = std::move(X);
      pend.Q = std::move(Q);
      pend.ok = std::move(ok);
      pend.e2 = std::move(e2);
    } else {
      exact_bond(k, X, rows, cols);
    }
    ++k;
  }
  if (pend.active) {  // the last bond's test
    if (side) TTS_HIP(hipStreamWaitEvent(s, ev.b, 0));
    Readback rb(s);
    rb.add(pok, pend.ok.get(), sizeof(pok));
    rb.add(&pe2, pend.e2.get(), sizeof(double));
    rb.sync();
    pend.active = false;
    if (!pending_accepted()) exact_bond(pend.k, pend.X, pend.rows, pend.cols);
  }
  {
    // last core: W (r_{d-1} x beta_{d-1}) times the exact last core (beta_{d-1} x n_d)
    const int nd = n[d - 1], bl = beta[d - 1];
    DBuf<double> C(A, static_cast<size_t>(rp) * nd);
    gemm(A, false, true, rp, nd, bl, 1.0, W.get(), rp, in.last_core, nd, 0.0, C.get(), rp, s);
    cores[d - 1].reset(A, sizeof(double) * static_cast<size_t>(rp) * nd);
    transpose(C.get(), rp, nd, rp, reinterpret_cast<double*>(cores[d - 1].get()), nd, s);
  }
  out.qr_ranks = r;
  TTS_HIP(hipEventRecord(mid, s));

  // ---------------- right-to-left truncated SVD sweep ----------------
  out.sigma.assign(d - 1, {});
  out.tail.assign(d - 1, 0.0);
  out.bond_delta.assign(d - 1, 0.0);
  // Truncation thresholds.  Fixed: delta = eps ||A||_F / sqrt(d-1) at every bond.
  // Dynamic (Algorithm 8, Sec. 3.5; with this sweep order its first loop is empty,
  // so the whole budget eps ||A||_F goes to this one sweep): with j bonds still to
  // truncate the threshold is rem / sqrt(j), and rem^2 then loses what the bond
  // discarded.  The discarded sums of all bonds stay within eps^2 ||A||_F^2.
  double rem2 = (in.eps * in.norm) * (in.eps * in.norm);
  for (int k = d; k >= 2; --k) {
    const int rl = static_cast<int>(r[k - 1]), nk = n[k - 1], rr = static_cast<int>(r[k]);
    const int m = nk * rr;
    const double delta2 = in.dynamic_delta ? rem2 / static_cast<double>(k - 1) : in.delta * in.delta;
    out.bond_delta[k - 2] = std::sqrt(delta2);
    SvdPart sv;
    truncated_svd(A, prec, reinterpret_cast<const double*>(cores[k - 1].get()), m, rl, delta2, in.max_rank, sv, s);
    logf("SVD bond %d: %d x %d, rank %d, discarded sum of sigma^2 %.3e ||A||^2 (threshold^2 %.3e), "
         "QR passes %d, Jacobi runs %d (last %d sweeps), V %s, %.3f ms (host)",
         k - 1, m, rl, sv.rank, sv.tail / (in.norm * in.norm), delta2 / (in.norm * in.norm), sv.qr_passes,
         sv.jacobi_runs, sv.jacobi_sweeps,
         sv.u_direct ? "not formed (U from G)" : (sv.v_substituted ? "by substitution" : "accumulated"),
         host_ms() - t_bond);
    t_bond = host_ms();
    out.sigma[k - 2] = std::move(sv.sigma);
    out.tail[k - 2] = sv.tail;
    rem2 = std::max(0.0, rem2 - sv.tail);
    const int rk = sv.rank;
    // core k = U (m x rk column-major = [rk][n_k][r_k] row-major); merge V*Sigma into
    // core k-1: unfold_2(G_{k-1}) (rows2 x rl) * VS (rl x rk)
    const int rows2 = static_cast<int>(r[k - 2]) * n[k - 2];
    DBuf<char> Pnew(A, sizeof(double) * static_cast<size_t>(rows2) * rk);
    gemm_prec(A, prec, true, false, rk, rows2, rl, 1.0, sv.VS.get(), rl, reinterpret_cast<double*>(cores[k - 2].get()),
              rl, 0.0, reinterpret_cast<double*>(Pnew.get()), rk, s);
    cores[k - 1] = std::move(sv.U);
    cores[k - 2] = std::move(Pnew);
    r[k - 1] = rk;
  }
  out.ranks = r;
  out.dtype = TT_DTYPE_F64;
  if (prec != TT_FP64) {
    // mixed-precision results are handed out in binary32
    for (int k = 0; k < d; ++k) {
      const size_t ne = static_cast<size_t>(r[k]) * n[k] * r[k + 1];
      DBuf<char> c32(A, sizeof(float) * ne);
      to_f32(reinterpret_cast<const double*>(cores[k].get()), ne, reinterpret_cast<float*>(c32.get()), s);
      cores[k] = std::move(c32);
    }
    out.dtype = TT_DTYPE_F32;
  }
  out.cores = std::move(cores);
}

}  // namespace tts
