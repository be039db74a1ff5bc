// Dense stage: TT-rounding of the exact sparse TT (QR sweep, truncated-SVD sweep).
#pragma once

#include <vector>

#include "common.hpp"

namespace tts {

struct RoundInput {
  int d = 0;
  std::vector<int64_t> dims;
  std::vector<int64_t> betas;              // ranks of the exact sparse TT, d+1
  double eps = 0.0, delta = 0.0, norm = 0.0;
  int max_rank = 0;
  bool dynamic_delta = false;  // per-bond thresholds from the remaining budget (Alg 8)
  double snap_rel = 0.0;       // (d-1) 2^-(key_bits+1) with the tolerant parallel test, else 0
  int precision = TT_FP64;
  // N_k (k = 1..d-1), CSC, rows rho = g_{k-1} * n_k + i_k
  std::vector<const int64_t*> n_colptr;
  std::vector<const int32_t*> n_row;
  std::vector<const double*> n_val;
  std::vector<uint32_t> n_nnz;
  const double* last_core = nullptr;       // G^(d): [beta_{d-1}][n_d]
};

struct RoundOutput {
  std::vector<int64_t> qr_ranks, ranks;
  std::vector<DBuf<char>> cores;
  int32_t dtype = TT_DTYPE_F64;
  std::vector<std::vector<double>> sigma;  // sigma[b-1]
  std::vector<double> tail;                // discarded sum of sigma^2 per bond
  std::vector<double> bond_delta;          // truncation threshold used per bond
};

// CholeskyQR2 of the column-major m x c matrix G (m >= c): Q (m x c), R (c x c upper,
// positive diagonal).  ok[0..3] (device) are set to 0 when a Cholesky factor breaks
// down or is too ill-conditioned; nothing is read back.
void cholqr2_async(Allocator* al, const double* G, int m, int c, double* Q, double* R, int32_t* ok, hipStream_t s);
// One (passes = 1) or two CholeskyQR passes; the same flags as cholqr2_async.
void cholqr_async(Allocator* al, const double* G, int m, int c, double* Q, double* R, int32_t* ok, int passes,
                  hipStream_t s);

// Truncated SVD of a column-major m x c matrix (left singular vectors U, m x rank,
// and V Sigma, c x rank, with the sign rule applied to both).
struct SvdPart {
  DBuf<char> U;                // m x rank, column-major (double)
  DBuf<double> VS;             // c x rank, column-major
  std::vector<double> sigma;   // c singular values, non-ascending
  double tail = 0.0;           // discarded sum of sigma^2
  int rank = 0;
  // the path taken: CholeskyQR passes of the final R (0: no QR, m <= c; 3: Householder
  // after CholeskyQR2 broke down), Jacobi runs, and whether the final one formed V by
  // substitution instead of accumulating the rotations
  int qr_passes = 0;
  int jacobi_runs = 0;
  int jacobi_sweeps = 0;  // sweeps of the final Jacobi run
  bool v_substituted = false;
  bool u_direct = false;  // U = G Bt_final Sigma^-2: neither Q nor V formed
};
void truncated_svd(Allocator* A, int prec, const double* G, int m, int c, double delta2, int max_rank, SvdPart& o,
                   hipStream_t s);
// Host check after a Jacobi SVD's read-back (info = the int32[4] of jacobi_svd, sigma
// its n singular values, rows the matrix's rows): TT_ERR_NONFINITE for a non-finite
// singular value; TT_ERR_DEVICE when the sweep cap stopped the iteration while a
// rotated product was still above round-off, rows u ||A||_F^2.
void svd_check(const int32_t info[4], const double* sigma, int n, int rows);

// Rounds the exact TT.  Records `mid` on the stream between the QR sweep and the
// truncated-SVD sweep.
void round_tt(Allocator& al, const RoundInput& in, RoundOutput& out, hipStream_t s, hipEvent_t mid);

// Dense exact cores [beta_{k-1}][n_k][beta_k] from N_k and the last core.
void densify_exact_cores(Allocator& al, const RoundInput& in, std::vector<DBuf<char>>& cores, hipStream_t s);

}  // namespace tts
