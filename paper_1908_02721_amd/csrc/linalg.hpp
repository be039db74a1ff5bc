// Dense FP64 building blocks of the rounding stage (gfx950).  All matrices are
// column-major with an explicit leading dimension.
#pragma once

#include "common.hpp"

namespace tts {

// Largest sigma_max / sigma_min for which the Jacobi SVD of a triangular factor forms
// V by substitution instead of accumulating the rotations (V orthonormal to about
// n u kappa).
constexpr double kJacobiNoVCond = 100.0;

// C = alpha * op(A) * op(B) + beta * C;  op(A) is m x k, op(B) is k x n.
// Split-K with a fixed-order reduction when the output is small (deterministic).
void gemm(Allocator* al, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s);
// The same product with the operands rounded to the precision `prec` (tt_precision):
// TT_FP64 as gemm; TT_FP32 binary32 operands, TT_BF16_FP32ACC bfloat16 operands, both
// on the matrix cores with binary32 accumulation.  Storage stays binary64.
void gemm_prec(Allocator* al, int prec, bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
               int lda, const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s);
// y = (float) x
void to_f32(const double* x, size_t n, float* y, hipStream_t s);

// X (rows = r * n_k, cols = ncols) = W x_1 N  with N in CSC (rows rho = g * n_k + i):
// X[a * n_k + i, b] = sum_g W[a, g] * N[g * n_k + i, b];  W is r x rw (ld ldw).
void spmm_left(const double* W, int r, int ldw, const int64_t* colptr, const int32_t* row, const double* val,
               int ncols, int nk, double* X, int ldx, hipStream_t s);

// w[g] = sum over entries (rho, b, c) of N with rho / nk == g of c^2 * wnext[b]   (deterministic)
void right_weights(Allocator* al, const int64_t* colptr, const int32_t* row, const double* val, int ncols,
                   uint32_t nnz, int nk, int ngroups, const double* wnext, double* w, hipStream_t s);
// w[g] = sum_i G[g, i]^2 for a row-major G (ngroups x nk)
void row_sumsq(const double* G, int ngroups, int nk, double* w, hipStream_t s);

// Y[:, j] = X[:, j] * sqrt(w[j])
void scale_cols_sqrt(const double* X, int rows, int cols, int ldx, const double* w, double* Y, int ldy,
                     hipStream_t s);
// Y[:, t] = X[:, piv[t]] * sqrt(w[piv[t]])  (w may be null: no scaling)
void gather_cols(const double* X, int rows, int ldx, const int32_t* piv, int r, const double* w, double* Y, int ldy,
                 hipStream_t s);

// Left-looking pivoted Cholesky of the n x n Gram matrix G: selects at most rmax
// pivots, stops when the largest remaining diagonal <= theta * max_j G_jj.
// L is n x rmax (ld n).  Writes piv[0..r) and *d_r (device int32).
void pivoted_cholesky(const double* G, int n, int ldg, int rmax, double theta, double* L, int32_t* piv, int32_t* d_r,
                      hipStream_t s);
// Upper-triangular U (r x r, ld r) = L[piv, :]^T  (the Cholesky factor of G[piv, piv]).
void pivot_factor(const double* L, int n, const int32_t* piv, int r, double* U, hipStream_t s);
// In-place Cholesky A = U^T U of an r x r SPD matrix (upper factor, lower part zeroed);
// *d_ok = 0 on breakdown or when max_j U_jj / min_j U_jj > max_ratio.
void cholesky_upper(double* A, int r, int lda, double max_ratio, int32_t* d_ok, hipStream_t s);

// X = Y U^{-1} for an upper-triangular r x r U (rows x r, column-major).
// *d_ok = 0 if U has a zero diagonal entry.
void trsm_right_upper(const double* Y, int rows, int r, int ldy, const double* U, int ldu, double* X, int ldx,
                      int32_t* d_ok, hipStream_t s, Allocator* al);

// out = sum_j w[j] * ||E[:, j]||^2  (deterministic), written to *d_out
void weighted_sumsq(Allocator* al, const double* E, int rows, int cols, int lde, const double* w, double* d_out,
                    hipStream_t s);

// Householder QR (LAPACK geqr2 conventions) in one workgroup, in place:
// R on and above the diagonal, reflectors below, tau[min(m,n)].
void householder_qr(double* A, int m, int n, int lda, double* tau, hipStream_t s);
// Economic QR of the column-major m x n matrix G (read only), Householder-based:
// Q (m x min(m, n)), R (min(m, n) x n) upper with a nonnegative diagonal.  Tall
// matrices (m >= 4 b, b = max(256, 2 n)) are factored by row blocks of b rows in
// parallel and the blocks' stacked R factors the same way (tall-skinny QR); others
// in one workgroup.
void qr_explicit(Allocator* al, const double* G, int m, int n, int ldg, double* Q, int ldq, double* R, int ldr,
                 hipStream_t s);
// Explicit Q (m x p) of the first p reflectors.
void householder_form_q(const double* A, int m, int p, int lda, const double* tau, double* Q, int ldq, hipStream_t s);
// R (p x n) from a factored A: upper part, diag made >= 0 (row signs flipped), and the
// matching column signs flipped in Q (m x p, may be null).
void householder_extract_r(const double* A, int m, int n, int lda, double* R, int ldr, double* Q, int ldq,
                           hipStream_t s);

// One-sided Jacobi SVD of the rows x c matrix A (in place: columns become u_j sigma_j),
// V (c x c) accumulates the rotations.  sigma[j] = ||A[:, j]||.  info (device int32[4],
// 8-byte aligned, may be null) receives the sweeps run, 1 if the last sweep rotated
// nothing (converged) or 0 if the sweep cap stopped it, and in info[2..3] the largest
// |a_p^T a_q| rotated in the last sweep (a double; 0 when converged).
// lower_tri: A is square and lower triangular (R^T of a QR).  For 16 < c <= 64 the
// rotations may then be left unaccumulated and V formed afterwards as A^{-1} A_final,
// when that is accurate (converged, sigma_max <= kJacobiNoVCond sigma_min); otherwise
// info[1] is set to -1, V is left unspecified, sigma holds the column norms the
// sweeps reached (the singular values when they converged), and the caller must call
// again with lower_tri = false on the original matrix (A is left unchanged then).
// want_v = false (with lower_tri): V is not needed, the 16 < c <= 64 kernels form none
// (info[1] = 1 when converged); other widths still return it.
// Returns whether the launch left the rotations unaccumulated (lower_tri honoured).
bool jacobi_svd(double* A, int rows, int c, int lda, double* V, int ldv, double* sigma, int32_t* info,
                hipStream_t s, bool lower_tri = false, bool want_v = true);

// Copy / transpose helpers.
void copy_matrix(const double* A, int rows, int cols, int lda, double* B, int ldb, hipStream_t s);
void transpose(const double* A, int rows, int cols, int lda, double* B, int ldb, hipStream_t s);
// B[:, t] = A[:, perm[t]] * (scale ? scale[t] : 1)
void permute_cols(const double* A, int rows, int lda, const int32_t* perm, const double* scale, int cols, double* B,
                  int ldb, hipStream_t s);
// Sign rule on U (rows x r): make the entry of largest magnitude of each column positive
// (lowest index on ties); the same flips are applied to the columns of VS (vrows x r).
void sign_fix(double* U, int rows, int r, int ldu, double* VS, int vrows, int ldv, hipStream_t s);

}  // namespace tts
