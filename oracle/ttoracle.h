/*
 * CPU oracle for the sparse tensor-train decomposition path (test infrastructure).
 *
 * A plain, single-threaded FP64 implementation written from the paper
 * ("Faster Tensor Train Decomposition for Sparse Data", arXiv 1908.02721).  It
 * exists only to check the HIP path: only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the HIP path.
 *
 * All indices are 0-based; tensors are linearised row-major (last mode fastest),
 * as in the paper's vectorisation definition (Sec. 2.2).  A TT core k is stored
 * dense, row-major, with shape [r_{k-1}][n_k][r_k].
 *
 * Status codes equal those of the product library's C-ABI.
 */
#ifndef TTORACLE_H
#define TTORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_ERR_ARG = 1,
  ORC_ERR_INDEX = 2,
  ORC_ERR_DUPLICATE = 3,
  ORC_ERR_NONFINITE = 4,
  ORC_ERR_EMPTY = 5,
  ORC_ERR_TOO_LARGE = 6,
};

typedef struct orc_result_s orc_result;

/* Decompose a COO tensor.
 *   idx : host int32 [nnz][d], 0-based;  val : host double [nnz]
 *   eps : relative Frobenius tolerance, 0 <= eps < 1
 *   max_rank : 0 = truncate by eps; > 0 = fixed-rank truncation (eps ignored)
 *   do_round : 0 = stop after the exact sparse TT (parallel-vector rounding);
 *              1 = also run the QR and truncated-SVD sweeps.
 *   dynamic_delta : 0 = the same threshold eps*||A||_F/sqrt(d-1) at every bond;
 *              1 = thresholds from the remaining budget (Algorithm 8).
 *   key_bits : 0 = exact parallel test; 1..52 = canonical values rounded to that
 *              many fraction bits (round half to even) before keying and storing.
 * On success *out owns every result; release with orc_free. */
int orc_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx,
                  const double* val, double eps, int32_t max_rank, int32_t do_round,
                  int32_t dynamic_delta, int32_t key_bits, orc_result** out);
/* The rounding of canonical values used with key_bits, applied to x[0..n). */
void orc_snap(const double* x, int64_t n, int32_t key_bits, double* out);
void orc_free(orc_result* r);

/* Summary.  info[0] = nnz kept, info[1] = rounded (0/1).
 * norm = ||A||_F; delta = per-bond threshold eps*||A||_F/sqrt(d-1). */
void orc_summary(const orc_result* r, int64_t* info, double* norm, double* delta);
/* Stage times in seconds: [ingest+validate, sparse levels, QR sweep, SVD sweep]. */
void orc_times(const orc_result* r, double* t4);

/* Level k (1..d-1) of the exact sparse stage.
 * sizes[0] = number of columns nnz_{k+1}, sizes[1] = beta_k, sizes[2] = nnz(N_k). */
void orc_level_sizes(const orc_result* r, int32_t k, int64_t* sizes);
/* Per column (row-major suffix order): col = row-major linear index of the
 * suffix (i_{k+1}..i_d); g = group; s = scale.  N_k in CSC (beta_k columns). */
void orc_level(const orc_result* r, int32_t k, int64_t* col, int32_t* g, double* s,
               int64_t* n_colptr, int64_t* n_row, double* n_val);
/* Exact last core G^(d) (dense [beta_{d-1}][n_d]). */
void orc_last_exact(const orc_result* r, double* out);

/* Final TT after rounding: ranks[d+1]; core k (1..d) dense. */
void orc_ranks(const orc_result* r, int64_t* ranks);
void orc_core(const orc_result* r, int32_t k, double* out);
/* Ranks after the left-to-right QR sweep (before truncation), ranks[d+1]. */
void orc_qr_ranks(const orc_result* r, int64_t* ranks);
/* Singular values seen at bond b (1..d-1) in the right-to-left sweep, sorted
 * non-ascending; count via orc_sigma_count.  tail = discarded sum of sigma^2. */
int64_t orc_sigma_count(const orc_result* r, int32_t b);
void orc_sigma(const orc_result* r, int32_t b, double* sig, double* tail);
/* Truncation threshold used at bond b (1..d-1) (unused in fixed-rank mode). */
double orc_bond_delta(const orc_result* r, int32_t b);

/* Entries y[m] of a TT at coordinates idx [m][d] (FP64). */
int orc_eval(int32_t d, const int64_t* dims, const int64_t* ranks, const double* const* cores,
             int64_t m, const int32_t* idx, double* y);
/* Gradient of sum_n gy[n] * TT(idx_n) with respect to every core (overwrites gcores). */
int orc_eval_grad(int32_t d, const int64_t* dims, const int64_t* ranks,
                  const double* const* cores, int64_t m, const int32_t* idx, const double* gy,
                  double* const* gcores);
/* ||A - B||_F of two TTs of equal mode sizes, from the TT of A - B (block cores,
 * TT sum lemma) reduced by a left-to-right Householder QR sweep. */
double orc_tt_diff_norm(int32_t d, const int64_t* dims, const int64_t* ranks_a,
                        const double* const* cores_a, const int64_t* ranks_b,
                        const double* const* cores_b);

#ifdef __cplusplus
}
#endif
#endif
