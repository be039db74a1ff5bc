/*
 * ttsparse -- sparse tensor-train decomposition on AMD Instinct MI355X (gfx950).
 *
 * C-ABI of libttsparse.so.  Implements the method of arXiv 1908.02721
 * ("Faster Tensor Train Decomposition for Sparse Data"):
 *   - an exact sparse TT built by parallel-vector rounding of each mode's sparse
 *     unfolding: the TT-SVD sweep (Algorithm 1) with every truncated SVD replaced
 *     by Deparallelisation (Algorithm 3, Sec. 2.4);
 *   - TT-rounding of that TT (Algorithm 2, run mirrored: a left-to-right QR sweep,
 *     then a right-to-left delta-truncated SVD sweep; fixed-rank truncation as in
 *     Sec. 3.4);
 *   - evaluation of TT entries at given coordinates (Sec. 2.3, entry formula) and
 *     its gradient with respect to every core.
 *
 * Conventions.
 *   Indices are 0-based.  Tensors are linearised row-major, last mode fastest (the
 *   vectorisation definition of Sec. 2.2).  Core k (1..d) is a dense row-major
 *   array [r_{k-1}][n_k][r_k] with r_0 = r_d = 1, i.e. unfold_2 of the core stored
 *   row-major.  "Device" pointers are HIP device memory; "host" pointers are
 *   ordinary memory.  `stream` is a hipStream_t (NULL = the null stream).
 *
 * Errors.  Every call returns a tt_status; no exception crosses the ABI.  On error
 * no result is returned (*out = NULL) and nothing leaks.  Argument errors are found
 * on the host before any launch; data errors (index out of range, non-finite value,
 * repeated coordinate) are found on the device.  tt_last_error() returns a message
 * for the calling thread's most recent failure.
 */
#ifndef TTSPARSE_H
#define TTSPARSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_D 64

typedef enum {
  TT_OK = 0,
  TT_ERR_ARG = 1,        /* invalid argument (host check) */
  TT_ERR_INDEX = 2,      /* a coordinate is outside [0, n_k) */
  TT_ERR_DUPLICATE = 3,  /* the same coordinate appears twice among the nonzeros */
  TT_ERR_NONFINITE = 4,  /* a value is NaN or infinite */
  TT_ERR_EMPTY = 5,      /* no nonzero is left after dropping explicit zeros */
  TT_ERR_TOO_LARGE = 6,  /* a size limit of this implementation is exceeded */
  TT_ERR_NOMEM = 7,      /* device allocation failed or device_mem_budget exceeded */
  TT_ERR_DEVICE = 8      /* a HIP runtime call failed */
} tt_status;

typedef enum {
  TT_FP64 = 0,          /* every step in binary64 */
  TT_FP32 = 1,          /* dense contractions of the truncated SVD sweep in binary32
                           (MFMA, FP32 accumulate); R factors, Gram and SVD steps in
                           binary64.  The left-to-right QR sweep, whose certified
                           deflation needs the exact rank deficiency of each
                           unfolding, runs in binary64 in every precision. */
  TT_BF16_FP32ACC = 2   /* as TT_FP32 with bfloat16 operands, FP32 accumulate */
} tt_precision;

typedef enum { TT_DTYPE_F64 = 0, TT_DTYPE_F32 = 1 } tt_dtype;

typedef struct {
  int32_t precision;          /* tt_precision */
  int32_t max_rank;           /* 0: truncate by eps; > 0: fixed-rank truncation
                                 (keep min(max_rank, #nonzero sigma)), eps ignored */
  int32_t keep_intermediates; /* 1: keep per-level maps for tt_get_level */
  int32_t sparse_only;        /* 1: stop after the exact sparse TT (no rounding);
                                 tt_get_core then returns the exact cores */
  uint64_t device_mem_budget; /* 0: unlimited; else TT_ERR_NOMEM when the working
                                 set of a stage would exceed it */
  /* Optional device allocator.  NULL: stream-ordered hipMallocAsync from the
     device's default pool.  alloc returns NULL on failure. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* alloc_ctx;
  int32_t dynamic_delta;      /* 0: the same threshold eps*||A||_F/sqrt(d-1) at every
                                 bond (Algorithm 2); 1: thresholds from the budget
                                 left by the bonds already truncated (Algorithm 8,
                                 Sec. 3.5): with j bonds to go, rem/sqrt(j), then
                                 rem^2 -= the bond's discarded sum of sigma^2, from
                                 rem = eps*||A||_F.  Same eps guarantee (the
                                 correctness theorem of Algorithm 8), usually lower
                                 ranks.  Ignored with max_rank > 0. */
  int32_t key_bits;           /* 0: exact parallel test (Algorithm 3; bitwise equal
                                 canonical columns).  1..52: tolerant test: every
                                 canonical value v/s is rounded to key_bits fraction
                                 bits (round half to even on its bit pattern) before
                                 it is keyed and stored in N_k, so columns parallel
                                 up to a relative perturbation well below 2^-key_bits
                                 group together.  Each N_k entry then moves by at most
                                 2^-(key_bits+1) relative; 52 is the exact test.
                                 Outside [0, 52]: TT_ERR_ARG. */
} tt_options;

typedef struct tt_result_s* tt_result; /* opaque, owned by the library */

/* Fill *opt with the defaults: FP64, eps truncation, no intermediates, full
   rounding, no budget, the library's own allocator. */
void tt_options_default(tt_options* opt);

/*
 * Decompose the sparse tensor given in COO form.
 *   d     : order, 2 <= d <= TT_MAX_D
 *   dims  : host int64[d], 1 <= n_k <= 2^31-1; the packed coordinate
 *           sum_k ceil(log2 n_k) must not exceed 63 bits, and every level's rows
 *           g_{k-1} n_k + i_k must stay below 2^31 (beta_{k-1} n_k <= 2^31; both
 *           else TT_ERR_TOO_LARGE)
 *   nnz   : number of stored entries, 0 <= nnz < 2^31
 *   idx   : device int32[nnz][d], row-major, 0-based (borrowed, not modified)
 *   val   : device double[nnz] (borrowed, not modified).  Explicit zeros (+-0) are
 *           dropped; NaN/Inf -> TT_ERR_NONFINITE; repeated coordinate among the
 *           nonzeros -> TT_ERR_DUPLICATE; out of range -> TT_ERR_INDEX (checked in
 *           that order of precedence).
 *   eps   : relative Frobenius tolerance, 0 <= eps < 1.  The result B satisfies
 *           ||A - B||_F <= eps ||A||_F (Algorithm 2, Theorem 9), up to round-off;
 *           eps = 0 drops only zero singular values.
 *   opt   : NULL for the defaults
 *   out   : receives the result handle; release it with tt_free
 * All work is enqueued on `stream`; the call waits for its own small device-to-
 * host counts and returns when the result is complete.  With the library's own
 * allocator and no budget, the sparse stage reads back twice in all (the input
 * checks and every level's column count after the sort, then every level's group and
 * entry counts), and is redone with a read-back after the ingest and per-level reads
 * (two per level, three for a level of more than 2048 groups) when the input holds
 * explicit zeros or a level has a column of more than 32 entries or more than 2048
 * groups; with allocator hooks or a budget it always reads that way.  The rounding
 * reads back once per bond (twice when a bond's QR or SVD is redone).
 */
tt_status tt_sparse_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx,
                              const double* val, double eps, const tt_options* opt, void* stream,
                              tt_result* out);

/*
 * The paper's fiber-trie FastTT (Algorithm 7): the exact TT of the nonzero p-fibers
 * reduced by Deparallelisation of quasi-permutation matrices (Algorithm 4 with
 * Algorithm 5; the Theorem on the rank-R TT), then rounded from core p outwards
 * (Algorithm 6: truncated-SVD sweep to the right, QR sweep back, truncated-SVD sweep
 * to the left, delta = eps ||A||_F / (sqrt(p-1) + sqrt(d-p))).  The result satisfies
 * ||A - B||_F <= eps ||A||_F (Algorithm 6's correctness theorem), up to round-off.
 *   p   : 1..d, or 0 to choose it by Algorithm 9 (least estimated SVD cost, the
 *         rank bounds of Algorithm 4, f_SVD(m, n) = m n min(m, n); lowest p on ties)
 *   other arguments, inputs, errors and the result handle as tt_sparse_decompose.
 *   The exact ranks r~ of Algorithm 4 are the result's sparse ranks
 *   (tt_get_sparse_ranks: betas), the ranks after the QR sweep its qr_ranks.
 *   Options: precision (as tt_sparse_decompose: the contractions with the cores
 *   in FP32 or BF16 on the matrix cores, Grams, R factors and the SVD in FP64,
 *   cores handed out in binary32), max_rank, sparse_only (exact cores, FP64),
 *   device_mem_budget, the allocator hooks and dynamic_delta apply (Algorithm 8 as stated: budgets
 *   sqrt(d-p)/(sqrt(d-p)+sqrt(p-1)) eps ||A||_F right of p and
 *   sqrt(p-1)/(...) eps ||A||_F left of p, bond k of the right sweep gets
 *   delta_right/sqrt(d-k), bond k-1 of the left sweep delta_left/sqrt(k-1), each
 *   budget then less the bond's discarded sum of sigma^2); key_bits and
 *   keep_intermediates give TT_ERR_ARG.  Every exact rank r~_k must be <= 16384 and every exact core at most
 *   4e9 entries (else TT_ERR_TOO_LARGE): the variant suits tensors with few, dense
 *   fibers.  tt_get_level is not available.
 */
tt_status tt_fasttt_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                              double eps, int32_t p, const tt_options* opt, void* stream, tt_result* out);

/* For a tt_fasttt_decompose result: the p used and R, its number of nonzero
   p-fibers.  TT_ERR_ARG for other results. */
tt_status tt_get_fasttt_info(tt_result r, int32_t* p, int64_t* fibers);

/* Algorithm 9 alone: the chosen p and, in costs (host double[d], may be NULL), the
   estimated cost of every p = 1..d.  Inputs as tt_sparse_decompose (nnz >= 1). */
tt_status tt_fasttt_select_p(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                             double* costs, int32_t* p, void* stream);

/*
 * Bond-2 Gram slice of the orthogonalisation sweep, for tensors whose second bond
 * is too wide to factor on one device (the left-to-right QR sweep of TT-rounding,
 * Algorithm 2 in Sec. 2.4, stopped at the Gram matrix of bond 2).  After the exact
 * sparse TT (as tt_sparse_decompose):
 *   bond 1: X_1 = unfold_2(G^(1)) (n_1 x beta_1) = Q_1 R_1, an economic QR with
 *     m = min(#nonzero rows of X_1, beta_1).  The bond-1 unfolding must be wide
 *     (beta_1 >= n_1, else TT_ERR_ARG) and then leaves Q_1 free up to an orthogonal
 *     factor; the call fixes it by the SVD: Q_1 = left singular vectors, singular
 *     values non-ascending, the entry of largest magnitude of each column positive
 *     (lowest index on ties); R_1 = Q_1^T X_1.  FP64 in every precision.
 *   X_2 = unfold_2(R_1 x_1 G^(2)) ((m n_2) x beta_2), block-sparse: block (j, i)
 *     (column j, slot i = i_2) is the m-vector sum over the entries
 *     (rho = g n_2 + i, column j, value c) of N_2 of c R_1[:, g].  In TT_FP64 it is
 *     computed and stored in binary64; in TT_FP32 / TT_BF16_FP32ACC its operands are
 *     rounded to binary32 / bfloat16 (via binary32), products accumulated and
 *     stored in binary32.
 *   the weighted Gram Gamma = X_2 diag(w_2) X_2^T in FP64, w_2[j] the squared norm
 *     of row j of the right part of bond 2 (the product of the exact cores 3..d,
 *     whose rows are mutually orthogonal).  Up to the orthogonal factor Q_1 (x) I,
 *     Gamma is the Gram matrix of the bond-2 unfolding of A: its eigenvalues are
 *     that unfolding's squared singular values and its trace is ||A||_F^2.
 * Arguments, inputs, errors and the handle as tt_sparse_decompose (d >= 3,
 * n_1 <= 208); options: precision, keep_intermediates (tt_get_level), key_bits,
 * device_mem_budget and the allocator hooks apply; max_rank, dynamic_delta and
 * sparse_only give TT_ERR_ARG.  The handle answers tt_get_info, tt_get_sparse_ranks,
 * tt_get_level, tt_get_times (stage 4 = the whole slice) and the tt_get_slice_*
 * calls below; it holds no cores.  Device memory: X_2 (nblocks m values) and the
 * packed Gram (n_2 (n_2 + 1) / 2 m^2 doubles) stay allocated until tt_free.
 */
tt_status tt_sparse_gram_slice(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                               const tt_options* opt, void* stream, tt_result* out);

/* Bond 1 of a Gram slice: *m; Q_1 (device, n_1 x m column-major), R_1 (device,
   m x beta_1 column-major), singular values of X_1 (host, m, non-ascending); all
   borrowed until tt_free.  Any pointer may be NULL.  TT_ERR_ARG for other results. */
tt_status tt_get_slice_bond1(tt_result r, int64_t* m, const double** q1, const double** r1, const double** sigma);

/* X_2 of a Gram slice, blocks stored slot-major: the blocks of slot i are
   [slot_ptr[i], slot_ptr[i+1]) (device int64[n_2 + 1]), ordered by column;
   blk_col (device int32[nblocks]) is each block's column j; vals (device,
   [nblocks][m], binary64 when *dtype is TT_DTYPE_F64, else binary32) the block
   vectors.  Borrowed until tt_free; any pointer may be NULL. */
tt_status tt_get_slice_x2(tt_result r, int64_t* nblocks, const int64_t** slot_ptr, const int32_t** blk_col,
                          const void** vals, int32_t* dtype);

/* The weighted Gram of a Gram slice, packed by blocks: rows and columns are
   q = i m + a (slot i = i_2, a = the bond-1 index); only the blocks (i, i2) with
   i <= i2 are stored, block (i, i2) at element offset
   (i n_2 - i (i - 1) / 2 + (i2 - i)) m^2, as an m x m row-major matrix
   (Gamma[(i, a), (i2, a2)] at a m + a2); Gamma is symmetric.  Also: wnorm2 =
   sum over the blocks of w_2[j] ||block||^2 (= trace Gamma, in FP64), npairs = the
   number of (slot, slot) pairs of the columns of N_2 (i < i2), flops = the
   algorithmic FP64 flops of the Gram (symmetric part: m (m + 1) per diagonal-block
   term, 2 m^2 per off-diagonal pair), host_ms[5] = the slice's stage times
   (bond-1 QR, X_2, pair lists, Gram, whole slice) from HIP events.  Any pointer
   may be NULL. */
tt_status tt_get_slice_gram(tt_result r, const double** gram, double* wnorm2, int64_t* npairs, double* flops,
                            double* host_ms);

/*
 * Matrix -> tensor coordinates for the matrix-in-TT-format (MPO) front-end
 * (Sec. 3.4, matrices in TT-format).  An M x N matrix, M = m_1...m_d,
 * N = n_1...n_d, is the d-way tensor with modes of size m_k n_k: the row index
 * has digits (i_1..i_d) in the mixed radix (m_1..m_d), the column index digits
 * (j_1..j_d) in (n_1..n_d), first digit most significant, and mode k holds
 * i_k n_k + j_k.  Decomposing that tensor (tt_sparse_decompose with dims
 * m_k n_k) gives the MPO; core k reshaped to [r_{k-1}][m_k][n_k][r_k] is the
 * MPO core.
 *   d        : 1 <= d <= TT_MAX_D
 *   row_dims : host int64[d] (m_k), col_dims : host int64[d] (n_k); each >= 1 with
 *              m_k n_k <= 2^31-1 (else TT_ERR_ARG); M, N <= 2^63 (else TT_ERR_TOO_LARGE)
 *   rows, cols : device int64[nnz] (borrowed); nnz in [0, 2^31)
 *   idx      : device int32[nnz][d], caller-owned, row-major, overwritten; entry e
 *              of the output belongs to entry e of the input (values need no copy)
 * A row outside [0, M) or a column outside [0, N) gives TT_ERR_INDEX (the
 * contents of idx are then unspecified).  Enqueued on `stream`; the call waits
 * for its one 4-byte read-back of that check.
 */
tt_status tt_matrix_to_tensor(int32_t d, const int64_t* row_dims, const int64_t* col_dims, int64_t nnz,
                              const int64_t* rows, const int64_t* cols, int32_t* idx, void* stream);

/* Final TT-ranks, host int64[d+1] (r_0 = r_d = 1). */
tt_status tt_get_ranks(tt_result r, int64_t* ranks);

/* Core k (1..d): a device pointer to [r_{k-1}][n_k][r_k], borrowed until tt_free,
   and its dtype (tt_dtype; FP64 in TT_FP64 mode, FP32 otherwise). */
tt_status tt_get_core(tt_result r, int32_t k, const void** dev_ptr, int32_t* dtype);

/* Summary: host_info[0] = nonzeros kept, [1] = rounded (0/1), [2] = d;
   norm = ||A||_F; delta = per-bond threshold eps*||A||_F/sqrt(d-1). */
tt_status tt_get_info(tt_result r, int64_t* host_info, double* norm, double* delta);

/* Ranks of the exact sparse TT (beta_k, host int64[d+1]) and the ranks after the
   left-to-right QR sweep (host int64[d+1]); either pointer may be NULL. */
tt_status tt_get_sparse_ranks(tt_result r, int64_t* betas, int64_t* qr_ranks);

/* Singular values met at bond b (1..d-1) in the right-to-left sweep, sorted
   non-ascending (host, borrowed until tt_free), their count, and the discarded
   sum of squares.  Not available with sparse_only. */
tt_status tt_get_sigma(tt_result r, int32_t b, int64_t* count, const double** host_sigma,
                       double* tail);

/* Truncation threshold used at bond b (1..d-1): eps*||A||_F/sqrt(d-1), or with
   dynamic_delta the one Algorithm 8 gave that bond (unused with max_rank > 0).
   TT_ERR_ARG for a sparse_only result or b out of range. */
tt_status tt_get_bond_delta(tt_result r, int32_t b, double* delta);

/* Stage times in milliseconds (host_ms[TT_NUM_STAGES]), measured with HIP events
   on the call's stream: ingest, sort, sparse levels, QR sweep, SVD sweep, total. */
#define TT_NUM_STAGES 6
tt_status tt_get_times(tt_result r, double* host_ms);

/*
 * Level k (1..d-1) of the exact sparse stage (needs keep_intermediates):
 *   ncols      : number of unfolding columns (nnz_{k+1})
 *   beta       : number of distinct (non-parallel) columns, i.e. beta_k
 *   col        : device int64[ncols], row-major linear index of each column's
 *                suffix (i_{k+1},...,i_d); the column order is unspecified
 *   g          : device int32[ncols], group of each column (transfer-matrix row);
 *                groups are numbered by first occurrence in row-major column order
 *   s          : device double[ncols], prefactor: column = s * N_k[:, g]
 *   n_colptr   : device int64[beta+1]; n_row: device int32[]; n_val: device double[]
 *                N_k in CSC form, rows rho = g_{k-1}*n_k + i_k ascending within a
 *                column; the entry at the smallest row of every column is 1.
 * All pointers are borrowed until tt_free.
 */
tt_status tt_get_level(tt_result r, int32_t k, int64_t* ncols, int64_t* beta, const int64_t** col,
                       const int32_t** g, const double** s, const int64_t** n_colptr,
                       const int32_t** n_row, const double** n_val);

/* Sizes of level k (1..d-1) of the sparse stage, kept without keep_intermediates:
   sizes[0] = number of unfolding columns (nnz_{k+1}, the entries of level k+1),
   sizes[1] = beta_k, sizes[2] = nnz(N_k).  TT_ERR_ARG for a fiber-trie result. */
tt_status tt_get_level_sizes(tt_result r, int32_t k, int64_t* sizes);

/*
 * Device memory of the library.  Blocks that the library's calls release are kept in
 * a cache, per stream and size class, and handed out again to later work on the
 * same stream, without synchronisation; a result's blocks return there at tt_free.
 * The cache holds them until tt_cache_trim, which waits for the device to finish all
 * work and frees every cached block (*bytes_released, may be NULL, receives their
 * total).  Streams are told apart by their handles: before destroying a stream the
 * library used, synchronise it (ordinary practice), so that a later stream that
 * receives the same handle cannot race with its work; or call tt_cache_trim.
 */
tt_status tt_cache_trim(uint64_t* bytes_released);

/* Release a result (NULL is ignored). */
void tt_free(tt_result r);

/*
 * Entries of a TT at m coordinates (entry formula of Sec. 2.3):
 *   y_n = G1[0, i1, :] G2[:, i2, :] ... Gd[:, id, 0].
 *   dims, ranks : host int64[d], int64[d+1] (ranks[0] = ranks[d] = 1, each <= 256)
 *   cores       : host array of d device pointers, core k [r_{k-1}][n_k][r_k]
 *   dtype       : tt_dtype of the cores and of y_out (FP32 or FP64)
 *   idx         : device int32[m][d];  y_out: device [m] (caller-owned, written)
 * Coordinates out of range -> TT_ERR_INDEX (checked on the device, y_out then
 * undefined).
 */
tt_status tt_eval_entries(int32_t d, const int64_t* dims, const int64_t* ranks,
                          const void* const* cores, int32_t dtype, int64_t m, const int32_t* idx,
                          void* y_out, void* stream);

/*
 * Gradient of L = sum_n grad_y[n] * y_n with respect to every core:
 *   dL/dG_k[a, i, b] = sum_{n: i_k^n = i} grad_y[n] * l_{k-1}^n[a] * r_{k+1}^n[b],
 * l and r being the left and right partial products.  grad_cores: host array of d
 * device pointers shaped like the cores (caller-owned, overwritten).  The result is
 * deterministic (fixed-order reduction).
 */
tt_status tt_eval_entries_backward(int32_t d, const int64_t* dims, const int64_t* ranks,
                                   const void* const* cores, int32_t dtype, int64_t m,
                                   const int32_t* idx, const void* grad_y, void* const* grad_cores,
                                   void* stream);

/*
 * tt_eval_entries without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments, result (y_out) and errors as tt_eval_entries; the entries
 * are computed entry by entry (left-to-right chain per coordinate), so they agree
 * with tt_eval_entries to round-off of a different summation order.  The call's
 * only scratch, a 4-byte coordinate-check flag, lives in a static 256-byte device
 * array of the library (one per device, held until the process ends); its size does
 * not depend on m or the ranks, so no input is too large for it.  The flag is
 * cleared by a kernel at the start of every call.  Calls that overlap on one device
 * (other streams, other threads) share that array and race: serialise them.
 * Returns after its one 4-byte read-back of the flag.
 */
tt_status tt_eval_entries_noalloc(int32_t d, const int64_t* dims, const int64_t* ranks,
                                  const void* const* cores, int32_t dtype, int64_t m, const int32_t* idx,
                                  void* y_out, void* stream);

/*
 * Evaluation plan: the same two operations as tt_eval_entries and
 * tt_eval_entries_backward (entry formula of Sec. 2.3 and its derivative), split
 * so that work which depends only on the coordinates is done once.
 *
 * tt_eval_plan_create sorts the m coordinates idx (device int32[m][d]) and builds
 * the prefix tree of the distinct coordinate prefixes and its index buckets.  The
 * plan owns copies of everything it needs: idx may be freed once the call returns.
 * Coordinates out of range -> TT_ERR_INDEX, and *plan is left NULL.
 *
 * tt_eval_plan_forward writes y_out (device [m], caller-owned) for the TT given by
 * ranks (host int64[d+1]), cores and dtype, as tt_eval_entries does.  With
 * save != 0 the plan keeps the left partial products of this call (device memory
 * owned by the plan, replacing any kept earlier) for a later backward.
 *
 * tt_eval_plan_backward writes the gradients, as tt_eval_entries_backward does.
 * With use_saved != 0 it reuses the left partial products of the last forward
 * called with save != 0 instead of recomputing them: the ranks and dtype must
 * match that call's (TT_ERR_ARG otherwise), and the caller guarantees that the
 * core values have not changed since.  The kept products stay for further calls.
 *
 * tt_eval_plan_create returns once its work has finished.  tt_eval_plan_forward and
 * tt_eval_plan_backward called on the creation stream return once their work is
 * enqueued: outputs are ready in stream order, and the input buffers must stay
 * valid until the stream reaches them.  Called on another stream, they wait for the
 * creation stream first and return once their work has finished.  A plan may be used
 * from one thread at a time; tt_eval_plan_free releases it (NULL is ignored), and
 * work on the creation stream that uses it must have been enqueued before.
 */
typedef struct tt_eval_plan_s* tt_eval_plan;
tt_status tt_eval_plan_create(int32_t d, const int64_t* dims, int64_t m, const int32_t* idx,
                              void* stream, tt_eval_plan* plan);
tt_status tt_eval_plan_forward(tt_eval_plan plan, const int64_t* ranks, const void* const* cores,
                               int32_t dtype, void* y_out, int32_t save, void* stream);
tt_status tt_eval_plan_backward(tt_eval_plan plan, const int64_t* ranks, const void* const* cores,
                                int32_t dtype, const void* grad_y, void* const* grad_cores,
                                int32_t use_saved, void* stream);
void tt_eval_plan_free(tt_eval_plan plan);

const char* tt_status_string(tt_status s);
const char* tt_last_error(void);

/*
 * Live timing of one kernel family, for roofline reporting.  After
 * tt_kernel_timer_start(family) every launch of that family (in any call, on any
 * stream) is bracketed by two HIP events on its own stream, and the algorithmic
 * bytes and flops of the launch (what the operation must move and compute, not
 * what the implementation happens to move) are accumulated.  tt_kernel_timer_read
 * waits for the recorded events and returns the totals; family NULL or "" stops
 * timing.  Families: "sort_scatter", "level_group", "level_canon",
 * "eval_forward", "eval_up", "eval_grad", "gemm" (FP64), "gemm_lp" (FP32/BF16
 * operands), "cholesky", "trsm", "jacobi" (algorithmic flops: one sweep).
 * Process-wide, not for concurrent use from several threads.
 */
tt_status tt_kernel_timer_start(const char* family);
tt_status tt_kernel_timer_read(double* total_ms, int64_t* launches, double* algo_bytes, double* algo_flops);

#ifdef __cplusplus
}
#endif
#endif /* TTSPARSE_H */
