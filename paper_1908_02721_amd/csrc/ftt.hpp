// Fiber-trie FastTT (Algorithms 4-7 and 9): the exact rank-reduced TT of the nonzero
// p-fibers and its middle-out rounding (Algorithm 6).
#pragma once

#include <vector>

#include "common.hpp"
#include "dense.hpp"

namespace tts {

struct FttExact {
  std::vector<int64_t> ranks;        // r~_0..r~_d
  std::vector<DBuf<char>> cores;     // dense [r~_{k-1}][n_k][r~_k] (double)
  double norm = 0.0;                 // ||A||_F
  int64_t nnz = 0;                   // nonzeros kept
  int64_t fibers = 0;                // R: nonzero p-fibers
  double ms_check = 0.0, ms_build = 0.0;
};

// Validates the COO input (index range, finiteness, zeros dropped, duplicates) and
// builds the exact TT of Algorithm 4 for the given p (1..d).  Errors as
// tt_sparse_decompose (TT_ERR_INDEX > TT_ERR_NONFINITE > TT_ERR_DUPLICATE, TT_ERR_EMPTY).
void ftt_exact(Allocator* al, const int32_t* idx, const double* val, uint32_t nnz, const std::vector<int64_t>& dims,
               int p, FttExact& out, hipStream_t s);

// Algorithm 9: the p of least estimated cost (lowest on ties); the fiber counts
// R_p of every p are computed on the device.  Needs the packed coordinate to fit in
// 63 bits (else TT_ERR_TOO_LARGE).
int ftt_select_p(Allocator* al, const int32_t* idx, const double* val, uint32_t nnz, const std::vector<int64_t>& dims,
                 std::vector<double>* costs, hipStream_t s);

// Algorithm 6 on the exact cores: SVD sweep from core p to the right, QR sweep back,
// SVD sweep from core p to the left, delta = eps ||A|| / (sqrt(p-1) + sqrt(d-p));
// with dynamic, the thresholds of Algorithm 8.  prec (tt_precision): the contractions
// with the cores (merges, U = Q U_R) in that precision on the matrix cores; Grams,
// R factors, triangular solves and the SVD stay in FP64; reduced-precision results
// are handed out in binary32.
void ftt_round(Allocator* al, const std::vector<int64_t>& dims, int p, double eps, double norm, int max_rank,
               bool dynamic, int prec, std::vector<DBuf<char>>& cores, std::vector<int64_t>& ranks, RoundOutput& out,
               hipEvent_t mid, hipStream_t s);

}  // namespace tts
