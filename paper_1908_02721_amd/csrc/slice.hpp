// Bond-2 Gram slice of the left-to-right QR sweep (TT-rounding, Alg 2, run left to
// right) for tensors whose second bond is too wide to factor on one device.
#pragma once

#include <vector>

#include "common.hpp"

namespace tts {

struct SliceInput {
  int d = 0;
  std::vector<int64_t> dims;
  std::vector<int64_t> betas;  // ranks of the exact sparse TT, d+1
  int precision = TT_FP64;
  // N_k (k = 1..d-1), CSC, rows rho = g_{k-1} * n_k + i_k
  std::vector<const int64_t*> n_colptr;
  std::vector<const int32_t*> n_row;
  std::vector<const double*> n_val;
  std::vector<uint32_t> n_nnz;
  const double* last_core = nullptr;  // G^(d): [beta_{d-1}][n_d]
};

struct SliceOut {
  int m = 0;                  // bond-1 rank (economic QR)
  DBuf<double> q1;            // n_1 x m, column-major
  DBuf<double> r1;            // m x beta_1, column-major
  std::vector<double> sigma1; // m singular values of X_1, non-ascending
  int64_t nblocks = 0, npairs = 0;
  DBuf<int64_t> slot_ptr;     // n_2 + 1: blocks of slot i are [slot_ptr[i], slot_ptr[i+1])
  DBuf<int32_t> blk_col;      // column j of every block (ascending within a slot)
  DBuf<char> x2;              // nblocks x m values (double in FP64 mode, else float)
  int32_t x2_dtype = TT_DTYPE_F64;
  DBuf<double> gram;          // packed upper block triangle, m x m row-major blocks
  double wnorm2 = 0.0;        // sum over blocks of w_2[j] ||block||^2 (= trace of the Gram)
  double ms[5] = {};          // bond-1 QR, X_2, pair lists, Gram, whole slice
  double gram_flops = 0.0;    // algorithmic flops of the Gram (symmetric part only)
};

// Runs the slice on the exact sparse TT.  Requires d >= 3, beta_1 >= n_1 (a wide
// bond-1 unfolding) and n_1 <= 208.
void gram_slice(Allocator& al, const SliceInput& in, SliceOut& out, hipStream_t s);

}  // namespace tts
