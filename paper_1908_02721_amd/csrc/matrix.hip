// Matrix -> tensor coordinates for the matrix-in-TT-format (MPO) front-end (Sec. 3.4).
//
// An M x N matrix with M = m_1 ... m_d and N = n_1 ... n_d is read as the tensor of
// order 2d with indices (i_1, j_1, ..., i_d, j_d), where (i_1..i_d) are the digits of
// the row index in the mixed radix (m_1..m_d), first digit most significant, and
// (j_1..j_d) those of the column index.  Merging each pair gives the d-way tensor
// with modes of size m_k n_k and index i_k n_k + j_k, whose TT cores, reshaped to
// [r_{k-1}][m_k][n_k][r_k], are the MPO cores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "common.hpp"

namespace tts {
namespace {

constexpr int kMT = 256;  // entries per workgroup

// Per digit: the radix, log2 of it when it is a power of two (else -1), and
// c = ceil(2^64 / radix) for the others.
struct Digit {
  uint64_t c;
  uint32_t m;
  int32_t sh;
};
struct Radix {
  Digit row[TT_MAX_D];
  Digit col[TT_MAX_D];
};

Digit make_digit(uint32_t m) {
  Digit g{0, m, -1};
  if ((m & (m - 1)) == 0) {
    g.sh = 0;
    while ((1u << g.sh) < m) ++g.sh;
  } else {
    g.c = UINT64_MAX / m + 1;  // ceil(2^64 / m): m is not a power of two
  }
  return g;
}

// q = x / m and r = x % m.  A power of two is a shift and a mask.  Otherwise, while
// x < 2^32, q = floor(c x / 2^64) with c = ceil(2^64 / m), exact for every 32-bit x
// and every m < 2^32 (Lemire, Kaser and Kurz, "Faster remainder by direct
// computation", 2019: it needs 64 >= 32 + log2 m); larger x divide in 64 bits.
__device__ __forceinline__ uint32_t divmod(uint64_t& x, const Digit& g) {
  if (g.sh >= 0) {
    const uint32_t r = static_cast<uint32_t>(x) & (g.m - 1);
    x >>= g.sh;
    return r;
  }
  if ((x >> 32) == 0) {
    const uint32_t q = static_cast<uint32_t>(__umul64hi(g.c, x));
    const uint32_t r = static_cast<uint32_t>(x) - q * g.m;
    x = q;
    return r;
  }
  const uint64_t q = x / g.m;
  const uint32_t r = static_cast<uint32_t>(x - q * g.m);
  x = q;
  return r;
}

// One thread per entry computes its d coordinates into an LDS tile (row stride
// d | 1, so that lanes of one store fall in different banks); the workgroup then
// writes the tile's kMT * d int32 to idx as 16-byte stores, consecutive lanes on
// consecutive 16-byte words (the tile starts at word e0 d, a multiple of 4 words
// since e0 is a multiple of kMT; with idx not 16-byte aligned, vec = false and
// every word is stored singly).  A row or column outside [0, M) / [0, N) raises
// bit 0 of *err.
__global__ __launch_bounds__(kMT) void k_matrix_coords(const int64_t* __restrict__ rows,
                                                       const int64_t* __restrict__ cols, int64_t nnz, int d,
                                                       uint64_t M, uint64_t N, Radix rx, int32_t* __restrict__ idx,
                                                       bool vec, uint32_t* __restrict__ err) {
  extern __shared__ int32_t tile[];
  const int ld = d | 1;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kMT;
  const int64_t e = e0 + threadIdx.x;
  bool bad = false;
  if (e < nnz) {
    const int64_t r = rows[e], c = cols[e];
    bad = r < 0 || c < 0 || static_cast<uint64_t>(r) >= M || static_cast<uint64_t>(c) >= N;
    uint64_t I = bad ? 0 : static_cast<uint64_t>(r);
    uint64_t J = bad ? 0 : static_cast<uint64_t>(c);
    for (int k = d - 1; k >= 0; --k) {
      const uint32_t ik = divmod(I, rx.row[k]);
      const uint32_t jk = divmod(J, rx.col[k]);
      tile[threadIdx.x * ld + k] = static_cast<int32_t>(ik * rx.col[k].m + jk);
    }
  }
  if (bad) atomicOr(err, 1u);
  __syncthreads();
  const int cnt = static_cast<int>(nnz - e0 < kMT ? nnz - e0 : kMT) * d;  // <= kMT * TT_MAX_D
  const int cnt4 = vec ? (cnt & ~3) : 0;
  int32_t* out = idx + e0 * d;
  // word w = 4 i + j sits at tile row t = w / d, column k = w % d; (t, k) of the
  // first word of each group is stepped by 4 kMT words, i.e. (q, r) = divmod(4 kMT, d)
  const int q = (4 * kMT) / d, r = (4 * kMT) - q * d;
  int w = 4 * static_cast<int>(threadIdx.x);
  int t = w / d, k = w - t * d;
  for (; w < cnt4; w += 4 * kMT) {
    int v[4];
    int tt = t, kk = k;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = tile[tt * ld + kk];
      if (++kk == d) {
        kk = 0;
        ++tt;
      }
    }
    *reinterpret_cast<int4*>(out + w) = make_int4(v[0], v[1], v[2], v[3]);
    t += q;
    k += r;
    if (k >= d) {
      k -= d;
      ++t;
    }
  }
  for (int w1 = cnt4 + static_cast<int>(threadIdx.x); w1 < cnt; w1 += kMT) {
    const int t1 = w1 / d;
    out[w1] = tile[t1 * ld + (w1 - t1 * d)];
  }
}

}  // namespace

tt_status matrix_coords(int32_t d, const int64_t* row_dims, const int64_t* col_dims, int64_t nnz,
                        const int64_t* rows, const int64_t* cols, int32_t* idx, hipStream_t s) {
  Radix rx{};
  unsigned __int128 M = 1, N = 1;
  for (int k = 0; k < d; ++k) {
    rx.row[k] = make_digit(static_cast<uint32_t>(row_dims[k]));
    rx.col[k] = make_digit(static_cast<uint32_t>(col_dims[k]));
    M *= static_cast<uint64_t>(row_dims[k]);
    N *= static_cast<uint64_t>(col_dims[k]);
    if (M > (static_cast<unsigned __int128>(1) << 63) || N > (static_cast<unsigned __int128>(1) << 63))
      fail(TT_ERR_TOO_LARGE, "matrix dimension M or N above 2^63");
  }
  if (nnz == 0) return TT_OK;
  Allocator al;
  al.stream = s;
  DBuf<uint32_t> err(&al, 1);
  TTS_HIP(hipMemsetAsync(err.get(), 0, sizeof(uint32_t), s));
  const int64_t blocks = (nnz + kMT - 1) / kMT;
  const size_t shm = sizeof(int32_t) * kMT * static_cast<size_t>(d | 1);
  {
    KTimer kt("mpo_coords", s, static_cast<double>(nnz) * (16.0 + 4.0 * d), 0.0);
    k_matrix_coords<<<static_cast<unsigned>(blocks), kMT, shm, s>>>(rows, cols, nnz, d, static_cast<uint64_t>(M),
                                                                     static_cast<uint64_t>(N), rx, idx,
                                                                     reinterpret_cast<uintptr_t>(idx) % 16 == 0, err.get());
    TTS_LAUNCH_CHECK();
  }
  uint32_t h = 0;
  {
    Readback rb(s);
    rb.add(&h, err.get(), sizeof(h));
    rb.sync();
  }
  if (h) fail(TT_ERR_INDEX, "a row or column index lies outside the matrix");
  return TT_OK;
}

}  // namespace tts

extern "C" tt_status tt_matrix_to_tensor(int32_t d, const int64_t* row_dims, const int64_t* col_dims, int64_t nnz,
                                         const int64_t* rows, const int64_t* cols, int32_t* idx, void* stream) {
  std::string why;
  if (d < 1 || d > TT_MAX_D) why = "d must be in [1, 64]";
  else if (!row_dims || !col_dims) why = "row_dims/col_dims is NULL";
  else if (nnz < 0 || nnz >= (int64_t(1) << 31)) why = "nnz must be in [0, 2^31)";
  else if (nnz > 0 && (!rows || !cols || !idx)) why = "rows/cols/idx is NULL";
  if (why.empty())
    for (int k = 0; k < d; ++k)
      if (row_dims[k] < 1 || col_dims[k] < 1 || row_dims[k] > INT32_MAX || col_dims[k] > INT32_MAX ||
          row_dims[k] * col_dims[k] > INT32_MAX)
        why = "every m_k, n_k must be >= 1 with m_k * n_k <= 2^31-1";
  if (!why.empty()) {
    tts::set_last_error(why);
    return TT_ERR_ARG;
  }
  try {
    return tts::matrix_coords(d, row_dims, col_dims, nnz, rows, cols, idx, static_cast<hipStream_t>(stream));
  } catch (const tts::Error& e) {
    tts::set_last_error(e.msg);
    return e.code;
  }
}
