// Dense FP64 kernels of the rounding stage (gfx950, wave64).
#include "linalg.hpp"

#include <algorithm>
#include <cstdlib>

#include "prim.hpp"

namespace tts {

namespace {

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// GEMM: 64x64 output tile per 256-thread workgroup, 4x4 register tile per
// thread (rows ty + 16r, columns tx + 16c), K staged through LDS in steps of 16.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = alpha * op(A) op(B) + beta * C on the FP64 matrix cores (column-major, op = T
// when ta / tb).  Workgroup = one 64 x 64 tile of C over the k range
// [blockIdx.z * kchunk, ...), 4 waves each owning a 32 x 32 quarter as 2 x 2 blocks
// of v_mfma_f64_16x16x4 (operand lanes: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k; accumulator register v of lane l holds row 4v + l/16, column l%16).
// Operand tiles go through LDS 16 k-steps at a time.  sym (C = A^T A): only tiles on
// or above the diagonal are computed, each written to both halves.  With `part` set,
// raw tile sums go to part[z] for a fixed-order split-K reduction.
__global__ __launch_bounds__(NT, 4) void k_gemm(int ta, int tb, int m, int n, int k, double alpha,
                                             const double* __restrict__ A, int lda, const double* __restrict__ B,
                                             int ldb, double beta, double* __restrict__ C, int ldc, int kchunk,
                                             double* __restrict__ part, int sym, int lin_tn) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  int bi = blockIdx.x, bj = blockIdx.y;
  if (lin_tn > 0) {  // blockIdx.x = bi * lin_tn + bj: a row block's column tiles run together
    bi = blockIdx.x / lin_tn;
    bj = blockIdx.x - bi * lin_tn;
  }
  if (sym) {  // blockIdx.x enumerates the tiles bi <= bj
    int rem = blockIdx.x;
    bj = 0;
    while (rem > bj) {
      rem -= bj + 1;
      ++bj;
    }
    bi = rem;
  }
  const int m0 = bi * GT, n0 = bj * GT;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  dbl4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
  // staging: all loads of a K-stage are issued together from clamped addresses and
  // masked when written to LDS; the next stage's loads go out before this stage's
  // MFMA.  Element e of a stage is A-tile entry (i, kk) and B-tile entry (kk, j),
  // enumerated so that consecutive e are consecutive in memory.
  constexpr int PL = GT * GK / NT;
  auto a_pos = [&](int e, int* i, int* kk) {
    if (!ta) {
      *i = e % GT;
      *kk = e / GT;
    } else {
      *kk = e % GK;
      *i = e / GK;
    }
  };
  auto b_pos = [&](int e, int* kk, int* j) {
    if (!tb) {
      *kk = e % GK;
      *j = e / GK;
    } else {
      *j = e % GT;
      *kk = e / GT;
    }
  };
  double av[PL], bv[PL];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = threadIdx.x + u * NT;
      int i, kk, j, kb2;
      a_pos(e, &i, &kk);
      b_pos(e, &kb2, &j);
      const int gi = m0 + i, gka = k0 + kk, gj = n0 + j, gkb = k0 + kb2;
      const bool oka = gi < m && gka < ke, okb = gj < n && gkb < ke;
      av[u] = A[oka ? (ta ? gka + static_cast<size_t>(gi) * lda : gi + static_cast<size_t>(gka) * lda) : 0];
      bv[u] = B[okb ? (tb ? gj + static_cast<size_t>(gkb) * ldb : gkb + static_cast<size_t>(gj) * ldb) : 0];
    }
  };
  if (kb < ke) load_stage(kb);
  for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = threadIdx.x + u * NT;
      int i, kk, j, kb2;
      a_pos(e, &i, &kk);
      b_pos(e, &kb2, &j);
      As[kk][i] = (m0 + i < m && k0 + kk < ke) ? (av[u]) : (0);
      Bs[kb2][j] = (n0 + j < n && k0 + kb2 < ke) ? (bv[u]) : (0);
    }
    __syncthreads();
    if (k0 + GK < ke) load_stage(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      const double a0 = As[ks + lk][wm + li], a1 = As[ks + lk][wm + 16 + li];
      const double b0 = Bs[ks + lk][wn + li], b1 = Bs[ks + lk][wn + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = m0 + wm + 16 * x + 4 * v + lk;
        const int gj = n0 + wn + 16 * y + li;
        if (gi >= m || gj >= n) continue;
        const double val = acc[x][y][v];
        const bool mirror = sym && bi < bj;
        if (part) {
          double* pz = part + static_cast<size_t>(blockIdx.z) * m * n;
          pz[gi + static_cast<size_t>(gj) * m] = val;
          if (mirror) pz[gj + static_cast<size_t>(gi) * m] = val;
        } else {
          double* cp = &C[gi + static_cast<size_t>(gj) * ldc];
          *cp = (beta == 0.0) ? alpha * val : fma(alpha, val, beta * (*cp));
          if (mirror) {
            double* cq = &C[gj + static_cast<size_t>(gi) * ldc];
            *cq = (beta == 0.0) ? alpha * val : fma(alpha, val, beta * (*cq));
          }
        }
      }
}

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Reduced-precision variant of k_gemm for the mixed-precision modes: operands are
// rounded to binary32 while staged in LDS (BF = 1: further to bfloat16, round to
// nearest even, when packed into MFMA operands) and multiplied on the matrix cores
// with binary32 accumulation -- v_mfma_f32_16x16x4_f32 (operands as in k_gemm) or
// v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16)..8(l/16)+7] and
// B[8(l/16)..+7][l%16]); both accumulate row 4(l/16)+v, column l%16 in register v.
// Storage stays binary64; split-K partials are summed in binary64.
template <int BF>
__global__ __launch_bounds__(NT) void k_gemm_lp(int ta, int tb, int m, int n, int k, double alpha,
                                                const double* __restrict__ A, int lda, const double* __restrict__ B,
                                                int ldb, double beta, double* __restrict__ C, int ldc, int kchunk,
                                                double* __restrict__ part, int sym, int lin_tn) {
  constexpr int LK = 32;
  __shared__ float As[LK][GT + 1];
  __shared__ float Bs[LK][GT + 1];
  int bi = blockIdx.x, bj = blockIdx.y;
  if (lin_tn > 0) {
    bi = blockIdx.x / lin_tn;
    bj = blockIdx.x - bi * lin_tn;
  }
  if (sym) {
    int rem = blockIdx.x;
    bj = 0;
    while (rem > bj) {
      rem -= bj + 1;
      ++bj;
    }
    bi = rem;
  }
  const int m0 = bi * GT, n0 = bj * GT;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(k, kb + kchunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  flt4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = flt4{0.f, 0.f, 0.f, 0.f};
  // staging: all loads of a K-stage are issued together from clamped addresses and
  // masked when written to LDS; the next stage's loads go out before this stage's
  // MFMA.  Element e of a stage is A-tile entry (i, kk) and B-tile entry (kk, j),
  // enumerated so that consecutive e are consecutive in memory.
  constexpr int PL = GT * LK / NT;
  auto a_pos = [&](int e, int* i, int* kk) {
    if (!ta) {
      *i = e % GT;
      *kk = e / GT;
    } else {
      *kk = e % LK;
      *i = e / LK;
    }
  };
  auto b_pos = [&](int e, int* kk, int* j) {
    if (!tb) {
      *kk = e % LK;
      *j = e / LK;
    } else {
      *j = e % GT;
      *kk = e / GT;
    }
  };
  double av[PL], bv[PL];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = threadIdx.x + u * NT;
      int i, kk, j, kb2;
      a_pos(e, &i, &kk);
      b_pos(e, &kb2, &j);
      const int gi = m0 + i, gka = k0 + kk, gj = n0 + j, gkb = k0 + kb2;
      const bool oka = gi < m && gka < ke, okb = gj < n && gkb < ke;
      av[u] = A[oka ? (ta ? gka + static_cast<size_t>(gi) * lda : gi + static_cast<size_t>(gka) * lda) : 0];
      bv[u] = B[okb ? (tb ? gj + static_cast<size_t>(gkb) * ldb : gkb + static_cast<size_t>(gj) * ldb) : 0];
    }
  };
  if (kb < ke) load_stage(kb);
  for (int k0 = kb; k0 < ke; k0 += LK) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int e = threadIdx.x + u * NT;
      int i, kk, j, kb2;
      a_pos(e, &i, &kk);
      b_pos(e, &kb2, &j);
      As[kk][i] = (m0 + i < m && k0 + kk < ke) ? static_cast<float>(av[u]) : static_cast<float>(0);
      Bs[kb2][j] = (n0 + j < n && k0 + kb2 < ke) ? static_cast<float>(bv[u]) : static_cast<float>(0);
    }
    __syncthreads();
    if (k0 + LK < ke) load_stage(k0 + LK);
    if (BF) {
      bf16x8 a0, a1, b0, b1;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0[u] = static_cast<__bf16>(As[8 * lk + u][wm + li]);
        a1[u] = static_cast<__bf16>(As[8 * lk + u][wm + 16 + li]);
        b0[u] = static_cast<__bf16>(Bs[8 * lk + u][wn + li]);
        b1[u] = static_cast<__bf16>(Bs[8 * lk + u][wn + 16 + li]);
      }
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    } else {
#pragma unroll
      for (int ks = 0; ks < LK; ks += 4) {
        const float a0 = As[ks + lk][wm + li], a1 = As[ks + lk][wm + 16 + li];
        const float b0 = Bs[ks + lk][wn + li], b1 = Bs[ks + lk][wn + 16 + li];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = m0 + wm + 16 * x + 4 * lk + v;
        const int gj = n0 + wn + 16 * y + li;
        if (gi >= m || gj >= n) continue;
        const double val = static_cast<double>(acc[x][y][v]);
        const bool mirror = sym && bi < bj;
        if (part) {
          double* pz = part + static_cast<size_t>(blockIdx.z) * m * n;
          pz[gi + static_cast<size_t>(gj) * m] = val;
          if (mirror) pz[gj + static_cast<size_t>(gi) * m] = val;
        } else {
          double* cp = &C[gi + static_cast<size_t>(gj) * ldc];
          *cp = (beta == 0.0) ? alpha * val : fma(alpha, val, beta * (*cp));
          if (mirror) {
            double* cq = &C[gj + static_cast<size_t>(gi) * ldc];
            *cq = (beta == 0.0) ? alpha * val : fma(alpha, val, beta * (*cq));
          }
        }
      }
}

__global__ __launch_bounds__(NT) void k_to_f32(const double* __restrict__ x, size_t n, float* __restrict__ y) {
  const size_t e = static_cast<size_t>(blockIdx.x) * NT + threadIdx.x;
  if (e < n) y[e] = static_cast<float>(x[e]);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_spmm_left(const double* __restrict__ W, int r, int ldw,
                                                  const int64_t* __restrict__ colptr, const int32_t* __restrict__ row,
                                                  const double* __restrict__ val, int nk, double* __restrict__ X,
                                                  int ldx) {
  const int a = blockIdx.x * NT + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= r) return;
  double* xc = X + static_cast<size_t>(b) * ldx + static_cast<size_t>(a) * nk;
  for (int64_t e = colptr[b]; e < colptr[b + 1]; ++e) {
    const int rho = row[e];
    const int g = rho / nk, i = rho - g * nk;
    xc[i] = fma(W[a + static_cast<size_t>(g) * ldw], val[e], xc[i]);
  }
}

__global__ __launch_bounds__(NT) void k_expand_cols(const int64_t* __restrict__ colptr, int ncols,
                                                    const int32_t* __restrict__ row, uint64_t* __restrict__ key,
                                                    uint64_t* __restrict__ ent, uint32_t* __restrict__ ecol) {
  const int b = blockIdx.x * NT + threadIdx.x;
  if (b >= ncols) return;
  for (int64_t e = colptr[b]; e < colptr[b + 1]; ++e) {
    key[e] = static_cast<uint64_t>(row[e]);
    ent[e] = static_cast<uint64_t>(e);
    ecol[e] = static_cast<uint32_t>(b);
  }
}

__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* a, uint32_t n, uint64_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(NT) void k_group_weights(const uint64_t* __restrict__ skey,
                                                      const uint64_t* __restrict__ sent, uint32_t nnz, int nk,
                                                      int ngroups, const double* __restrict__ val,
                                                      const uint32_t* __restrict__ ecol,
                                                      const double* __restrict__ wnext, double* __restrict__ w) {
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= ngroups) return;
  const uint32_t lo = lower_bound_u64(skey, nnz, static_cast<uint64_t>(g) * nk);
  const uint32_t hi = lower_bound_u64(skey, nnz, static_cast<uint64_t>(g + 1) * nk);
  double s = 0.0;
  for (uint32_t t = lo; t < hi; ++t) {
    const uint64_t e = sent[t];
    const double c = val[e];
    s = fma(c * c, wnext[ecol[e]], s);
  }
  w[g] = s;
}

__global__ __launch_bounds__(NT) void k_row_sumsq(const double* __restrict__ G, int ngroups, int nk,
                                                  double* __restrict__ w) {
  const int g = blockIdx.x * NT + threadIdx.x;
  if (g >= ngroups) return;
  double s = 0.0;
  for (int i = 0; i < nk; ++i) {
    const double x = G[static_cast<size_t>(g) * nk + i];
    s = fma(x, x, s);
  }
  w[g] = s;
}

__global__ __launch_bounds__(NT) void k_scale_cols(const double* __restrict__ X, int rows, int ldx,
                                                   const int32_t* __restrict__ piv, const double* __restrict__ w,
                                                   double* __restrict__ Y, int ldy) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= rows) return;
  const int j = piv ? piv[t] : t;
  const double sc = w ? sqrt(w[j]) : 1.0;
  Y[i + static_cast<size_t>(t) * ldy] = X[i + static_cast<size_t>(j) * ldx] * sc;
}

// ---------------------------------------------------------------------------
// Block-wide helpers for single-workgroup kernels (1024 threads).
// ---------------------------------------------------------------------------
constexpr int BT = 1024;

__device__ double block_sum_1024(double x, double* red) {
  x = wave_sum_f64(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < BT / 64; ++i) s += red[i];
    red[16] = s;
  }
  __syncthreads();
  s = red[16];
  __syncthreads();
  return s;
}

// Lane moves within rows of 16 lanes (DPP, no LDS round trip).  quad_perm [1,0,3,2]
// and [2,3,0,1] swap neighbours and pairs, row_half_mirror reverses each 8 lanes,
// row_mirror each 16: applied in that order, each one combines aligned groups of
// 2, 4, 8 and 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over an aligned group of G lanes (G = 1, 2, 4, 8 or 16); every lane gets it.
template <int G>
__device__ __forceinline__ double group_sum(double x) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if (G >= 2) x += dpp_move<0xB1>(x);
  if (G >= 4) x += dpp_move<0x4E>(x);
  if (G >= 8) x += dpp_move<0x141>(x);
  if (G >= 16) x += dpp_move<0x140>(x);
  return x;
}
__device__ __forceinline__ double group8_sum(double x) { return group_sum<8>(x); }

// G lanes per output: lane q sums the partials z = q (mod G) with four interleaved
// running sums, and the G lane sums are added by a DPP group sum (a fixed order), so
// that 4 G loads per output are in flight at once.
template <int G>
__global__ __launch_bounds__(NT) void k_gemm_reduce(int m, int n, int ns, const double* __restrict__ part,
                                                    double alpha, double beta, double* __restrict__ C, int ldc) {
  const size_t g = static_cast<size_t>(blockIdx.x) * NT + threadIdx.x;
  const size_t e = g / G;
  const int q = static_cast<int>(g % G);
  const size_t mn = static_cast<size_t>(m) * n;
  const bool ok = e < mn;  // the whole group of G lanes agrees
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (ok) {
    int z = q;
    for (; z + 3 * G < ns; z += 4 * G) {
      s0 += part[static_cast<size_t>(z) * mn + e];
      s1 += part[static_cast<size_t>(z + G) * mn + e];
      s2 += part[static_cast<size_t>(z + 2 * G) * mn + e];
      s3 += part[static_cast<size_t>(z + 3 * G) * mn + e];
    }
    for (; z < ns; z += G) s0 += part[static_cast<size_t>(z) * mn + e];
  }
  const double s = group_sum<G>((s0 + s1) + (s2 + s3));
  if (!ok || q != 0) return;
  const int i = static_cast<int>(e % m), j = static_cast<int>(e / m);
  double* cp = &C[i + static_cast<size_t>(j) * ldc];
  *cp = (beta == 0.0) ? alpha * s : fma(alpha, s, beta * (*cp));
}

// Three group sums at once, their moves interleaved so that they overlap.
template <int G>
__device__ __forceinline__ void group_sum3(double& a, double& b, double& c) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  {
    const double x = dpp_move<0xB1>(a), y = dpp_move<0xB1>(b), z = dpp_move<0xB1>(c);
    a += x;
    b += y;
    c += z;
  }
  {
    const double x = dpp_move<0x4E>(a), y = dpp_move<0x4E>(b), z = dpp_move<0x4E>(c);
    a += x;
    b += y;
    c += z;
  }
  {
    const double x = dpp_move<0x141>(a), y = dpp_move<0x141>(b), z = dpp_move<0x141>(c);
    a += x;
    b += y;
    c += z;
  }
  if (G == 16) {
    const double x = dpp_move<0x140>(a), y = dpp_move<0x140>(b), z = dpp_move<0x140>(c);
    a += x;
    b += y;
    c += z;
  }
}
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                          __builtin_amdgcn_readlane(__double2loint(x), lane));
}
// Largest v over the wave (NaN counts as -inf), and the lowest lane holding it.
// Every lane of the wave must be active.
__device__ __forceinline__ void wave_argmax_lane(double v, double* vmax, int* lane) {
  v = (v == v) ? v : -HUGE_VAL;
  double m = v;
  m = fmax(m, dpp_move<0xB1>(m));
  m = fmax(m, dpp_move<0x4E>(m));
  m = fmax(m, dpp_move<0x141>(m));
  m = fmax(m, dpp_move<0x140>(m));
  m = fmax(fmax(readlane_f64(m, 0), readlane_f64(m, 16)), fmax(readlane_f64(m, 32), readlane_f64(m, 48)));
  const uint64_t hit = __ballot(v == m);
  *vmax = m;
  *lane = __ffsll(static_cast<unsigned long long>(hit)) - 1;
}

// Argmax over per-wave candidates (value, index) kept in LDS: lane i of the calling
// wave reads candidate i; the largest value wins, the lowest index among equal
// values.  Every lane of the wave gets the winner.
template <int NW>
__device__ __forceinline__ void slot_argmax(const double* sv, const int* si, double* pv, int* p) {
  const int lane = threadIdx.x & 63;
  const double v = (lane < NW) ? sv[lane] : -HUGE_VAL;
  const int ix = (lane < NW) ? si[lane] : 0;
  int wl;
  wave_argmax_lane(v, pv, &wl);
  const uint64_t hit = __ballot(v == *pv);
  if (__popcll(hit) > 1) {
    int c = (v == *pv) ? ix : INT_MAX;
    for (int o = 32; o > 0; o >>= 1) c = min(c, __shfl_xor(c, o, 64));
    *p = c;
  } else {
    *p = __builtin_amdgcn_readlane(ix, wl);
  }
}

// Rotation (cs, sn) that makes two columns with squared norms a, b and inner
// product g orthogonal: the smaller-angle Jacobi rotation, tan(2 theta) = 2g / (b - a)
// with |theta| <= pi/4.  With d = b - a, e = 2g and h = sqrt(d^2 + e^2), the half-angle
// formulas give cs^2 = (h + |d|) / 2h and sn = sign(d) e / (2h cs), so
// cs = w rsqrt(w) and sn = sign(d) e (1/2h) rsqrt(w) for w = (h + |d|) / 2h: two
// reciprocal square roots and no cancellation (h + |d| adds positive numbers).
// Outside [1e-140, 1e140] for |d| and |e|, where d^2 + e^2 could overflow or lose
// its low part, Rutishauser's formulas are used instead: zeta = (b - a) / 2g,
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), cs = 1 / sqrt(1 + t^2), sn = cs t.
// Both give tan(theta) = sign(d) e / (|d| + h).  Reciprocals and reciprocal square
// roots come from the hardware estimates refined by two Newton steps (a few ulp; a
// rotation only needs cs^2 + sn^2 = 1 to rounding level, which both forms keep).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
// sqrt(x) and 1 / sqrt(x) from one refined reciprocal square root (a few ulp) for x
// in the normal range, IEEE sqrt and division outside it.
__device__ __forceinline__ void sqrt_and_rsqrt(double x, double* sq, double* inv) {
  if (x > 1e-280 && x < 1e280) {
    const double r = rsq_nr(x);
    *inv = r;
    *sq = x * r;
  } else {
    *sq = sqrt(x);
    *inv = 1.0 / *sq;
  }
}
__device__ __forceinline__ void jacobi_rotation(double a, double b, double g, double* cs, double* sn) {
  const double d = b - a, e = 2.0 * g;
  const double m = fmax(fabs(d), fabs(e));
  if (m > 1e-140 && m < 1e140) {
    const double s2 = fma(d, d, e * e);
    const double r = rsq_nr(s2);                       // 1 / h
    const double w = (fma(s2, r, fabs(d))) * (0.5 * r);  // (h + |d|) / 2h
    const double y = rsq_nr(w);
    *cs = w * y;
    *sn = (d >= 0.0 ? 0.5 : -0.5) * e * r * y;
    return;
  }
  double t;
  if (fabs(g) < 1e-290) {  // reciprocal estimates are not valid near the subnormal range
    const double zeta = (b - a) / (2.0 * g);
    t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
  } else {
    const double zeta = (b - a) * rcp_nr(2.0 * g);
    const double az = fabs(zeta);
    if (az > 1e150) {
      t = 0.5 / zeta;
    } else {
      const double q = fma(zeta, zeta, 1.0);
      const double root = q * rsq_nr(q);
      t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + root);
    }
  }
  const double c = rsq_nr(fma(t, t, 1.0));
  *cs = c;
  *sn = c * t;
}

__device__ void block_argmax_1024(double v, int idx, double* redv, int* redi, double* outv, int* outi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    redv[w] = v;
    redi[w] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = redv[0];
    int bi = redi[0];
    for (int i = 1; i < BT / 64; ++i)
      if (redv[i] > bv || (redv[i] == bv && redi[i] < bi)) {
        bv = redv[i];
        bi = redi[i];
      }
    redv[16] = bv;
    redi[16] = bi;
  }
  __syncthreads();
  *outv = redv[16];
  *outi = redi[16];
  __syncthreads();
}

// Left-looking pivoted Cholesky (dynamic LDS: n doubles for the Schur diagonal).
template <int LPJ>
__global__ __launch_bounds__(BT) void k_pivoted_cholesky(const double* __restrict__ G, int n, int ldg, int rmax,
                                                         double theta, double* __restrict__ L,
                                                         int32_t* __restrict__ piv, int32_t* __restrict__ d_r,
                                                         int tl) {
  extern __shared__ double sm[];
  double* dg = sm;      // n: diagonal of the current Schur complement (-1 once pivoted)
  double* Lc = sm + n;  // the first tl columns of L, n x tl (LDS copy)
  __shared__ double redv[17];
  __shared__ int redi[17];
  __shared__ double slotv[2][BT / 64];  // per-wave argmax candidates, double-buffered
  __shared__ int sloti[2][BT / 64];
  constexpr int PIVS = 1024;             // pivots kept in LDS until the end
  __shared__ int pivs[PIVS];
  double gmax = 0.0;
  for (int j = threadIdx.x; j < n; j += BT) {
    dg[j] = G[j + static_cast<size_t>(j) * ldg];
    gmax = fmax(gmax, dg[j]);
  }
  double mv;
  int mi;
  block_argmax_1024(gmax, 0, redv, redi, &mv, &mi);
  const double thr = theta * mv;
  // LPJ lanes share column j of the update; lane `sub` takes steps l = sub (mod LPJ)
  constexpr int JPB = BT / LPJ;
  const int sub = threadIdx.x % LPJ, jj = threadIdx.x / LPJ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int r = 0;
  for (int t = 0; t < rmax; ++t) {
    // argmax of the diagonal (largest value, lowest index on ties): each thread's own
    // candidate, a DPP wave reduction, one barrier, then every thread reduces the
    // per-wave candidates (in index order, so a tie keeps the lower index)
    double v = -1.0;
    int idx = n;
    for (int j = threadIdx.x; j < n; j += BT)
      if (dg[j] > v || (dg[j] == v && j < idx)) {
        v = dg[j];
        idx = j;
      }
    double wv;
    int wl;
    wave_argmax_lane(v, &wv, &wl);
    const int widx = __builtin_amdgcn_readlane(idx, wl);
    if (n > BT) {
      // a lane may hold a later index than another lane with the same value
      const uint64_t hit = __ballot(v == wv);
      if (__popcll(hit) > 1) {
        int c = (v == wv) ? idx : n;
        for (int o = 32; o > 0; o >>= 1) c = min(c, __shfl_xor(c, o, 64));
        if (lane == 0) sloti[t & 1][w] = c;
      } else if (lane == 0) {
        sloti[t & 1][w] = widx;
      }
    } else if (lane == 0) {
      sloti[t & 1][w] = widx;
    }
    if (lane == 0) slotv[t & 1][w] = wv;
    __syncthreads();
    double pv;
    int p;
    slot_argmax<BT / 64>(slotv[t & 1], sloti[t & 1], &pv, &p);
    if (!(pv > thr)) break;
    if (threadIdx.x == 0) {
      if (t < PIVS)
        pivs[t] = p;
      else
        piv[t] = p;
    }
    double sq, inv;
    sqrt_and_rsqrt(pv, &sq, &inv);
    for (int j0 = 0; j0 < n; j0 += JPB) {
      const int j = j0 + jj;
      const bool live = j < n && j != p && dg[min(j, n - 1)] >= 0.0;
      // the Gram entry is requested first so that its latency overlaps the dot product
      const double gjp = (live && sub == 0) ? G[j + static_cast<size_t>(p) * ldg] : 0.0;
      // s = G[j, p] - sum_{l < t} L[j, l] L[p, l], four independent partial sums;
      // steps l < tl from the LDS copy (row p read as a broadcast), the rest from memory
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      if (live) {
        const int tlim = min(t, tl);
        const double* Cj = Lc + j;
        const double* Cp = Lc + p;
        int l = sub;
        for (; l + 3 * LPJ < tlim; l += 4 * LPJ) {
          s0 = fma(Cj[l * n], Cp[l * n], s0);
          s1 = fma(Cj[(l + LPJ) * n], Cp[(l + LPJ) * n], s1);
          s2 = fma(Cj[(l + 2 * LPJ) * n], Cp[(l + 2 * LPJ) * n], s2);
          s3 = fma(Cj[(l + 3 * LPJ) * n], Cp[(l + 3 * LPJ) * n], s3);
        }
        for (; l < tlim; l += LPJ) s0 = fma(Cj[l * n], Cp[l * n], s0);
        const double* Lj = L + j;
        const double* Lp = L + p;
        for (; l + 3 * LPJ < t; l += 4 * LPJ) {
          s0 = fma(Lj[static_cast<size_t>(l) * n], Lp[static_cast<size_t>(l) * n], s0);
          s1 = fma(Lj[static_cast<size_t>(l + LPJ) * n], Lp[static_cast<size_t>(l + LPJ) * n], s1);
          s2 = fma(Lj[static_cast<size_t>(l + 2 * LPJ) * n], Lp[static_cast<size_t>(l + 2 * LPJ) * n], s2);
          s3 = fma(Lj[static_cast<size_t>(l + 3 * LPJ) * n], Lp[static_cast<size_t>(l + 3 * LPJ) * n], s3);
        }
        for (; l < t; l += LPJ) s0 = fma(Lj[static_cast<size_t>(l) * n], Lp[static_cast<size_t>(l) * n], s0);
      }
      const double acc = group_sum<LPJ>((s0 + s1) + (s2 + s3));
      if (sub == 0 && j < n) {
        double x;
        if (j == p) {
          x = sq;
          dg[j] = -1.0;
        } else if (!live) {
          x = 0.0;  // already a pivot: its Schur row is zero
        } else {
          x = (gjp - acc) * inv;
          dg[j] = dg[j] - x * x;
        }
        // columns kept in LDS go to memory after the loop, so that the barrier
        // does not wait for their stores
        if (t < tl)
          Lc[j + t * n] = x;
        else
          L[j + static_cast<size_t>(t) * n] = x;
      }
    }
    __syncthreads();
    r = t + 1;
  }
  for (int e = threadIdx.x; e < n * min(r, tl); e += BT) L[e] = Lc[e];
  for (int e = threadIdx.x; e < min(r, PIVS); e += BT) piv[e] = pivs[e];
  if (threadIdx.x == 0) *d_r = r;
}

// Left-looking pivoted Cholesky for n <= NREG * LPJ (at most 128) by NTH = n_max * LPJ
// threads: the whole Gram matrix is staged in LDS once, and the LPJ lanes of column j
// keep row j of L in registers (lane `sub` holds L[j, l] for l = sub (mod LPJ)).  A
// step costs a DPP argmax, a barrier, the pivot's row of L published to LDS, a second
// barrier, and a dot product over the t columns so far.  Same pivot rule, threshold
// and output as k_pivoted_cholesky.
template <int LPJ, int NREG, int NTH>
__global__ __launch_bounds__(NTH) void k_pivchol_lds(const double* __restrict__ G, int n, int ldg, int rmax,
                                                     double theta, double* __restrict__ L,
                                                     int32_t* __restrict__ piv, int32_t* __restrict__ d_r) {
  constexpr int NMAX = NREG * LPJ, NW = NTH / 64;
  static_assert(NMAX * LPJ == NTH, "one lane group per column");
  extern __shared__ double gs[];  // n x n, column-major
  __shared__ double prow[NMAX];
  __shared__ double slotv[2][NW];
  __shared__ int sloti[2][NW];
  __shared__ int pivs[NMAX];
  {  // staging: a thread's loads are issued together (clamped addresses)
    constexpr int PER = NMAX * NMAX / NTH;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + NTH * u, i = e % n, j = e / n;
      v[u] = G[(j < n) ? i + static_cast<size_t>(j) * ldg : 0];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + NTH * u;
      if (e < n * n) gs[e] = v[u];
    }
  }
  for (int e = threadIdx.x; e < NMAX; e += NTH) prow[e] = 0.0;
  __syncthreads();
  const int sub = threadIdx.x % LPJ, j = threadIdx.x / LPJ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double dj = (j < n) ? gs[j + j * n] : -1.0;  // Schur diagonal of column j (-1 once pivoted)
  double thr;
  {  // threshold: theta times the largest diagonal entry of G
    double wv;
    int wl;
    wave_argmax_lane(j < n ? dj : 0.0, &wv, &wl);
    if (lane == 0) slotv[1][w] = wv;
    __syncthreads();
    double mv;
    int unused;
    slot_argmax<NW>(slotv[1], sloti[1], &mv, &unused);
    thr = theta * mv;
    __syncthreads();
  }
  double lr[NREG];
#pragma unroll
  for (int u = 0; u < NREG; ++u) lr[u] = 0.0;
  int r = 0;
  for (int t = 0; t < rmax; ++t) {
    double wv;
    int wl;
    wave_argmax_lane(dj, &wv, &wl);
    if (lane == 0) {
      slotv[t & 1][w] = wv;
      sloti[t & 1][w] = (w * 64 + wl) / LPJ;
    }
    __syncthreads();
    double pv;
    int p;
    slot_argmax<NW>(slotv[t & 1], sloti[t & 1], &pv, &p);
    if (!(pv > thr)) break;
    if (threadIdx.x == 0) pivs[t] = p;
    if (j == p) {
#pragma unroll
      for (int u = 0; u < NREG; ++u) prow[sub + u * LPJ] = lr[u];
    }
    __syncthreads();
    double sq, inv;
    sqrt_and_rsqrt(pv, &sq, &inv);
    const double gjp = gs[min(j, n - 1) + p * n];
    // sum over l < t of L[j, l] L[p, l]: this lane's terms l = sub + u LPJ, u < ul
    const int ul = (t + LPJ - 1) / LPJ;
    // in groups of four terms (entries past t are zero on both sides), each group's
    // loads issued together
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int u = 0; u < NREG; u += 4) {
      if (u < ul) {
        const double p0 = prow[sub + u * LPJ], p1 = prow[sub + (u + 1) * LPJ];
        const double p2 = prow[sub + (u + 2) * LPJ], p3 = prow[sub + (u + 3) * LPJ];
        s0 = fma(lr[u], p0, s0);
        s1 = fma(lr[u + 1], p1, s1);
        s0 = fma(lr[u + 2], p2, s0);
        s1 = fma(lr[u + 3], p3, s1);
      }
    }
    const double s = group_sum<LPJ>(s0 + s1);
    double x = 0.0;
    if (j == p) {
      x = sq;
      dj = -1.0;
    } else if (j < n && dj >= 0.0) {
      x = (gjp - s) * inv;
      dj = dj - x * x;
    }
    // columns already pivoted (dj = -1), or whose Schur diagonal has gone negative by
    // rounding, keep dj and get a zero entry
    const int ut = t / LPJ, st = t % LPJ;
#pragma unroll
    for (int u = 0; u < NREG; ++u)
      if (u == ut && sub == st) lr[u] = x;
    r = t + 1;
  }
  // the loop touches no global memory, so its barriers never wait for stores: L and
  // the pivots are written once, here
  __syncthreads();
  if (j < n) {
#pragma unroll
    for (int u = 0; u < NREG; ++u) {
      const int l = sub + u * LPJ;
      if (l < r) L[j + static_cast<size_t>(l) * n] = lr[u];
    }
  }
  for (int t = threadIdx.x; t < r; t += NTH) piv[t] = pivs[t];
  if (threadIdx.x == 0) *d_r = r;
}

// Blocked left-looking pivoted Cholesky by one PB_NTH-thread workgroup.  A round takes
// up to PB_KB candidates at once: the live column of largest Schur diagonal d_max
// (lowest index on ties) and, in index order, the other live columns with
// d_j >= PB_GAMMA d_max.  One wave factors the candidates' Schur block in that order,
// accepting a candidate only while its updated diagonal is still above the threshold
// and >= PB_GAMMA d_max, and every other column's new entries follow from one
// triangular solve with the accepted pivots' factor.  So each pivot's diagonal is
// within PB_GAMMA of the largest Schur diagonal at its step (threshold pivoting;
// greedy pivoting is PB_GAMMA = 1), with five barriers a round instead of two per
// pivot.  Same threshold, stopping rule and output layout as k_pivoted_cholesky
// (L is n x r with leading dimension n, piv[t] the column of pivot t); the pivots may
// come in another order.  Dynamic LDS: the Schur diagonal (n doubles) and the
// candidates' rows of L (PB_KB x rmax doubles).
constexpr int PB_NTH = 512, PB_KB = 8;  // KB * KB = one wave
constexpr int PB_QT = 2;                 // 16-row tiles a wave takes at a time
constexpr int PB_KS = 4;                // matrix-core steps (of 4 columns) per load batch
constexpr double PB_GAMMA = 0.25;
__global__ __launch_bounds__(PB_NTH) void k_pivchol_block(const double* __restrict__ G, int n, int ldg, int rmax,
                                                          double theta, double* __restrict__ L,
                                                          int32_t* __restrict__ piv, int32_t* __restrict__ d_r) {
  constexpr int NTH = PB_NTH, NW = NTH / 64, KB = PB_KB, SQ = NTH / (KB * KB);
  static_assert(KB * KB == 64 && SQ >= 1 && SQ <= 16, "one wave holds the candidates' block");
  extern __shared__ double sm[];
  double* dg = sm;         // n: Schur diagonal, -1 once pivoted
  double* crow = sm + n;   // KB x rmax: the candidates' rows of L (entries l < t)
  __shared__ double S[KB][KB];    // the candidates' Schur block (lower part)
  __shared__ double Lpp[KB][KB];  // factor of the accepted pivots, in acceptance order
  __shared__ double rdg[KB];      // 1 / Lpp[i][i]
  __shared__ double Ht[NW][16 * PB_QT][KB + 1];  // each wave's products, padded
  __shared__ int cand[KB], pcand[KB], pcol[KB];  // candidates; accepted i -> candidate, column
  __shared__ int nctl[2];                        // candidates, accepted
  __shared__ double slotv[NW];
  __shared__ int sloti[NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // the diagonal of G, its largest entry and column (lowest index on ties), every thread
  auto block_argmax = [&](double* pv, int* pi) {
    double v = -1.0;
    int idx = n;
    for (int j = threadIdx.x; j < n; j += NTH) {
      const double x = G[j + static_cast<size_t>(j) * ldg];
      dg[j] = x;
      if (x > v) {
        v = x;
        idx = j;
      }
    }
    double wv;
    int wl;
    wave_argmax_lane(v, &wv, &wl);
    int widx = __builtin_amdgcn_readlane(idx, wl);
    if (n > NTH) {  // a lower lane may hold a later index with the same value
      int c = (v == wv) ? idx : n;
      for (int o = 32; o > 0; o >>= 1) c = min(c, __shfl_xor(c, o, 64));
      widx = c;
    }
    if (lane == 0) {
      slotv[w] = wv;
      sloti[w] = widx;
    }
    __syncthreads();
    slot_argmax<NW>(slotv, sloti, pv, pi);
  };
  double dmax;
  int am;
  block_argmax(&dmax, &am);
  const double thr = theta * dmax;
  int t = 0;
  for (;;) {
    if (t > 0) slot_argmax<NW>(slotv, sloti, &dmax, &am);  // written by the last round
    if (!(dmax > thr) || t >= rmax) break;  // uniform
    const int cap = min(KB, rmax - t);
    // candidates: the largest first, then the others >= PB_GAMMA d_max in index order
    if (w == 0) {
      int cnt = 1;
      for (int j0 = 0; j0 < n && cnt < cap; j0 += 64) {
        const int j = j0 + lane;
        const double x = (j < n) ? dg[j] : -1.0;
        const bool c = j != am && x > thr && x >= PB_GAMMA * dmax;
        const uint64_t m = __ballot(c);
        const int pos = cnt + __popcll(m & lanemask_lt());
        if (c && pos < cap) cand[pos] = j;
        cnt = min(cap, cnt + __popcll(m));
      }
      if (lane == 0) {
        cand[0] = am;
        nctl[0] = cnt;
      }
    }
    __syncthreads();
    const int nc = nctl[0];
    // their rows of L so far
    for (int e = threadIdx.x; e < nc * t; e += NTH) {
      const int a = e / t, l = e - a * t;
      crow[a * rmax + l] = L[cand[a] + static_cast<size_t>(l) * n];
    }
    __syncthreads();
    {  // their Schur block, SQ lanes an entry
      const int e = threadIdx.x / SQ, q = threadIdx.x % SQ, a = e / KB, b = e % KB;
      const bool ok = a < nc && b < nc;
      const double g = ok ? G[cand[a] + static_cast<size_t>(cand[b]) * ldg] : 0.0;
      double acc = 0.0;
      if (ok)
        for (int l = q; l < t; l += SQ) acc = fma(crow[a * rmax + l], crow[b * rmax + l], acc);
      acc = group_sum<SQ>(acc);
      if (q == 0) S[a][b] = ok ? g - acc : 0.0;
    }
    __syncthreads();
    if (w == 0) {
      // lane (a, c) = (lane / KB, lane % KB) holds entry (a, c) of the candidates' Schur
      // block, factored in candidate order; a candidate is accepted while its diagonal
      // qualifies.  At step p lane (a, p) keeps l_a = S[a][p] / sqrt(S[p][p]).
      const int a = lane / KB, c = lane % KB;
      double sv = S[a][c], myl = 0.0, myinv = 0.0;
      int na = 0;
      uint32_t accm = 0;
#pragma unroll
      for (int p = 0; p < KB; ++p) {
        if (p < nc) {
          const double spp = readlane_f64(sv, p * KB + p);
          if (spp > thr && spp >= PB_GAMMA * dmax && na < cap) {
            double sq, inv;
            sqrt_and_rsqrt(spp, &sq, &inv);
            const double la = __shfl(sv, a * KB + p, 64) * inv;
            const double lc = __shfl(sv, c * KB + p, 64) * inv;
            if (c == p) {
              myl = sv * inv;
              myinv = inv;
            }
            sv = fma(-la, lc, sv);
            if (lane == 0) {
              pcand[na] = p;
              pcol[na] = cand[p];
            }
            accm |= 1u << p;
            ++na;
          }
        }
      }
      // the accepted rows of the factor, in acceptance order, zero elsewhere (above
      // the diagonal and in the rows and columns of unused slots)
      Lpp[a][c] = 0.0;
      if (lane < KB) rdg[lane] = 0.0;
      if (((accm >> a) & 1u) && ((accm >> c) & 1u)) {
        const int ia = __popc(accm & ((1u << a) - 1u)), ic = __popc(accm & ((1u << c) - 1u));
        Lpp[ia][ic] = (ic <= ia) ? myl : 0.0;
        if (a == c) rdg[ia] = myinv;
      }
      if (lane == 0) nctl[1] = na;
    }
    __syncthreads();
    const int b = nctl[1];
    if (b == 0) break;  // uniform: no candidate qualified after rounding
    // The new entries t .. t + b - 1 of every row j: H[j][i] = sum_{l < t} L[j, l]
    // L[p_i, l] on the FP64 matrix cores, a wave taking PB_QT tiles of 16 rows at a
    // time (A = rows of L from memory, B = the accepted pivots' rows, zero past slot
    // b), then each lane solves one of those rows: x = (G[j, P] - H[j]) Lpp^-T.  Slots
    // i >= b meet zero rows and columns of Lpp and so give zero.  The lanes also
    // track the largest new Schur diagonal of their rows for the next round.
    {
      const int li = lane & 15, lk = lane >> 4;
      const double* crb = crow + pcand[min(li, b - 1)] * rmax;
      const bool bok = li < b;
      int pc[KB];
#pragma unroll
      for (int i = 0; i < KB; ++i) pc[i] = pcol[min(i, b - 1)];
      double bestv = -1.0;
      int besti = n;
      for (int p0 = 0; p0 < n; p0 += NW * PB_QT * 16) {
        const int wr0 = p0 + w * PB_QT * 16;  // this wave's first row in this pass
        if (wr0 >= n) break;                   // uniform within the wave
        const int nq = min(PB_QT, (n - wr0 + 15) / 16);
        const int j = wr0 + lane;  // the row this lane solves
        const bool solver = lane < 16 * nq && j < n;
        const double dj = solver ? dg[j] : -1.0;
        int pr = -1;
#pragma unroll
        for (int i = 0; i < KB; ++i)
          if (i < b && pc[i] == j) pr = i;
        const bool live = solver && pr < 0 && dj >= 0.0;
        double gv[KB];  // requested first, so that their latency overlaps the products
#pragma unroll
        for (int i = 0; i < KB; ++i) gv[i] = live ? G[j + static_cast<size_t>(pc[i]) * ldg] : 0.0;
        dbl4 acc[PB_QT];
#pragma unroll
        for (int q = 0; q < PB_QT; ++q) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
        // PB_KS steps of four at a time, all their loads issued together (the loads'
        // latency, not the products, bounds this phase)
        for (int k0 = 0; k0 < t; k0 += 4 * PB_KS) {
          double av[PB_QT][PB_KS], bv[PB_KS];
#pragma unroll
          for (int u = 0; u < PB_KS; ++u) {
            const int l = k0 + 4 * u + lk, lc = min(l, t - 1);
            const double bb = crb[lc];
            bv[u] = (l < t && bok) ? bb : 0.0;
#pragma unroll
            for (int q = 0; q < PB_QT; ++q) {
              const int ar = min(wr0 + 16 * q + li, n - 1);  // clamped: computed, not used
              const double a = (q < nq) ? L[ar + static_cast<size_t>(lc) * n] : 0.0;
              av[q][u] = (l < t) ? a : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < PB_KS; ++u)
            if (k0 + 4 * u < t)
#pragma unroll
              for (int q = 0; q < PB_QT; ++q)
                if (q < nq) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q][u], bv[u], acc[q], 0, 0, 0);
        }
        // accumulator v of lane (li, lk) in tile q is H[wr0 + 16q + 4v + lk][li]: through
        // LDS to the solving lanes (the wave's own buffer: LDS keeps a wave's order)
        if (li < KB) {
#pragma unroll
          for (int q = 0; q < PB_QT; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) Ht[w][16 * q + 4 * v + lk][li] = acc[q][v];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (solver) {
          double x[KB];
          if (pr >= 0) {
#pragma unroll
            for (int i = 0; i < KB; ++i) x[i] = Lpp[pr][i];
          } else if (live) {
#pragma unroll
            for (int i = 0; i < KB; ++i) {
              double r = gv[i] - Ht[w][lane][i];
#pragma unroll
              for (int k = 0; k < i; ++k) r = fma(-x[k], Lpp[i][k], r);
              x[i] = r * rdg[i];
            }
          } else {
#pragma unroll
            for (int i = 0; i < KB; ++i) x[i] = 0.0;  // pivoted earlier, or negative by rounding
          }
          double dn = dj;
#pragma unroll
          for (int i = 0; i < KB; ++i) {
            if (i < b) L[j + static_cast<size_t>(t + i) * n] = x[i];
            dn = fma(-x[i], x[i], dn);
          }
          const double dnew = (pr >= 0) ? -1.0 : (live ? dn : dj);
          dg[j] = dnew;
          if (dnew > bestv) {  // rows of later passes have higher indices
            bestv = dnew;
            besti = j;
          }
        }
        // the tile buffer is reused by the next pass
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // this wave's largest new diagonal (lowest index on ties) for the next round
      double wv;
      int wl;
      wave_argmax_lane(bestv, &wv, &wl);
      int c = (bestv == wv) ? besti : n;
      for (int o = 32; o > 0; o >>= 1) c = min(c, __shfl_xor(c, o, 64));
      if (lane == 0) {
        slotv[w] = wv;
        sloti[w] = c;
      }
    }
    if (threadIdx.x < b) piv[t + threadIdx.x] = pcol[threadIdx.x];
    t += b;
    __syncthreads();
  }
  if (threadIdx.x == 0) *d_r = t;
}

__global__ __launch_bounds__(NT) void k_pivot_factor(const double* __restrict__ L, int n,
                                                     const int32_t* __restrict__ piv, int r, double* __restrict__ U) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= r * r) return;
  const int t = e % r, s = e / r;  // U[t, s] = L[piv[s], t] for t <= s
  U[t + static_cast<size_t>(s) * r] = (t <= s) ? L[piv[s] + static_cast<size_t>(t) * n] : 0.0;
}

// Blocked Cholesky of r <= R (R = 64 or 128, upper factor) by one 256-thread
// workgroup; the matrix is padded to R x R with a unit diagonal and kept row-major in
// LDS.  For each of the R / 16 block columns J: wave 0 factors the diagonal block (right-looking,
// wave-local synchronisation only), one lane per column solves the block row to its
// right (U_JJ^T X = A_JK), and the trailing upper blocks are updated on the matrix
// cores (A_KL -= U_JK^T U_JL, v_mfma_f64_16x16x4).  Failure rules as in
// k_cholesky_upper: a non-positive pivot, or max/min of the diagonal above max_ratio.
template <int R>
__global__ __launch_bounds__(256) void k_cholesky_mfma(double* __restrict__ Ag, int r, int lda, double max_ratio,
                                                       int32_t* __restrict__ ok) {
  constexpr int NB = R / 16;        // block columns
  constexpr int PT = R * R / 256;   // entries per thread
  __shared__ double a[R][R + 1];
  __shared__ double rdiag[R];  // reciprocals of the diagonal of the factor
  __shared__ int bad, near_id;
  const int tid = threadIdx.x;
  for (int u0 = 0; u0 < PT; u0 += 16) {  // staging: 16 loads of each thread at a time (clamped addresses)
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * (u0 + u), i = e % R, j = e / R;
      v[u] = Ag[(i < r && j < r) ? i + static_cast<size_t>(j) * lda : 0];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * (u0 + u), i = e % R, j = e / R;
      a[i][j] = (i < r && j < r) ? v[u] : (i == j ? 1.0 : 0.0);
    }
  }
  if (tid == 0) {
    bad = 0;
    near_id = 1;
  }
  __syncthreads();
  // A = I + E with max |E_ij| <= 2^-34 (the second Gram of CholeskyQR2): its factor is
  // I + triu(E, 1) + diag(E) / 2 up to terms below n max|E|^2 <= 2^-62, under the
  // rounding of the entries, and needs no sequential steps
  {
    bool far = false;
#pragma unroll 16
    for (int u = 0; u < PT; ++u) {
      const int e = tid + 256 * u, i = e % R, j = e / R;
      if (i <= j && j < r) far = far || !(fabs(a[i][j] - (i == j ? 1.0 : 0.0)) <= 0x1p-34);
    }
    if (far) near_id = 0;
  }
  __syncthreads();
  if (near_id) {
    for (int e = tid; e < r * r; e += 256) {
      const int i = e % r, j = e / r;
      const double v = a[i][j];
      Ag[i + static_cast<size_t>(j) * lda] = (i > j) ? 0.0 : (i == j ? 1.0 + 0.5 * (v - 1.0) : v);
    }
    if (tid == 0) *ok = 1;
    return;
  }
  const int w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  for (int J = 0; J < NB; ++J) {
    const int b = 16 * J;
    if (w == 0) {
      // the diagonal block in registers: lane (li, lk) holds rows lk + 4u (u < 4) of its
      // column li; row jj of the factor reaches the other lanes by cross-lane permutes
      double e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = a[b + lk + 4 * u][b + li];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int uj = jj >> 2, kj = jj & 3;
        const double d = readlane_f64(e[uj], jj + 16 * kj);
        const bool pos = d > 0.0;
        if (!pos && lane == 0) bad = 1;
        double piv, ip;
        sqrt_and_rsqrt(pos ? d : 1.0, &piv, &ip);
        if (lk == kj) e[uj] = (li == jj) ? piv : (li > jj ? e[uj] * ip : e[uj]);
        if (lane == jj + 16 * kj) rdiag[b + jj] = ip;
        const double ujc = __shfl(e[uj], li + 16 * kj, 64);  // factor entry (jj, li)
        double uji[4];                                        // factor entries (jj, lk + 4u)
#pragma unroll
        for (int u = 0; u < 4; ++u) uji[u] = __shfl(e[uj], lk + 4 * u + 16 * kj, 64);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = lk + 4 * u;
          if (i > jj && li >= i) e[u] = fma(-uji[u], ujc, e[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) a[b + lk + 4 * u][b + li] = e[u];
    }
    __syncthreads();
    const int rest = R - b - 16;
    if (rest > 0 && tid < rest) {
      const int c = b + 16 + tid;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double v = a[b + i][c];
#pragma unroll
        for (int l = 0; l < i; ++l) v = fma(-a[b + l][b + i], x[l], v);
        x[i] = v * rdiag[b + i];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) a[b + i][c] = x[i];
    }
    __syncthreads();
    // trailing upper blocks (K, L), J < K <= L, round-robin over the waves
    int t = 0;
    for (int K = J + 1; K < NB; ++K)
      for (int L = K; L < NB; ++L, ++t) {
        if (t % 4 != w) continue;
        dbl4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = a[16 * K + 4 * v + lk][16 * L + li];
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[b + kk + lk][16 * K + li], a[b + kk + lk][16 * L + li], acc, 0,
                                                     0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) a[16 * K + 4 * v + lk][16 * L + li] = acc[v];
      }
    __syncthreads();
  }
  for (int e = tid; e < r * r; e += 256) {
    const int i = e % r, j = e / r;
    Ag[i + static_cast<size_t>(j) * lda] = (bad || i > j) ? 0.0 : a[i][j];
  }
  if (tid == 0) {
    int fail = bad;
    if (!fail) {
      double dmin = INFINITY, dmax = 0.0;
      for (int i = 0; i < r; ++i) {
        dmin = fmin(dmin, a[i][i]);
        dmax = fmax(dmax, a[i][i]);
      }
      fail = dmax > max_ratio * dmin;
    }
    *ok = fail ? 0 : 1;
  }
}

// Right-looking Cholesky, upper factor, in global memory, one workgroup.
__global__ __launch_bounds__(BT) void k_cholesky_upper(double* __restrict__ A, int r, int lda, double max_ratio,
                                                       int32_t* __restrict__ ok) {
  __shared__ double piv, dmin, dmax;
  __shared__ int bad;
  if (threadIdx.x == 0) {
    bad = 0;
    dmin = INFINITY;
    dmax = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    if (threadIdx.x == 0) {
      const double a = A[j + static_cast<size_t>(j) * lda];
      if (!(a > 0.0)) bad = 1;
      piv = (a > 0.0) ? sqrt(a) : 1.0;
      A[j + static_cast<size_t>(j) * lda] = piv;
      dmin = fmin(dmin, piv);
      dmax = fmax(dmax, piv);
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / piv;
    for (int c = j + 1 + threadIdx.x; c < r; c += BT) A[j + static_cast<size_t>(c) * lda] *= inv;
    __syncthreads();
    // trailing update of the upper triangle: A[i, c] -= A[j, i] * A[j, c], j < i <= c
    const int w = r - j - 1;
    const long long tot = static_cast<long long>(w) * w;
    for (long long e = threadIdx.x; e < tot; e += BT) {
      const int i = j + 1 + static_cast<int>(e % w), c = j + 1 + static_cast<int>(e / w);
      if (i <= c) A[i + static_cast<size_t>(c) * lda] -= A[j + static_cast<size_t>(i) * lda] * A[j + static_cast<size_t>(c) * lda];
    }
    __syncthreads();
  }
  // zero the strict lower part
  for (long long e = threadIdx.x; e < static_cast<long long>(r) * r; e += BT) {
    const int i = static_cast<int>(e % r), c = static_cast<int>(e / r);
    if (i > c) A[i + static_cast<size_t>(c) * lda] = 0.0;
  }
  if (threadIdx.x == 0) *ok = (bad || dmax > max_ratio * dmin) ? 0 : 1;
}

// Right triangular solve X = Y U^{-1} (U upper, r <= 64), blocked, 64 rows of Y per
// workgroup.  U is padded to 64 x 64 with a unit diagonal.  Wave w solves rows
// 16w..16w+15 block column by block column (16 columns each): the update
// T = Y_J - sum_{I<J} X_I U_IJ runs on the matrix cores (v_mfma_f64_16x16x4), then
// X_J solves X_J U_JJ = T by substitution, one lane per row -- the standard blocked
// algorithm, backward stable like plain substitution.  The tile stays in LDS and each
// wave touches only its own rows, so the block loop needs no barrier.  *ok = 0 if U
// has a zero diagonal entry.
__global__ __launch_bounds__(256) void k_trsm_mfma(const double* __restrict__ Y, int rows, int r, int ldy,
                                                   const double* __restrict__ U, int ldu, double* __restrict__ X,
                                                   int ldx, int32_t* __restrict__ ok) {
  __shared__ double us[64][65];
  __shared__ double xs[64][65];
  __shared__ double dinv[64];  // reciprocals of U's diagonal (0 for a zero pivot)
  const int row0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  {  // staging: the 32 loads of each thread are issued together (clamped addresses)
    double uv[16], yv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, i = e % 64, l = e / 64;
      uv[u] = U[(i < r && l < r) ? i + static_cast<size_t>(l) * ldu : 0];
      yv[u] = Y[(row0 + i < rows && l < r) ? row0 + i + static_cast<size_t>(l) * ldy : 0];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 256 * u, i = e % 64, l = e / 64;
      us[i][l] = (i < r && l < r) ? uv[u] : (i == l ? 1.0 : 0.0);
      xs[i][l] = (row0 + i < rows && l < r) ? yv[u] : 0.0;
    }
  }
  __syncthreads();
  if (tid < 64) {
    const double dd = us[tid][tid];
    if (dd == 0.0) *ok = 0;
    dinv[tid] = (dd != 0.0) ? 1.0 / dd : 0.0;
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int rw = 16 * w;
  for (int J = 0; J < 4; ++J) {
    if (J > 0) {
      dbl4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = xs[rw + 4 * v + lk][16 * J + li];
      for (int I = 0; I < J; ++I)
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-xs[rw + li][16 * I + kk + lk],
                                                     us[16 * I + kk + lk][16 * J + li], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) xs[rw + 4 * v + lk][16 * J + li] = acc[v];
    }
    if (lk == 0) {
      const int bj = 16 * J;
      double x[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        double v = xs[rw + li][bj + jj];
#pragma unroll
        for (int l = 0; l < jj; ++l) v = fma(-x[l], us[bj + l][bj + jj], v);
        x[jj] = v * dinv[bj + jj];
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) xs[rw + li][bj + jj] = x[jj];
    }
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e % 64, l = e / 64;
    if (row0 + i < rows && l < r) X[row0 + i + static_cast<size_t>(l) * ldx] = xs[i][l];
  }
}

// Right triangular solve X = Y U^{-1} (U upper, r <= RM): one lane per row of Y,
// one wave per workgroup (many workgroups for tall Y); U and the reciprocals of its
// diagonal broadcast from LDS; forward substitution across the row with two
// independent partial sums per entry.
template <int RM>
__global__ __launch_bounds__(64) void k_trsm_right_upper(const double* __restrict__ Y, int rows, int r, int ldy,
                                                         const double* __restrict__ U, int ldu, double* __restrict__ X,
                                                         int ldx, int32_t* __restrict__ ok) {
  __shared__ double us[RM * RM];
  __shared__ double dinv[RM];
  for (int e = threadIdx.x; e < r * r; e += 64) us[e] = U[(e % r) + static_cast<size_t>(e / r) * ldu];
  __syncthreads();
  for (int j = threadIdx.x; j < r; j += 64) {
    const double dd = us[j + j * r];
    if (dd == 0.0 && blockIdx.x == 0) *ok = 0;
    dinv[j] = (dd != 0.0) ? 1.0 / dd : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= rows) return;
  double x[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j < r) {
      double v0 = Y[i + static_cast<size_t>(j) * ldy], v1 = 0.0;
      const double* uj = us + j * r;
#pragma unroll
      for (int l = 0; l + 1 < j; l += 2) {
        v0 = fma(-x[l], uj[l], v0);
        v1 = fma(-x[l + 1], uj[l + 1], v1);
      }
      if (j & 1) v0 = fma(-x[j - 1], uj[j - 1], v0);
      x[j] = (v0 + v1) * dinv[j];
      X[i + static_cast<size_t>(j) * ldx] = x[j];
    }
  }
}

__global__ __launch_bounds__(NT) void k_col_sumsq(const double* __restrict__ E, int rows, int lde,
                                                  double* __restrict__ out) {
  __shared__ double red[NT / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < rows; i += NT) {
    const double x = E[i + static_cast<size_t>(j) * lde];
    s = fma(x, x, s);
  }
  s = wave_sum_f64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    out[j] = t;
  }
}

__global__ __launch_bounds__(NT) void k_weighted_total(const double* __restrict__ cs, const double* __restrict__ w,
                                                       int cols, double* __restrict__ out) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (int j = threadIdx.x; j < cols; j += NT) s += (w ? w[j] : 1.0) * cs[j];
  s = wave_sum_f64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < NT / 64; ++i) t += red[i];
    *out = t;
  }
}

// Householder QR, one workgroup, LAPACK geqr2/larfg conventions.
__device__ void householder_qr_body(double* __restrict__ A, int m, int n, int lda, double* __restrict__ tau) {
  __shared__ double red[17];
  __shared__ double sh_tau, sh_beta, sh_scale;
  const int p = min(m, n);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = 0; j < p; ++j) {
    double* x = A + static_cast<size_t>(j) * lda;
    double s = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += BT) s = fma(x[i], x[i], s);
    const double xn2 = block_sum_1024(s, red);
    if (threadIdx.x == 0) {
      const double alpha = x[j];
      if (xn2 == 0.0) {
        sh_tau = 0.0;
        sh_beta = alpha;
        sh_scale = 1.0;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        sh_tau = (beta - alpha) / beta;
        sh_scale = 1.0 / (alpha - beta);
        sh_beta = beta;
      }
      tau[j] = sh_tau;
    }
    __syncthreads();
    const double tj = sh_tau, sc = sh_scale;
    for (int i = j + 1 + threadIdx.x; i < m; i += BT) x[i] *= sc;
    __syncthreads();
    if (threadIdx.x == 0) x[j] = sh_beta;
    if (tj != 0.0) {
      for (int c = j + 1 + wv; c < n; c += BT / 64) {
        double* y = A + static_cast<size_t>(c) * lda;
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w = fma(x[i], y[i], w);
        w = wave_sum_f64(w);
        w = tj * (w + y[j]);
        if (lane == 0) y[j] -= w;
        for (int i = j + 1 + lane; i < m; i += 64) y[i] = fma(-w, x[i], y[i]);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(BT) void k_householder_qr(double* __restrict__ A, int m, int n, int lda,
                                                       double* __restrict__ tau) {
  householder_qr_body(A, m, n, lda, tau);
}

// Row block i of a tall m x n matrix: rows [i b, i b + m_i), m_i = b except the last
// block, which takes the remainder (b <= m_i < 2b).
__device__ __forceinline__ int tsqr_rows(int m, int b, int nblk, int i) { return i + 1 < nblk ? b : m - i * b; }

// Householder QR of every row block, one workgroup per block; tau of block i at tau + i n.
__global__ __launch_bounds__(BT) void k_householder_qr_blocks(double* __restrict__ A, int m, int n, int lda, int b,
                                                              int nblk, double* __restrict__ tau) {
  const int i = blockIdx.x;
  householder_qr_body(A + static_cast<size_t>(i) * b, tsqr_rows(m, b, nblk, i), n, lda, tau + static_cast<size_t>(i) * n);
}

__device__ void householder_form_q_body(const double* __restrict__ A, int m, int p, int lda,
                                        const double* __restrict__ tau, double* __restrict__ Q, int ldq) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (long long e = threadIdx.x; e < static_cast<long long>(m) * p; e += BT) {
    const int i = static_cast<int>(e % m), c = static_cast<int>(e / m);
    Q[i + static_cast<size_t>(c) * ldq] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tj = tau[j];
    const double* v = A + static_cast<size_t>(j) * lda;
    if (tj != 0.0) {
      for (int c = j + wv; c < p; c += BT / 64) {
        double* y = Q + static_cast<size_t>(c) * ldq;
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w = fma(v[i], y[i], w);
        w = wave_sum_f64(w);
        w = tj * (w + y[j]);
        if (lane == 0) y[j] -= w;
        for (int i = j + 1 + lane; i < m; i += 64) y[i] = fma(-w, v[i], y[i]);
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(BT) void k_householder_form_q(const double* __restrict__ A, int m, int p, int lda,
                                                           const double* __restrict__ tau, double* __restrict__ Q,
                                                           int ldq) {
  householder_form_q_body(A, m, p, lda, tau, Q, ldq);
}

// Explicit Q (m_i x n) of every row block, one workgroup per block.
__global__ __launch_bounds__(BT) void k_householder_form_q_blocks(const double* __restrict__ A, int m, int n, int lda,
                                                                  int b, int nblk, const double* __restrict__ tau,
                                                                  double* __restrict__ Q, int ldq) {
  const int i = blockIdx.x;
  householder_form_q_body(A + static_cast<size_t>(i) * b, tsqr_rows(m, b, nblk, i), n, lda,
                          tau + static_cast<size_t>(i) * n, Q + static_cast<size_t>(i) * b, ldq);
}

// S = the blocks' R factors stacked: rows [i n, (i+1) n) of S (ld = nblk n) hold the
// upper triangle of block i's factored rows.
__global__ __launch_bounds__(NT) void k_stack_r(const double* __restrict__ A, int n, int lda, int b, int nblk,
                                                double* __restrict__ S) {
  const long long e = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
  const long long ls = static_cast<long long>(nblk) * n;
  if (e >= ls * n) return;
  const int row = static_cast<int>(e % ls), c = static_cast<int>(e / ls);
  const int i = row / n, r = row - i * n;
  S[e] = (c >= r) ? A[static_cast<size_t>(i) * b + r + static_cast<size_t>(c) * lda] : 0.0;
}

// Q = diag(Q_i) Q_S: rows of block i are Q_i (m_i x n, in Qb) times rows [i n, (i+1) n)
// of Q_S (ld = nblk n).  One thread per output row, 16 output columns per pass.
__global__ __launch_bounds__(NT) void k_tsqr_combine(const double* __restrict__ Qb, int m, int n, int b, int nblk,
                                                     const double* __restrict__ QS, double* __restrict__ Q, int ldq) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= m) return;
  const int i = min(r / b, nblk - 1);
  const size_t ls = static_cast<size_t>(nblk) * n;
  const double* qs = QS + static_cast<size_t>(i) * n;
  for (int c0 = 0; c0 < n; c0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int t = 0; t < n; ++t) {
      const double a = Qb[r + static_cast<size_t>(t) * m];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + u < n) acc[u] = fma(a, qs[t + static_cast<size_t>(c0 + u) * ls], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c0 + u < n) Q[r + static_cast<size_t>(c0 + u) * ldq] = acc[u];
  }
}

__global__ __launch_bounds__(NT) void k_extract_r(const double* __restrict__ A, int p, int n, int lda,
                                                  double* __restrict__ R, int ldr) {
  const long long e = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
  if (e >= static_cast<long long>(p) * n) return;
  const int i = static_cast<int>(e % p), c = static_cast<int>(e / p);
  const double sg = (A[i + static_cast<size_t>(i) * lda] < 0.0) ? -1.0 : 1.0;
  R[i + static_cast<size_t>(c) * ldr] = (c >= i) ? sg * A[i + static_cast<size_t>(c) * lda] : 0.0;
}

__global__ __launch_bounds__(NT) void k_flip_q(const double* __restrict__ A, int m, int p, int lda,
                                               double* __restrict__ Q, int ldq) {
  const long long e = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
  if (e >= static_cast<long long>(m) * p) return;
  const int i = static_cast<int>(e % m), c = static_cast<int>(e / m);
  if (A[c + static_cast<size_t>(c) * lda] < 0.0) Q[i + static_cast<size_t>(c) * ldq] = -Q[i + static_cast<size_t>(c) * ldq];
}

// One-sided (Hestenes) Jacobi, one workgroup of NTH threads = NTH/GW groups of GW
// lanes, one column pair per group per step, circle-method pair ordering.
// The matrix and V live in LDS when they fit (use_lds), else in global memory.
template <int NTH, int GW>
__global__ __launch_bounds__(NTH) void k_jacobi(double* __restrict__ Ag, int rows, int c, int lda,
                                                double* __restrict__ Vg, int ldv, double* __restrict__ sigma,
                                                int use_lds, int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  extern __shared__ double sm[];
  __shared__ int rotated;
  double* A = Ag;
  double* V = Vg;
  int la = lda, lv = ldv;
  if (use_lds) {
    A = sm;
    V = sm + static_cast<size_t>(rows) * c;
    la = rows;
    lv = c;
    for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
      const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
      A[i + static_cast<size_t>(j) * la] = Ag[i + static_cast<size_t>(j) * lda];
    }
  }
  for (long long e = threadIdx.x; e < static_cast<long long>(c) * c; e += NTH) {
    const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
    V[i + static_cast<size_t>(j) * lv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  constexpr int NG = NTH / GW;
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int N = c + (c & 1);  // players (a virtual empty column when c is odd)
  // a column pair counts as orthogonal when |a_p . a_q| <= rows * eps * ||a_p|| ||a_q||,
  // the rounding level of the computed dot product itself
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < N - 1; ++rd) {
      for (int k = grp; k < N / 2; k += NG) {
        int p, q;
        if (k == 0) {
          p = rd;
          q = N - 1;
        } else {
          p = (rd + k) % (N - 1);
          q = (rd - k + (N - 1)) % (N - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= c) continue;  // pair with the virtual column (uniform within the group)
        double* ap = A + static_cast<size_t>(p) * la;
        double* aq = A + static_cast<size_t>(q) * la;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = gl; i < rows; i += GW) {
          const double x = ap[i], y = aq[i];
          a = fma(x, x, a);
          b = fma(y, y, b);
          g = fma(x, y, g);
        }
#pragma unroll
        for (int o = GW / 2; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, GW);
          b += __shfl_xor(b, o, GW);
          g += __shfl_xor(g, o, GW);
        }
        if (a == 0.0 || b == 0.0) continue;
        if (!(fabs(g) > tol * sqrt(a) * sqrt(b))) continue;
        double cs, sn;
        if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
        jacobi_rotation(a, b, g, &cs, &sn);
        for (int i = gl; i < rows; i += GW) {
          const double x = ap[i], y = aq[i];
          ap[i] = cs * x - sn * y;
          aq[i] = sn * x + cs * y;
        }
        double* vp = V + static_cast<size_t>(p) * lv;
        double* vq = V + static_cast<size_t>(q) * lv;
        for (int i = gl; i < c; i += GW) {
          const double x = vp[i], y = vq[i];
          vp[i] = cs * x - sn * y;
          vq[i] = sn * x + cs * y;
        }
        if (gl == 0) rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) {
      conv_ = 1;
      break;
    }
    __syncthreads();
  }
  // column norms
  for (int j = grp; j < c; j += NG) {
    const double* aj = A + static_cast<size_t>(j) * la;
    double sacc = 0.0;
    for (int i = gl; i < rows; i += GW) sacc = fma(aj[i], aj[i], sacc);
#pragma unroll
    for (int o = GW / 2; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, GW);
    if (gl == 0) sigma[j] = sqrt(sacc);
  }
  if (use_lds) {
    __syncthreads();
    for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
      const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
      Ag[i + static_cast<size_t>(j) * lda] = A[i + static_cast<size_t>(j) * la];
    }
    for (long long e = threadIdx.x; e < static_cast<long long>(c) * c; e += NTH) {
      const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
      Vg[i + static_cast<size_t>(j) * ldv] = V[i + static_cast<size_t>(j) * lv];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// One-sided Jacobi for matrices whose A fits in LDS but A and V together do not
// (c and rows up to VT * GW): A in LDS, V in global memory (it stays in L2).  The
// pair order, threshold and rotation are those of k_jacobi.  Each lane holds its VT
// entries of both columns of A (and then of V) in registers, all loads issued before
// the arithmetic; the group sums are DPP row reductions.
template <int NTH, int GW, int VT>
__global__ __launch_bounds__(NTH) void k_jacobi_lv(double* __restrict__ Ag, int rows, int c, int lda,
                                                   double* __restrict__ V, int ldv, double* __restrict__ sigma, int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  extern __shared__ double A[];  // rows x c, column-major, leading dimension rows
  __shared__ int rotated;
  for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
    const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
    A[e] = Ag[i + static_cast<size_t>(j) * lda];
  }
  for (long long e = threadIdx.x; e < static_cast<long long>(c) * c; e += NTH) {
    const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
    V[i + static_cast<size_t>(j) * ldv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  constexpr int NG = NTH / GW;
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int N = c + (c & 1);
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < N - 1; ++rd) {
      for (int k = grp; k < N / 2; k += NG) {
        int p, q;
        if (k == 0) {
          p = rd;
          q = N - 1;
        } else {
          p = (rd + k) % (N - 1);
          q = (rd - k + (N - 1)) % (N - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= c) continue;  // pair with the virtual column (uniform within the group)
        double* ap = A + static_cast<size_t>(p) * rows;
        double* aq = A + static_cast<size_t>(q) * rows;
        double xa[VT], ya[VT];
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          const int i = min(gl + t * GW, rows - 1);
          xa[t] = ap[i];
          ya[t] = aq[i];
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int t = 0; t < VT; ++t)
          if (gl + t * GW < rows) {
            a = fma(xa[t], xa[t], a);
            b = fma(ya[t], ya[t], b);
            g = fma(xa[t], ya[t], g);
          }
        a = group_sum<GW>(a);
        b = group_sum<GW>(b);
        g = group_sum<GW>(g);
        if (a == 0.0 || b == 0.0) continue;
        if (!(fabs(g) > tol * sqrt(a) * sqrt(b))) continue;
        double cs, sn;
        if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
        jacobi_rotation(a, b, g, &cs, &sn);
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          const int i = gl + t * GW;
          if (i < rows) {
            ap[i] = cs * xa[t] - sn * ya[t];
            aq[i] = sn * xa[t] + cs * ya[t];
          }
        }
        double* vp = V + static_cast<size_t>(p) * ldv;
        double* vq = V + static_cast<size_t>(q) * ldv;
        double xv[VT], yv[VT];
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          const int i = min(gl + t * GW, c - 1);
          xv[t] = vp[i];
          yv[t] = vq[i];
        }
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          const int i = gl + t * GW;
          if (i < c) {
            vp[i] = cs * xv[t] - sn * yv[t];
            vq[i] = sn * xv[t] + cs * yv[t];
          }
        }
        if (gl == 0) rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) {
      conv_ = 1;
      break;
    }
    __syncthreads();
  }
  for (int j = grp; j < c; j += NG) {
    const double* aj = A + static_cast<size_t>(j) * rows;
    double sacc = 0.0;
    for (int i = gl; i < rows; i += GW) sacc = fma(aj[i], aj[i], sacc);
#pragma unroll
    for (int o = GW / 2; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, GW);
    if (gl == 0) sigma[j] = sqrt(sacc);
  }
  __syncthreads();
  for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
    const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
    Ag[i + static_cast<size_t>(j) * lda] = A[e];
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// The same Jacobi in two phases for c <= 138 (when V alone fits in LDS): the sweeps
// run on A in LDS and log every slot's rotation (cos, sin) -- (1, 0) for a pair left
// alone -- to `rot` in global memory; A goes back to memory, and V is then built in
// LDS by replaying the log round by round (each group loads its next rotation one
// round ahead).  No V traffic crosses L2 inside the sweeps.
template <int NTH, int GW, int VT>
__global__ __launch_bounds__(NTH) void k_jacobi_log(double* __restrict__ Ag, int rows, int c, int lda,
                                                    double* __restrict__ Vg, int ldv, double* __restrict__ sigma,
                                                    double2* __restrict__ rot, int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  extern __shared__ double sm[];  // A (rows x c), later V (c x c)
  __shared__ int rotated, nsw;
  double* A = sm;
  for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
    const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
    A[e] = Ag[i + static_cast<size_t>(j) * lda];
  }
  if (threadIdx.x == 0) nsw = 0;
  __syncthreads();
  constexpr int NG = NTH / GW;
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int N = c + (c & 1), H = N / 2;
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  auto pair_of = [&](int rd, int k, int* pp, int* qq) {
    int p, q;
    if (k == 0) {
      p = rd;
      q = N - 1;
    } else {
      p = (rd + k) % (N - 1);
      q = (rd - k + (N - 1)) % (N - 1);
    }
    *pp = min(p, q);
    *qq = max(p, q);
  };
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < N - 1; ++rd) {
      double2* lr = rot + (static_cast<size_t>(sweep) * (N - 1) + rd) * H;
      for (int k = grp; k < H; k += NG) {
        int p, q;
        pair_of(rd, k, &p, &q);
        double cs = 1.0, sn = 0.0;
        if (q < c) {  // uniform within the group
          double* ap = A + static_cast<size_t>(p) * rows;
          double* aq = A + static_cast<size_t>(q) * rows;
          double xa[VT], ya[VT];
#pragma unroll
          for (int t = 0; t < VT; ++t) {
            const int i = min(gl + t * GW, rows - 1);
            xa[t] = ap[i];
            ya[t] = aq[i];
          }
          double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
          for (int t = 0; t < VT; ++t)
            if (gl + t * GW < rows) {
              a = fma(xa[t], xa[t], a);
              b = fma(ya[t], ya[t], b);
              g = fma(xa[t], ya[t], g);
            }
          a = group_sum<GW>(a);
          b = group_sum<GW>(b);
          g = group_sum<GW>(g);
          if (a != 0.0 && b != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
            if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
            jacobi_rotation(a, b, g, &cs, &sn);
#pragma unroll
            for (int t = 0; t < VT; ++t) {
              const int i = gl + t * GW;
              if (i < rows) {
                ap[i] = cs * xa[t] - sn * ya[t];
                aq[i] = sn * xa[t] + cs * ya[t];
              }
            }
            if (gl == 0) rotated = 1;
          }
        }
        if (gl == 0) lr[k] = make_double2(cs, sn);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) nsw = sweep + 1;
    if (!rotated) {
      conv_ = 1;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int j = grp; j < c; j += NG) {
    const double* aj = A + static_cast<size_t>(j) * rows;
    double sacc = 0.0;
    for (int i = gl; i < rows; i += GW) sacc = fma(aj[i], aj[i], sacc);
    sacc = group_sum<GW>(sacc);
    if (gl == 0) sigma[j] = sqrt(sacc);
  }
  for (long long e = threadIdx.x; e < static_cast<long long>(rows) * c; e += NTH) {
    const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
    Ag[i + static_cast<size_t>(j) * lda] = A[e];
  }
  __syncthreads();
  // replay: V = product of the logged rotations, in LDS (c x c)
  double* V = sm;
  for (long long e = threadIdx.x; e < static_cast<long long>(c) * c; e += NTH) {
    const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
    V[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int total = nsw * (N - 1);  // rounds to replay
  if (N > 1) {
    // each group's slots: k = grp, grp + NG, ... (at most two for c <= 138 and NG = 64)
    double2 nxt0 = (total > 0 && grp < H) ? rot[grp] : make_double2(1.0, 0.0);
    double2 nxt1 = (total > 0 && grp + NG < H) ? rot[grp + NG] : make_double2(1.0, 0.0);
    for (int t = 0; t < total; ++t) {
      const int rd = t % (N - 1);
      const double2 cur0 = nxt0, cur1 = nxt1;
      if (t + 1 < total) {
        const double2* nr = rot + static_cast<size_t>(t + 1) * H;
        if (grp < H) nxt0 = nr[grp];
        if (grp + NG < H) nxt1 = nr[grp + NG];
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int k = grp + s2 * NG;
        const double2 cr = s2 == 0 ? cur0 : cur1;
        if (k >= H || cr.y == 0.0) continue;
        int p, q;
        pair_of(rd, k, &p, &q);
        double* vp = V + static_cast<size_t>(p) * c;
        double* vq = V + static_cast<size_t>(q) * c;
        double xv[VT], yv[VT];
#pragma unroll
        for (int u = 0; u < VT; ++u) {
          const int i = min(gl + u * GW, c - 1);
          xv[u] = vp[i];
          yv[u] = vq[i];
        }
#pragma unroll
        for (int u = 0; u < VT; ++u) {
          const int i = gl + u * GW;
          if (i < c) {
            vp[i] = cr.x * xv[u] - cr.y * yv[u];
            vq[i] = cr.y * xv[u] + cr.x * yv[u];
          }
        }
      }
      __syncthreads();
    }
  }
  for (long long e = threadIdx.x; e < static_cast<long long>(c) * c; e += NTH) {
    const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
    Vg[i + static_cast<size_t>(j) * ldv] = V[e];
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// One-sided Jacobi with A and V held in registers, for c <= 16 VT columns of at most
// 16 VT rows.  Group k of 16 lanes holds two columns of A with the matching columns of
// V (lane l: entries l, l + 16, ...) and rotates them as one pair per step.  The pairs
// follow the odd-even ordering of positions 0..N-1, N = c + (c & 1): even steps pair
// (2k, 2k+1), odd steps (2k+1, 2k+2) with positions N-1 and 0 left alone, and the two
// columns of a pair trade positions, so that N steps meet every pair of columns once.
// Group k holds positions (2k, 2k+1) before an even step and (2k+1, 2k+2 mod N)
// before an odd one; between steps each group hands one column (A, V and its index)
// to a neighbour through LDS, half the LDS traffic of a round that loads and stores
// both columns, and V needs no second pass.  Rotation rule and stopping test as in
// k_jacobi; column j of A and V goes back to column j.
template <int VT>
__global__ __launch_bounds__(1024) void k_jacobi_oe(double* __restrict__ Ag, int rows, int c, int lda,
                                                   double* __restrict__ Vg, int ldv, double* __restrict__ sigma,
                                                   int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  __syncthreads();
  constexpr int GW = 16;
  constexpr int SL = 2 * VT * GW;   // doubles per slot: an A column, then its V column
  extern __shared__ double slot[];  // [H][SL]
  __shared__ int sid[64];
  __shared__ int rotated;
  const int N = c + (c & 1), H = N / 2;
  const int k = threadIdx.x / GW, gl = threadIdx.x % GW;
  const bool act = k < H;  // uniform within a group
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  double x[VT], y[VT], vx[VT], vy[VT];
  int ix = 2 * k, iy = 2 * k + 1;  // column held at the first and second position
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    const int i = gl + t * GW;
    x[t] = (act && i < rows && ix < c) ? Ag[i + static_cast<size_t>(ix) * lda] : 0.0;
    y[t] = (act && i < rows && iy < c) ? Ag[i + static_cast<size_t>(iy) * lda] : 0.0;
    vx[t] = (ix < c && i == ix) ? 1.0 : 0.0;  // the padding column (index c) stays zero
    vy[t] = (iy < c && i == iy) ? 1.0 : 0.0;
  }
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int st = 0; st < N; ++st) {
      const bool odd = st & 1;
      const bool idle = odd && k == H - 1;
      if (act && !idle) {
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int t = 0; t < VT; ++t) {  // entries past rows are zero
          a = fma(x[t], x[t], a);
          b = fma(y[t], y[t], b);
          g = fma(x[t], y[t], g);
        }
        group_sum3<GW>(a, b, g);
        if (a != 0.0 && b != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
          double cs, sn;
          if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
          jacobi_rotation(a, b, g, &cs, &sn);
#pragma unroll
          for (int t = 0; t < VT; ++t) {
            const double xa = x[t], ya = y[t], xv = vx[t], yv = vy[t];
            x[t] = cs * xa - sn * ya;
            y[t] = sn * xa + cs * ya;
            vx[t] = cs * xv - sn * yv;
            vy[t] = sn * xv + cs * yv;
          }
          if (gl == 0) rotated = 1;
        }
      }
      // after an even step position 2k holds y and 2k+1 holds x: y goes to group k-1,
      // the column at 2k+2 comes from group k+1.  After an odd step position 2k+2
      // holds x (y for the idle pair, which did not trade): it goes to group k+1, the
      // column at 2k comes from group k-1.
      if (idle) {
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          const double ta = x[t], tv = vx[t];
          x[t] = y[t];
          vx[t] = vy[t];
          y[t] = ta;
          vy[t] = tv;
        }
        const int ti = ix;
        ix = iy;
        iy = ti;
      }
      if (act) {
        double* my = slot + static_cast<size_t>(k) * SL;
#pragma unroll
        for (int t = 0; t < VT; ++t) {
          my[t * GW + gl] = odd ? x[t] : y[t];
          my[(VT + t) * GW + gl] = odd ? vx[t] : vy[t];
        }
        if (gl == 0) sid[k] = odd ? ix : iy;
      }
      __syncthreads();
      if (act) {
        const int nb = odd ? (k == 0 ? H - 1 : k - 1) : (k == H - 1 ? 0 : k + 1);
        const double* in = slot + static_cast<size_t>(nb) * SL;
        if (odd) {
#pragma unroll
          for (int t = 0; t < VT; ++t) {
            x[t] = in[t * GW + gl];
            vx[t] = in[(VT + t) * GW + gl];
          }
          ix = sid[nb];
        } else {
#pragma unroll
          for (int t = 0; t < VT; ++t) {
            y[t] = in[t * GW + gl];
            vy[t] = in[(VT + t) * GW + gl];
          }
          iy = sid[nb];
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) {
      conv_ = 1;
      break;
    }
  }
  if (act) {
    double sa = 0.0, sb = 0.0, dummy = 0.0;
#pragma unroll
    for (int t = 0; t < VT; ++t) {
      sa = fma(x[t], x[t], sa);
      sb = fma(y[t], y[t], sb);
    }
    group_sum3<GW>(sa, sb, dummy);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = h == 0 ? ix : iy;
      if (j >= c) continue;  // the padding column
      if (gl == 0) sigma[j] = sqrt(h == 0 ? sa : sb);
#pragma unroll
      for (int t = 0; t < VT; ++t) {
        const int i = gl + t * GW;
        if (i < rows) Ag[i + static_cast<size_t>(j) * lda] = h == 0 ? x[t] : y[t];
        if (i < c) Vg[i + static_cast<size_t>(j) * ldv] = h == 0 ? vx[t] : vy[t];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// One-sided cyclic Jacobi (round-robin pair order) for c <= 64 columns of at most
// GW * RPL rows, A and V staged in LDS.  32 groups of GW lanes, one column pair per
// group per round; a lane holds its RPL entries of both columns in registers for the
// round, so all loads of a round are in flight together.  Rotation rule and stopping
// test as in k_jacobi.
template <int GW, int RPL>
__global__ __launch_bounds__(32 * GW) void k_jacobi_reg(double* __restrict__ Ag, int rows, int c, int lda,
                                                        double* __restrict__ Vg, int ldv, double* __restrict__ sigma, int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  constexpr int NTH = 32 * GW;
  constexpr int VPL = (64 + GW - 1) / GW;
  extern __shared__ double sm[];
  __shared__ int rotated;
  // odd leading dimensions: the lane groups of a wave work on different columns, and
  // a column stride of an even number of doubles would put them on the same banks
  const int la = rows | 1, lv = c | 1;
  double* A = sm;                                // rows x c, leading dimension la
  double* V = sm + static_cast<size_t>(la) * c;  // c x c, leading dimension lv
  for (int e = threadIdx.x; e < rows * c; e += NTH) {
    const int i = e % rows, j = e / rows;
    A[i + j * la] = Ag[i + static_cast<size_t>(j) * lda];
  }
  for (int e = threadIdx.x; e < c * c; e += NTH) {
    const int i = e % c, j = e / c;
    V[i + j * lv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int N = c + (c & 1);  // players (a virtual empty column when c is odd)
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < N - 1; ++rd) {
      int p = 0, q = c;
      if (grp < N / 2) {
        if (grp == 0) {
          p = rd;
          q = N - 1;
        } else {
          p = (rd + grp) % (N - 1);
          q = (rd - grp + (N - 1)) % (N - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
      }
      if (q < c) {  // uniform within the group
        double* ap = A + static_cast<size_t>(p) * la;
        double* aq = A + static_cast<size_t>(q) * la;
        double x[RPL], y[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int i = gl + u * GW;
          x[u] = (i < rows) ? ap[i] : 0.0;
          y[u] = (i < rows) ? aq[i] : 0.0;
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          a = fma(x[u], x[u], a);
          b = fma(y[u], y[u], b);
          g = fma(x[u], y[u], g);
        }
#pragma unroll
        for (int o = GW / 2; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, GW);
          b += __shfl_xor(b, o, GW);
          g += __shfl_xor(g, o, GW);
        }
        if (a != 0.0 && b != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
          double cs, sn;
          if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
          jacobi_rotation(a, b, g, &cs, &sn);
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int i = gl + u * GW;
            if (i < rows) {
              ap[i] = cs * x[u] - sn * y[u];
              aq[i] = sn * x[u] + cs * y[u];
            }
          }
          double* vp = V + static_cast<size_t>(p) * lv;
          double* vq = V + static_cast<size_t>(q) * lv;
          double xv[VPL], yv[VPL];
#pragma unroll
          for (int u = 0; u < VPL; ++u) {
            const int i = gl + u * GW;
            xv[u] = (i < c) ? vp[i] : 0.0;
            yv[u] = (i < c) ? vq[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < VPL; ++u) {
            const int i = gl + u * GW;
            if (i < c) {
              vp[i] = cs * xv[u] - sn * yv[u];
              vq[i] = sn * xv[u] + cs * yv[u];
            }
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) {
      conv_ = 1;
      break;
    }
    __syncthreads();
  }
  for (int j = grp; j < c; j += NTH / GW) {
    const double* aj = A + static_cast<size_t>(j) * la;
    double sacc = 0.0;
    for (int i = gl; i < rows; i += GW) sacc = fma(aj[i], aj[i], sacc);
#pragma unroll
    for (int o = GW / 2; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, GW);
    if (gl == 0) sigma[j] = sqrt(sacc);
  }
  for (int e = threadIdx.x; e < rows * c; e += NTH) {
    const int i = e % rows, j = e / rows;
    Ag[i + static_cast<size_t>(j) * lda] = A[i + j * la];
  }
  for (int e = threadIdx.x; e < c * c; e += NTH) {
    const int i = e % c, j = e / c;
    Vg[i + static_cast<size_t>(j) * ldv] = V[i + j * lv];
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// One-sided Jacobi for c <= 64 columns of at most 64 rows: k_jacobi_reg with
// 8-lane groups, both A and V zero-padded to 64 rows in LDS so that every lane moves
// its 8 entries of a column as four 16-byte LDS accesses with no bounds tests, and
// the group's dot products reduced with DPP moves.
__global__ __launch_bounds__(256) void k_jacobi64(double* __restrict__ Ag, int rows, int c, int lda,
                                                  double* __restrict__ Vg, int ldv, double* __restrict__ sigma, int max_sweeps, int32_t* __restrict__ info) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  if (threadIdx.x == 0) gmax_ = 0ull;
  constexpr int GW = 8, NTH = 256, LD = 64;
  extern __shared__ double2 sm16[];  // 16-byte aligned: columns are read as double2
  __shared__ int rotated;
  double* A = reinterpret_cast<double*>(sm16);   // 64 x c (rows >= `rows` are zero)
  double* V = A + static_cast<size_t>(LD) * c;   // 64 x c (rows >= c are zero)
  {  // staging: each thread's loads are issued together (clamped addresses)
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = threadIdx.x + NTH * u, i = e % LD, j = e / LD;
      v[u] = Ag[(i < rows && j < c) ? i + static_cast<size_t>(j) * lda : 0];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = threadIdx.x + NTH * u, i = e % LD, j = e / LD;
      if (j < c) {
        A[e] = (i < rows) ? v[u] : 0.0;
        V[e] = (i == j) ? 1.0 : 0.0;
      }
    }
  }
  __syncthreads();
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const int N = c + (c & 1);
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps && N > 1; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    // round-robin positions of this group's pair, advanced by one (mod N - 1) per
    // round instead of recomputed with divisions: group 0 pairs rd with N - 1, group
    // k pairs rd + k with rd - k
    int pp = (grp == 0) ? 0 : grp % (N - 1);
    int qq = (grp == 0) ? N - 1 : (N - 1 - grp % (N - 1)) % (N - 1);
    for (int rd = 0; rd < N - 1; ++rd) {
      int p = 0, q = c;
      if (grp < N / 2) {
        p = min(pp, qq);
        q = max(pp, qq);
      }
      pp = (pp + 1 == N - 1) ? 0 : pp + 1;
      if (grp != 0) qq = (qq + 1 == N - 1) ? 0 : qq + 1;
      if (q < c) {  // uniform within the group
        double2* ap = reinterpret_cast<double2*>(A + static_cast<size_t>(p) * LD) + gl;
        double2* aq = reinterpret_cast<double2*>(A + static_cast<size_t>(q) * LD) + gl;
        double2 x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[u] = ap[8 * u];
          y[u] = aq[8 * u];
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a = fma(x[u].x, x[u].x, fma(x[u].y, x[u].y, a));
          b = fma(y[u].x, y[u].x, fma(y[u].y, y[u].y, b));
          g = fma(x[u].x, y[u].x, fma(x[u].y, y[u].y, g));
        }
        a = group8_sum(a);
        b = group8_sum(b);
        g = group8_sum(g);
        // |g| > tol sqrt(a b), as g^2 > tol^2 a b while a b is a normal number
        const double ab = a * b;
        const bool rot = (ab > 1e-280 && ab < 1e280) ? (g * g > tol * tol * ab) : (fabs(g) > tol * sqrt(a) * sqrt(b));
        if (a != 0.0 && b != 0.0 && rot) {
          double cs, sn;
          if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
          jacobi_rotation(a, b, g, &cs, &sn);
          double2* vp = reinterpret_cast<double2*>(V + static_cast<size_t>(p) * LD) + gl;
          double2* vq = reinterpret_cast<double2*>(V + static_cast<size_t>(q) * LD) + gl;
          double2 xv[4], yv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            xv[u] = vp[8 * u];
            yv[u] = vq[8 * u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            ap[8 * u] = double2{cs * x[u].x - sn * y[u].x, cs * x[u].y - sn * y[u].y};
            aq[8 * u] = double2{sn * x[u].x + cs * y[u].x, sn * x[u].y + cs * y[u].y};
            vp[8 * u] = double2{cs * xv[u].x - sn * yv[u].x, cs * xv[u].y - sn * yv[u].y};
            vq[8 * u] = double2{sn * xv[u].x + cs * yv[u].x, sn * xv[u].y + cs * yv[u].y};
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) {
      conv_ = 1;
      break;
    }
    __syncthreads();
  }
  for (int j = grp; j < c; j += NTH / GW) {
    const double2* aj = reinterpret_cast<const double2*>(A + static_cast<size_t>(j) * LD) + gl;
    double sacc = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) sacc = fma(aj[8 * u].x, aj[8 * u].x, fma(aj[8 * u].y, aj[8 * u].y, sacc));
    sacc = group8_sum(sacc);
    if (gl == 0) sigma[j] = sqrt(sacc);
  }
  for (int e = threadIdx.x; e < LD * c; e += NTH) {
    const int i = e % LD, j = e / LD;
    if (i < rows) Ag[i + static_cast<size_t>(j) * lda] = A[e];
    if (i < c) Vg[i + static_cast<size_t>(j) * ldv] = V[e];
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// Convergence test of a one-sided Jacobi on the 64 x NC matrix A in LDS (column-major,
// leading dimension 64), by all 256 threads: true when no pair (p, q) would rotate,
// i.e. g^2 <= tol^2 a b for a = |a_p|^2, b = |a_q|^2, g = a_p^T a_q (the sweep's own
// test), which is what a further sweep would find before its first rotation.  The
// Gram matrix comes from the FP64 matrix cores on a padded copy T (NC x 65) and the
// squared norms nrm (NC), both LDS scratch.  Three barriers.
template <int NC>
__device__ bool jacobi_gram_converged(const double* A, double tol, double* T, double* nrm, int* viol) {
  constexpr int NTH = 256, TP = 65, NB = NC / 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  for (int e = tid; e < NC * 64; e += NTH) T[(e >> 6) * TP + (e & 63)] = A[e];
  if (tid == 0) *viol = 0;
  {  // squared column norms, NTH / NC lanes a column, in the order of the sweep's sums
    constexpr int LPC = NTH / NC, RPL = 64 / LPC;
    const int j = tid / LPC, q = tid % LPC;
    double sacc = 0.0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const double x = A[j * 64 + q * RPL + u];
      sacc = fma(x, x, sacc);
    }
    sacc = group_sum<LPC>(sacc);
    if (q == 0) nrm[j] = sacc;
  }
  __syncthreads();
  int t = 0;
  for (int P = 0; P < NB; ++P)
    for (int Q = P; Q < NB; ++Q, ++t) {
      if (t % (NTH / 64) != w) continue;  // uniform within the wave
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < 64; k0 += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[(16 * P + li) * TP + k0 + lk], T[(16 * Q + li) * TP + k0 + lk],
                                                   acc, 0, 0, 0);
      bool bad = false;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pp = 16 * P + 4 * v + lk, qq = 16 * Q + li;
        if (pp < qq) {
          const double a = nrm[pp], b = nrm[qq], g = acc[v], ab = a * b;
          const bool rot = (ab > 1e-280 && ab < 1e280) ? (g * g > tol * tol * ab) : (fabs(g) > tol * sqrt(a) * sqrt(b));
          bad = bad || (a != 0.0 && b != 0.0 && rot);
        }
      }
      if (bad) *viol = 1;
    }
  __syncthreads();
  const bool ok = *viol == 0;
  __syncthreads();
  return ok;
}

// One-sided Jacobi for NC/2 < c <= NC columns (NC = 32 or 64) of at most 64 rows,
// padded to 64 x NC, with a hierarchical parallel ordering that keeps one column of
// each pair in registers.  A sweep has log2(NC) phases: in phase h the NC columns form
// 2^h blocks of S = NC >> h; in each block the first S/2 columns stay with their
// groups ("kept") while the last S/2 circulate: in round s of the phase, group i of a
// block pairs its kept column i with circulating column S/2 + (i + s) mod S/2.  The
// phases pair every two columns exactly once in NC - 1 rounds, and per round a group
// reads and writes only the circulating column (of A and of V) through LDS: half the
// LDS traffic of an ordering in which both columns move.  Groups are
// GW = 512 / NC lanes; a lane holds 64 / GW rows of a column as double2 pairs.
// Padded columns are zero and never rotate.  Same rotation, stopping test and output
// as k_jacobi64, except that after a sweep whose rotated pairs all had g^2 <= 1e-12 a b
// the next sweep is replaced by jacobi_gram_converged (the stopping test on every pair
// of the Gram matrix), and run only if some pair fails it.
//
// ACCV = false is for a square lower-triangular input L (c x c, c = rows), such as
// R^T from a QR: the rotations are not accumulated (a quarter of a round's work);
// after convergence the accumulated rotation J = L^{-1} A_final is formed by forward
// substitution, whose columns are orthonormal to about n u kappa(L).  That is used
// only when the sweeps converged and sigma_max <= kJacobiNoVCond sigma_min; otherwise
// the kernel writes only sigma and info (info[1] = -1), leaves A as it was, and the
// caller runs the ACCV = true kernel.  With want_v = 0 (ACCV = false) no V is formed
// at all: A_final, sigma and info only, for callers that need the left singular
// vectors of the triangular factor's product and not the rotations.
template <int NC, bool ACCV>
__global__ __launch_bounds__(256) void k_jacobi64h(double* __restrict__ Ag, int rows, int c, int lda,
                                                   double* __restrict__ Vg, int ldv, double* __restrict__ sigma, int max_sweeps, int32_t* __restrict__ info,
                                                   int want_v) {
  __shared__ unsigned long long gmax_;  // bits of the largest |a_p^T a_q| rotated in the last sweep
  // set when the current sweep rotates a pair with g^2 > 1e-12 a b
  __shared__ int bigrot;
  if (threadIdx.x == 0) {
    gmax_ = 0ull;
    bigrot = 0;
  }
  constexpr int NTH = 256, LD = 64, GW = 512 / NC, UP = 32 / GW;
  static_assert(NC == 32 || NC == 64, "32 or 64 columns");
  __shared__ double2 sA[NC * LD / 2];  // 64 x NC, column-major (rows >= `rows` zero)
  __shared__ double2 sV[NC * LD / 2];  // 64 x NC: V (identity outside the leading c x c block), or L
  __shared__ int rotated;
  __shared__ double smax_[NTH / 64], smin_[NTH / 64];
  __shared__ double gT[NC * 65], gnrm[NC];  // scratch of the Gram convergence test
  __shared__ int gviol;
  double* A = reinterpret_cast<double*>(sA);
  double* V = reinterpret_cast<double*>(sV);
  {  // staging: each thread's loads are issued together (clamped addresses)
    constexpr int PER = NC * LD / NTH;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + NTH * u, i = e % LD, j = e / LD;
      v[u] = Ag[(i < rows && j < c) ? i + static_cast<size_t>(j) * lda : 0];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + NTH * u, i = e % LD, j = e / LD;
      A[e] = (i < rows && j < c) ? v[u] : 0.0;
      // ACCV: V = I; otherwise a copy of the input (L) for the substitution
      V[e] = ACCV ? ((i == j) ? 1.0 : 0.0) : A[e];
    }
  }
  __syncthreads();
  const int grp = threadIdx.x / GW, gl = threadIdx.x % GW;
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  int nsw_ = 0, conv_ = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    nsw_ = sweep + 1;
    if (threadIdx.x == 0) {
      rotated = 0;
    }
    bool any = false;
    for (int lh = (NC == 64 ? 5 : 4); lh >= 0; --lh) {
      const int half = 1 << lh;
      const int blk = grp >> lh, i = grp & (half - 1);
      const int kc = blk * 2 * half + i;  // kept column
      double2 ka[UP], kv[UP];
      {
        const double2* ap = sA + kc * (LD / 2) + gl;
        const double2* vp = sV + kc * (LD / 2) + gl;
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          ka[u] = ap[GW * u];
          if (ACCV) kv[u] = vp[GW * u];
        }
      }
      int qi = i;  // (i + st) mod half, stepped without a division
      for (int st = 0; st < half; ++st) {
        const int qc = blk * 2 * half + half + qi;  // circulating column
        qi = (qi + 1 == half) ? 0 : qi + 1;
        double2* aq = sA + qc * (LD / 2) + gl;
        double2* vq = sV + qc * (LD / 2) + gl;
        // with 64 columns the LDS traffic decides: V is read only for a rotation;
        // with 32, the latency does, and V is read together with A
        constexpr bool PRE_V = NC == 32;
        double2 y[UP], yv[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          y[u] = aq[GW * u];
          if (ACCV && PRE_V) yv[u] = vq[GW * u];
        }
        double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          a = fma(ka[u].x, ka[u].x, fma(ka[u].y, ka[u].y, a));
          b = fma(y[u].x, y[u].x, fma(y[u].y, y[u].y, b));
          g = fma(ka[u].x, y[u].x, fma(ka[u].y, y[u].y, g));
        }
        group_sum3<GW>(a, b, g);
        const double ab = a * b;
        const bool rot = (ab > 1e-280 && ab < 1e280) ? (g * g > tol * tol * ab) : (fabs(g) > tol * sqrt(a) * sqrt(b));
        if (a != 0.0 && b != 0.0 && rot) {  // uniform within the group
          double cs, sn;
          if (sweep == max_sweeps - 1) atomicMax(&gmax_, static_cast<unsigned long long>(__double_as_longlong(fabs(g))));
          if (gl == 0 && !(g * g <= 1e-12 * ab)) bigrot = 1;
          jacobi_rotation(a, b, g, &cs, &sn);
          if (ACCV && !PRE_V) {
#pragma unroll
            for (int u = 0; u < UP; ++u) yv[u] = vq[GW * u];
          }
#pragma unroll
          for (int u = 0; u < UP; ++u) {
            const double2 x = ka[u];
            ka[u] = double2{cs * x.x - sn * y[u].x, cs * x.y - sn * y[u].y};
            aq[GW * u] = double2{sn * x.x + cs * y[u].x, sn * x.y + cs * y[u].y};
            if (ACCV) {
              const double2 xv = kv[u];
              kv[u] = double2{cs * xv.x - sn * yv[u].x, cs * xv.y - sn * yv[u].y};
              vq[GW * u] = double2{sn * xv.x + cs * yv[u].x, sn * xv.y + cs * yv[u].y};
            }
          }
          any = true;
        }
        __syncthreads();
      }
      {  // the kept column goes back before the next phase regroups the columns
        double2* ap = sA + kc * (LD / 2) + gl;
        double2* vp = sV + kc * (LD / 2) + gl;
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          ap[GW * u] = ka[u];
          if (ACCV) vp[GW * u] = kv[u];
        }
      }
      __syncthreads();
    }
    if (any && gl == 0) rotated = 1;
    __syncthreads();
    if (!rotated) {
      conv_ = 1;
      break;
    }
    // Jacobi converges quadratically: once every pair a sweep rotated had g^2 <= 1e-12
    // a b, the next sweep is expected to rotate nothing.  Instead of running it, the
    // Gram matrix tells whether it would (the same test on every pair).
    const bool small = bigrot == 0;
    __syncthreads();
    if (threadIdx.x == 0) bigrot = 0;  // for the next sweep, before its first round
    __syncthreads();
    if (small && sweep + 1 < max_sweeps && jacobi_gram_converged<NC>(A, tol, gT, gnrm, &gviol)) {
      conv_ = 1;
      break;
    }
  }
  // column norms (sigma); without V also their extremes, for the condition test
  double smax = 0.0, smin = HUGE_VAL;
  for (int j = grp; j < c; j += NTH / GW) {
    const double2* aj = sA + j * (LD / 2) + gl;
    double sacc = 0.0;
#pragma unroll
    for (int u = 0; u < UP; ++u) sacc = fma(aj[GW * u].x, aj[GW * u].x, fma(aj[GW * u].y, aj[GW * u].y, sacc));
    sacc = group_sum<GW>(sacc);
    const double sj = sqrt(sacc);
    if (gl == 0) sigma[j] = sj;
    smax = fmax(smax, sj);
    smin = fmin(smin, sj);
  }
  if (!ACCV && want_v) {
    // every lane of a group holds its columns' values: the wave extremes cover them
    for (int o = 32; o > 0; o >>= 1) {
      smax = fmax(smax, __shfl_xor(smax, o, 64));
      smin = fmin(smin, __shfl_xor(smin, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      smax_[threadIdx.x >> 6] = smax;
      smin_[threadIdx.x >> 6] = smin;
    }
    __syncthreads();
    double gmx = 0.0, gmn = HUGE_VAL;
    for (int w = 0; w < NTH / 64; ++w) {
      gmx = fmax(gmx, smax_[w]);
      gmn = fmin(gmn, smin_[w]);
    }
    const bool use = conv_ && nsw_ > 0 && gmn > 0.0 && gmx <= kJacobiNoVCond * gmn;
    if (!use) {  // uniform: the caller reruns with the rotations accumulated
      if (threadIdx.x == 0 && info) {
        info[0] = nsw_;
        info[1] = -1;
        *reinterpret_cast<double*>(info + 2) = 0.0;
      }
      return;
    }
    // J = L^{-1} A_final by forward substitution: 4 lanes per column j, lane `sub`
    // keeps x_l for l = sub (mod 4) and sums those terms of each row's dot product
    constexpr int SL = 4, XR = NC / SL;
    const int j = threadIdx.x / SL, sub = threadIdx.x % SL;
    if (j < NC) {  // NTH / SL = 64 >= NC column groups; groups past c idle
      double x[XR];
#pragma unroll
      for (int u = 0; u < XR; ++u) x[u] = 0.0;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        if (i < c) {  // uniform
          double sdot = 0.0;
#pragma unroll
          for (int u = 0; u < XR; ++u) {
            const int l = sub + SL * u;
            if (l < i) sdot = fma(V[i + LD * l], x[u], sdot);
          }
          sdot = group_sum<SL>(sdot);
          const double xi = (j < c) ? (A[i + LD * j] - sdot) / V[i + LD * i] : 0.0;
          if (sub == i % SL) x[i / SL] = xi;
          if (sub == 0 && j < c) Vg[i + static_cast<size_t>(j) * ldv] = xi;
        }
      }
    }
  }
  for (int e = threadIdx.x; e < LD * c; e += NTH) {
    const int i = e % LD, j = e / LD;
    if (i < rows) Ag[i + static_cast<size_t>(j) * lda] = A[e];
    if (ACCV && i < c) Vg[i + static_cast<size_t>(j) * ldv] = V[e];
  }
  __syncthreads();
  if (threadIdx.x == 0 && info) {  // sweeps run, whether the last one rotated nothing, its largest |g|
    info[0] = nsw_;
    info[1] = (nsw_ == 0 || conv_) ? 1 : 0;
    const double gm = (nsw_ == 0 || conv_) ? 0.0 : __longlong_as_double(static_cast<long long>(gmax_));
    *reinterpret_cast<double*>(info + 2) = gm;
  }
}

// Block-pair step of a one-sided block Jacobi sweep for wide matrices: workgroup w
// takes the pair of column blocks given by the circle method for round `rd`,
// stages both blocks of A (rows x 2b) and of V (c x 2b) in LDS, runs inner Jacobi
// sweeps over their 2b columns (8 pairs at a time, 32 lanes per pair) until no
// rotation happens (at most 4), and writes them back.  *flag |= any rotation.
constexpr int BJ_B = 8;
__global__ __launch_bounds__(NT) void k_bjacobi_round(double* __restrict__ Ag, int rows, int c, int lda,
                                                      double* __restrict__ Vg, int ldv, int nb, int rd,
                                                      int32_t* __restrict__ flag) {
  extern __shared__ double sm[];
  __shared__ int cols_idx[2 * BJ_B];
  __shared__ int rot_any, rot_sweep;
  const int w = blockIdx.x;
  int P, Qb;
  if (w == 0) {
    P = rd;
    Qb = nb - 1;
  } else {
    P = (rd + w) % (nb - 1);
    Qb = (rd - w + (nb - 1)) % (nb - 1);
  }
  double* As = sm;                                           // rows x 2b
  double* Vs = sm + static_cast<size_t>(rows) * 2 * BJ_B;   // c x 2b
  if (threadIdx.x < 2 * BJ_B) {
    const int blk = (threadIdx.x < BJ_B) ? P : Qb;
    const int col = blk * BJ_B + (threadIdx.x % BJ_B);
    cols_idx[threadIdx.x] = (col < c) ? col : -1;
  }
  if (threadIdx.x == 0) rot_any = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < rows * 2 * BJ_B; e += NT) {
    const int i = e % rows, j = e / rows;
    const int col = cols_idx[j];
    As[e] = (col >= 0) ? Ag[i + static_cast<size_t>(col) * lda] : 0.0;
  }
  for (int e = threadIdx.x; e < c * 2 * BJ_B; e += NT) {
    const int i = e % c, j = e / c;
    const int col = cols_idx[j];
    Vs[e] = (col >= 0) ? Vg[i + static_cast<size_t>(col) * ldv] : 0.0;
  }
  __syncthreads();
  const int grp = threadIdx.x >> 5, gl = threadIdx.x & 31;
  constexpr int NL = 2 * BJ_B;
  const double tol = static_cast<double>(max(rows, 16)) * 2.220446049250313e-16;
  for (int inner = 0; inner < 4; ++inner) {
    if (threadIdx.x == 0) rot_sweep = 0;
    __syncthreads();
    for (int r2 = 0; r2 < NL - 1; ++r2) {
      const int k = grp;  // NL/2 = 8 pairs, 8 groups of 32 lanes
      int p, q;
      if (k == 0) {
        p = r2;
        q = NL - 1;
      } else {
        p = (r2 + k) % (NL - 1);
        q = (r2 - k + (NL - 1)) % (NL - 1);
      }
      if (p > q) {
        const int t = p;
        p = q;
        q = t;
      }
      if (cols_idx[p] >= 0 && cols_idx[q] >= 0) {
        double* ap = As + static_cast<size_t>(p) * rows;
        double* aq = As + static_cast<size_t>(q) * rows;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = gl; i < rows; i += 32) {
          const double x = ap[i], y = aq[i];
          a = fma(x, x, a);
          b = fma(y, y, b);
          g = fma(x, y, g);
        }
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
          a += __shfl_xor(a, o, 32);
          b += __shfl_xor(b, o, 32);
          g += __shfl_xor(g, o, 32);
        }
        if (a != 0.0 && b != 0.0 && fabs(g) > tol * sqrt(a) * sqrt(b)) {
          double cs, sn;
          jacobi_rotation(a, b, g, &cs, &sn);
          for (int i = gl; i < rows; i += 32) {
            const double x = ap[i], y = aq[i];
            ap[i] = cs * x - sn * y;
            aq[i] = sn * x + cs * y;
          }
          double* vp = Vs + static_cast<size_t>(p) * c;
          double* vq = Vs + static_cast<size_t>(q) * c;
          for (int i = gl; i < c; i += 32) {
            const double x = vp[i], y = vq[i];
            vp[i] = cs * x - sn * y;
            vq[i] = sn * x + cs * y;
          }
          if (gl == 0) {
            rot_sweep = 1;
            rot_any = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!rot_sweep) break;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < rows * 2 * BJ_B; e += NT) {
    const int i = e % rows, j = e / rows;
    const int col = cols_idx[j];
    if (col >= 0) Ag[i + static_cast<size_t>(col) * lda] = As[e];
  }
  for (int e = threadIdx.x; e < c * 2 * BJ_B; e += NT) {
    const int i = e % c, j = e / c;
    const int col = cols_idx[j];
    if (col >= 0) Vg[i + static_cast<size_t>(col) * ldv] = Vs[e];
  }
  if (threadIdx.x == 0 && rot_any) atomicOr(flag, 1);
}

__global__ __launch_bounds__(NT) void k_eye(double* __restrict__ V, int c, int ldv) {
  const long long e = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
  if (e >= static_cast<long long>(c) * c) return;
  const int i = static_cast<int>(e % c), j = static_cast<int>(e / c);
  V[i + static_cast<size_t>(j) * ldv] = (i == j) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(NT) void k_col_norms(const double* __restrict__ A, int rows, int c, int lda,
                                                  double* __restrict__ sigma) {
  __shared__ double red[NT / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < rows; i += NT) s = fma(A[i + static_cast<size_t>(j) * lda], A[i + static_cast<size_t>(j) * lda], s);
  s = wave_sum_f64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    sigma[j] = sqrt(t);
  }
}

__global__ __launch_bounds__(NT) void k_copy(const double* __restrict__ A, int rows, int cols, int lda,
                                             double* __restrict__ B, int ldb) {
  const long long e = static_cast<long long>(blockIdx.x) * NT + threadIdx.x;
  if (e >= static_cast<long long>(rows) * cols) return;
  const int i = static_cast<int>(e % rows), j = static_cast<int>(e / rows);
  B[i + static_cast<size_t>(j) * ldb] = A[i + static_cast<size_t>(j) * lda];
}

__global__ __launch_bounds__(NT) void k_transpose(const double* __restrict__ A, int rows, int cols, int lda,
                                                  double* __restrict__ B, int ldb) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = bx + tx, j = by + k;
    tile[k][tx] = (i < rows && j < cols) ? A[i + static_cast<size_t>(j) * lda] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = by + tx, i = bx + k;  // B[j, i] = A[i, j]
    if (i < rows && j < cols) B[j + static_cast<size_t>(i) * ldb] = tile[tx][k];
  }
}

__global__ __launch_bounds__(NT) void k_permute_cols(const double* __restrict__ A, int rows, int lda,
                                                     const int32_t* __restrict__ perm,
                                                     const double* __restrict__ scale, double* __restrict__ B,
                                                     int ldb) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= rows) return;
  const double sc = scale ? scale[t] : 1.0;
  B[i + static_cast<size_t>(t) * ldb] = A[i + static_cast<size_t>(perm[t]) * lda] * sc;
}

// One wave per column: entry of largest magnitude (lowest index on ties) made positive.
// Sign rule on columns of at most kSignRows rows: one workgroup per column finds the
// entry of largest magnitude (lowest index on ties; each thread's loads issued together)
// and, if it is negative, flips the column of U and the matching column of VS.
__global__ __launch_bounds__(NT) void k_sign_fix(double* __restrict__ U, int rows, int r, int ldu,
                                                 double* __restrict__ VS, int vrows, int ldv) {
  __shared__ double wb[NT / 64];
  __shared__ int wi[NT / 64];
  __shared__ int flip;
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* u = U + static_cast<size_t>(j) * ldu;
  double best = -1.0;
  int bi = rows;
  constexpr int PER = 4;
  for (int i0 = threadIdx.x; i0 < rows; i0 += NT * PER) {
    double a[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int i = i0 + t * NT;
      a[t] = (i < rows) ? fabs(u[i]) : -1.0;
    }
#pragma unroll
    for (int t = 0; t < PER; ++t)
      if (a[t] > best) {  // rows visited in increasing order per thread: ties keep the lower
        best = a[t];
        bi = i0 + t * NT;
      }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    wb[w] = best;
    wi[w] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = wb[0];
    int x = wi[0];
    for (int v = 1; v < NT / 64; ++v)
      if (wb[v] > b || (wb[v] == b && wi[v] < x)) {
        b = wb[v];
        x = wi[v];
      }
    flip = (x < rows && u[x] < 0.0) ? 1 : 0;
  }
  __syncthreads();
  if (!flip) return;
  for (int i = threadIdx.x; i < rows; i += NT) u[i] = -u[i];
  double* v = VS + static_cast<size_t>(j) * ldv;
  for (int i = threadIdx.x; i < vrows; i += NT) v[i] = -v[i];
}

// Tall columns: each workgroup finds the entry of largest magnitude (lowest index on
// ties) of one slice of rows of one column; slices are combined in order by
// k_sign_decide, and k_apply_sign flips the columns whose entry is negative.
constexpr int kSignRows = 4096;  // longer columns take the sliced path
__global__ __launch_bounds__(NT) void k_colmax_slices(const double* __restrict__ U, int rows, int ldu, int slice,
                                                      double* __restrict__ pabs, int* __restrict__ pidx,
                                                      double* __restrict__ pval) {
  __shared__ double sb[NT];
  __shared__ int si[NT];
  const int j = blockIdx.y, sl = blockIdx.x;
  const int i0 = sl * slice, i1 = min(rows, i0 + slice);
  const double* u = U + static_cast<size_t>(j) * ldu;
  double best = -1.0;
  int bi = rows;
  for (int i = i0 + threadIdx.x; i < i1; i += 4 * NT) {
    double a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = (i + t * NT < i1) ? fabs(u[i + t * NT]) : -1.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (a[t] > best) {  // increasing index within a thread: a tie keeps the earlier one
        best = a[t];
        bi = i + t * NT;
      }
  }
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double ob = sb[threadIdx.x + o];
      const int oi = si[threadIdx.x + o];
      if (ob > sb[threadIdx.x] || (ob == sb[threadIdx.x] && oi < si[threadIdx.x])) {
        sb[threadIdx.x] = ob;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int q = j * gridDim.x + sl;
    pabs[q] = sb[0];
    pidx[q] = si[0];
    pval[q] = si[0] < rows ? u[si[0]] : 0.0;
  }
}

__global__ __launch_bounds__(NT) void k_sign_decide(const double* __restrict__ pabs, const int* __restrict__ pidx,
                                                    const double* __restrict__ pval, int nslices, int r,
                                                    double* __restrict__ sgn) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= r) return;
  double best = -1.0, v = 0.0;
  int bi = 0x7fffffff;
  for (int sl = 0; sl < nslices; ++sl) {  // slices in row order: a tie keeps the earlier one
    const int q = j * nslices + sl;
    if (pabs[q] > best || (pabs[q] == best && pidx[q] < bi)) {
      best = pabs[q];
      bi = pidx[q];
      v = pval[q];
    }
  }
  sgn[j] = (v < 0.0) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(NT) void k_apply_sign(double* __restrict__ X, int rows, int cols, int ld,
                                                   const double* __restrict__ sgn) {
  const size_t e = static_cast<size_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= static_cast<size_t>(rows) * cols) return;
  const int j = static_cast<int>(e / rows), i = static_cast<int>(e - static_cast<size_t>(j) * rows);
  if (sgn[j] < 0.0) X[i + static_cast<size_t>(j) * ld] = -X[i + static_cast<size_t>(j) * ld];
}

}  // namespace

void gemm_prec(Allocator* al, int prec, bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
               int lda, const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  // C = A^T A: compute the upper tiles only
  const bool sym = ta && !tb && A == B && lda == ldb && m == n;
  const int kstep = (prec == TT_FP64) ? GK : 32;
  const int tm = (m + GT - 1) / GT, tn = (n + GT - 1) / GT;
  const int tiles = sym ? tm * (tm + 1) / 2 : tm * tn;
  int ns = 1;
  // split K until about 1024 workgroups (a few per CU, so that the k-stage latency
  // of one overlaps another's) with at least 32 rows of K each: a workgroup's k-stages
  // each wait for memory, so a short chunk finishes sooner.  The partial sums are kept
  // to at most 2^21 values (16 MB, a few microseconds for the reduction to read).
  if (tiles < 256 && k > 32) {
    const int64_t mn = static_cast<int64_t>(m) * n;
    const int cap_part = static_cast<int>(std::max<int64_t>(1, (int64_t(1) << 21) / mn));
    ns = std::min({(k + 31) / 32, std::max(1, 1024 / tiles), 256, cap_part});
  }
  int kchunk = (k + ns - 1) / ns;
  kchunk = ((kchunk + kstep - 1) / kstep) * kstep;
  if (kchunk == 0) kchunk = kstep;
  ns = std::max(1, (k + kchunk - 1) / kchunk);
  KTimer kt(prec == TT_FP64 ? "gemm" : "gemm_lp", s,
            8.0 * (static_cast<double>(m) * k + static_cast<double>(k) * n + static_cast<double>(m) * n),
            2.0 * static_cast<double>(m) * n * k);
  // a few column tiles: linear tile order with the column index fastest, so that the
  // tiles sharing a block of rows of op(A) run together and it is read from HBM once
  const int lin_tn = (!sym && tn > 1 && tn <= 8 && static_cast<int64_t>(tm) * tn < (int64_t(1) << 31)) ? tn : 0;
  const dim3 grid = sym ? dim3(tiles, 1, ns) : lin_tn ? dim3(tm * tn, 1, ns) : dim3(tm, tn, ns);
  DBuf<double> part;
  if (ns > 1) part.reset(al, static_cast<size_t>(ns) * m * n);
  const int kc = (ns == 1) ? std::max(kchunk, k) : kchunk;
  double* pp = (ns == 1) ? nullptr : part.get();
  if (prec == TT_FP64)
    k_gemm<<<grid, NT, 0, s>>>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kc, pp, sym, lin_tn);
  else if (prec == TT_FP32)
    k_gemm_lp<0><<<grid, NT, 0, s>>>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kc, pp, sym, lin_tn);
  else
    k_gemm_lp<1><<<grid, NT, 0, s>>>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, kc, pp, sym, lin_tn);
  TTS_LAUNCH_CHECK();
  if (ns > 1) {
    const size_t mn = static_cast<size_t>(m) * n;
    if (ns >= 32)
      k_gemm_reduce<8><<<grid_for(mn * 8, NT), NT, 0, s>>>(m, n, ns, part.get(), alpha, beta, C, ldc);
    else if (ns >= 8)
      k_gemm_reduce<2><<<grid_for(mn * 2, NT), NT, 0, s>>>(m, n, ns, part.get(), alpha, beta, C, ldc);
    else
      k_gemm_reduce<1><<<grid_for(mn, NT), NT, 0, s>>>(m, n, ns, part.get(), alpha, beta, C, ldc);
    TTS_LAUNCH_CHECK();
  }
}

void gemm(Allocator* al, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  gemm_prec(al, TT_FP64, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

void to_f32(const double* x, size_t n, float* y, hipStream_t s) {
  if (n == 0) return;
  k_to_f32<<<grid_for(n, NT), NT, 0, s>>>(x, n, y);
  TTS_LAUNCH_CHECK();
}

void spmm_left(const double* W, int r, int ldw, const int64_t* colptr, const int32_t* row, const double* val,
               int ncols, int nk, double* X, int ldx, hipStream_t s) {
  if (r <= 0 || ncols <= 0) return;
  k_spmm_left<<<dim3(grid_for(r, NT), ncols), NT, 0, s>>>(W, r, ldw, colptr, row, val, nk, X, ldx);
  TTS_LAUNCH_CHECK();
}

void right_weights(Allocator* al, const int64_t* colptr, const int32_t* row, const double* val, int ncols,
                   uint32_t nnz, int nk, int ngroups, const double* wnext, double* w, hipStream_t s) {
  DBuf<uint64_t> key(al, nnz), ent(al, nnz), kt(al, nnz), vt(al, nnz);
  DBuf<uint32_t> ecol(al, nnz);
  k_expand_cols<<<grid_for(ncols, NT), NT, 0, s>>>(colptr, ncols, row, key.get(), ent.get(), ecol.get());
  TTS_LAUNCH_CHECK();
  int bits = 0;
  while (bits < 63 && (static_cast<uint64_t>(ngroups) * nk - 1) >> bits) ++bits;
  if (radix_sort_pairs_pp(al, key.get(), ent.get(), kt.get(), vt.get(), nnz, bits, s)) {
    key.swap(kt);
    ent.swap(vt);
  }
  k_group_weights<<<grid_for(ngroups, NT), NT, 0, s>>>(key.get(), ent.get(), nnz, nk, ngroups, val, ecol.get(), wnext,
                                                       w);
  TTS_LAUNCH_CHECK();
}

void row_sumsq(const double* G, int ngroups, int nk, double* w, hipStream_t s) {
  k_row_sumsq<<<grid_for(ngroups, NT), NT, 0, s>>>(G, ngroups, nk, w);
  TTS_LAUNCH_CHECK();
}

void scale_cols_sqrt(const double* X, int rows, int cols, int ldx, const double* w, double* Y, int ldy,
                     hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  k_scale_cols<<<dim3(grid_for(rows, NT), cols), NT, 0, s>>>(X, rows, ldx, nullptr, w, Y, ldy);
  TTS_LAUNCH_CHECK();
}

void gather_cols(const double* X, int rows, int ldx, const int32_t* piv, int r, const double* w, double* Y, int ldy,
                 hipStream_t s) {
  if (rows <= 0 || r <= 0) return;
  k_scale_cols<<<dim3(grid_for(rows, NT), r), NT, 0, s>>>(X, rows, ldx, piv, w, Y, ldy);
  TTS_LAUNCH_CHECK();
}

void pivoted_cholesky(const double* G, int n, int ldg, int rmax, double theta, double* L, int32_t* piv, int32_t* d_r,
                      hipStream_t s) {
  const size_t base = sizeof(double) * static_cast<size_t>(n);
  const size_t cap = 150 * 1024;
  if (base > cap) fail(TT_ERR_TOO_LARGE, "pivoted Cholesky: Gram matrix too large for one workgroup");
  // as many leading columns of L as fit are kept in LDS
  const int tl = static_cast<int>(std::min<size_t>(rmax, (cap - base) / (sizeof(double) * n)));
  const size_t shm = base + sizeof(double) * static_cast<size_t>(n) * tl;
  const size_t shm_block = sizeof(double) * (static_cast<size_t>(n) + static_cast<size_t>(PB_KB) * rmax);
  if (n > 32 && shm_block <= cap) {
    k_pivchol_block<<<1, PB_NTH, shm_block, s>>>(G, n, ldg, rmax, theta, L, piv, d_r);
  } else if (n <= 64) {
    k_pivchol_lds<8, 8, 512><<<1, 512, sizeof(double) * n * n, s>>>(G, n, ldg, rmax, theta, L, piv, d_r);
  } else if (n <= 128) {
    k_pivchol_lds<4, 32, 512><<<1, 512, sizeof(double) * n * n, s>>>(G, n, ldg, rmax, theta, L, piv, d_r);
  } else if (n * 16 <= BT)
    k_pivoted_cholesky<16><<<1, BT, shm, s>>>(G, n, ldg, rmax, theta, L, piv, d_r, tl);
  else if (n * 8 <= BT)
    k_pivoted_cholesky<8><<<1, BT, shm, s>>>(G, n, ldg, rmax, theta, L, piv, d_r, tl);
  else if (n * 4 <= BT)
    k_pivoted_cholesky<4><<<1, BT, shm, s>>>(G, n, ldg, rmax, theta, L, piv, d_r, tl);
  else if (n * 2 <= BT)
    k_pivoted_cholesky<2><<<1, BT, shm, s>>>(G, n, ldg, rmax, theta, L, piv, d_r, tl);
  else
    k_pivoted_cholesky<1><<<1, BT, shm, s>>>(G, n, ldg, rmax, theta, L, piv, d_r, tl);
  TTS_LAUNCH_CHECK();
}

void pivot_factor(const double* L, int n, const int32_t* piv, int r, double* U, hipStream_t s) {
  k_pivot_factor<<<grid_for(static_cast<size_t>(r) * r, NT), NT, 0, s>>>(L, n, piv, r, U);
  TTS_LAUNCH_CHECK();
}

void cholesky_upper(double* A, int r, int lda, double max_ratio, int32_t* d_ok, hipStream_t s) {
  // r^3 / 3 multiply-adds; the matrix is read and written once
  KTimer kt("cholesky", s, 16.0 * r * r, 2.0 * r * r * r / 3.0);
  if (r <= 64) {
    k_cholesky_mfma<64><<<1, 256, 0, s>>>(A, r, lda, max_ratio, d_ok);
    TTS_LAUNCH_CHECK();
    return;
  }
  if (r <= 128) {
    k_cholesky_mfma<128><<<1, 256, 0, s>>>(A, r, lda, max_ratio, d_ok);
    TTS_LAUNCH_CHECK();
    return;
  }
  k_cholesky_upper<<<1, BT, 0, s>>>(A, r, lda, max_ratio, d_ok);
  TTS_LAUNCH_CHECK();
}

namespace {

// X = Y U^{-1}.  Up to 64 columns by substitution kernels; wider U in blocks of 64
// columns: X1 = Y1 U11^{-1}, then X2 = (Y2 - X1 U12) U22^{-1} (GEMM update).
void trsm_blocks(const double* Y, int rows, int r, int ldy, const double* U, int ldu, double* X, int ldx,
                 int32_t* d_ok, hipStream_t s, Allocator* al) {
  if (r <= 64 && rows >= 256) {
    k_trsm_mfma<<<grid_for(rows, 64), 256, 0, s>>>(Y, rows, r, ldy, U, ldu, X, ldx, d_ok);
    TTS_LAUNCH_CHECK();
    return;
  }
  if (r <= 64) {
    if (r <= 32)
      k_trsm_right_upper<32><<<grid_for(rows, 64), 64, 0, s>>>(Y, rows, r, ldy, U, ldu, X, ldx, d_ok);
    else
      k_trsm_right_upper<64><<<grid_for(rows, 64), 64, 0, s>>>(Y, rows, r, ldy, U, ldu, X, ldx, d_ok);
    TTS_LAUNCH_CHECK();
    return;
  }
  constexpr int B = 64;
  const int r2 = r - B;
  DBuf<double> Y2(al, static_cast<size_t>(rows) * r2);
  copy_matrix(Y + static_cast<size_t>(B) * ldy, rows, r2, ldy, Y2.get(), rows, s);
  trsm_blocks(Y, rows, B, ldy, U, ldu, X, ldx, d_ok, s, al);
  gemm(al, false, false, rows, r2, B, -1.0, X, ldx, U + static_cast<size_t>(B) * ldu, ldu, 1.0, Y2.get(), rows, s);
  trsm_blocks(Y2.get(), rows, r2, rows, U + B + static_cast<size_t>(B) * ldu, ldu, X + static_cast<size_t>(B) * ldx,
              ldx, d_ok, s, al);
}

}  // namespace

void trsm_right_upper(const double* Y, int rows, int r, int ldy, const double* U, int ldu, double* X, int ldx,
                      int32_t* d_ok, hipStream_t s, Allocator* al) {
  if (rows <= 0 || r <= 0) return;
  // rows * r^2 / 2 multiply-adds; Y read, X written, U read once
  KTimer kt("trsm", s, 8.0 * (2.0 * rows * r + static_cast<double>(r) * r), static_cast<double>(rows) * r * r);
  trsm_blocks(Y, rows, r, ldy, U, ldu, X, ldx, d_ok, s, al);
}

void weighted_sumsq(Allocator* al, const double* E, int rows, int cols, int lde, const double* w, double* d_out,
                    hipStream_t s) {
  DBuf<double> cs(al, std::max(cols, 1));
  if (cols > 0) {
    k_col_sumsq<<<cols, NT, 0, s>>>(E, rows, lde, cs.get());
    TTS_LAUNCH_CHECK();
  }
  k_weighted_total<<<1, NT, 0, s>>>(cs.get(), w, cols, d_out);
  TTS_LAUNCH_CHECK();
}

void householder_qr(double* A, int m, int n, int lda, double* tau, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  k_householder_qr<<<1, BT, 0, s>>>(A, m, n, lda, tau);
  TTS_LAUNCH_CHECK();
}

void householder_form_q(const double* A, int m, int p, int lda, const double* tau, double* Q, int ldq, hipStream_t s) {
  if (m <= 0 || p <= 0) return;
  k_householder_form_q<<<1, BT, 0, s>>>(A, m, p, lda, tau, Q, ldq);
  TTS_LAUNCH_CHECK();
}

void qr_explicit(Allocator* al, const double* G, int m, int n, int ldg, double* Q, int ldq, double* R, int ldr,
                 hipStream_t s) {
  const int p = std::min(m, n);
  if (p <= 0) return;
  // tall: row blocks of b >= 2n rows (at least 256), factored in parallel
  const int b = std::max(256, 2 * n);
  if (m < 4 * b) {
    DBuf<double> Af(al, static_cast<size_t>(m) * n), th(al, p);
    copy_matrix(G, m, n, ldg, Af.get(), m, s);
    householder_qr(Af.get(), m, n, m, th.get(), s);
    householder_form_q(Af.get(), m, p, m, th.get(), Q, ldq, s);
    householder_extract_r(Af.get(), m, n, m, R, ldr, Q, ldq, s);
    return;
  }
  const int nblk = m / b;  // the last block takes the remainder
  const int ls = nblk * n;
  DBuf<double> Af(al, static_cast<size_t>(m) * n), tb(al, static_cast<size_t>(nblk) * n),
      Qb(al, static_cast<size_t>(m) * n), S(al, static_cast<size_t>(ls) * n), QS(al, static_cast<size_t>(ls) * n);
  copy_matrix(G, m, n, ldg, Af.get(), m, s);
  k_householder_qr_blocks<<<nblk, BT, 0, s>>>(Af.get(), m, n, m, b, nblk, tb.get());
  TTS_LAUNCH_CHECK();
  k_stack_r<<<grid_for(static_cast<size_t>(ls) * n, NT), NT, 0, s>>>(Af.get(), n, m, b, nblk, S.get());
  TTS_LAUNCH_CHECK();
  k_householder_form_q_blocks<<<nblk, BT, 0, s>>>(Af.get(), m, n, m, b, nblk, tb.get(), Qb.get(), m);
  TTS_LAUNCH_CHECK();
  // the stack (nblk n rows) the same way: blocks again while it is tall, R with diag >= 0
  qr_explicit(al, S.get(), ls, n, ls, QS.get(), ls, R, ldr, s);
  k_tsqr_combine<<<grid_for(static_cast<size_t>(m), NT), NT, 0, s>>>(Qb.get(), m, n, b, nblk, QS.get(), Q, ldq);
  TTS_LAUNCH_CHECK();
}

void householder_extract_r(const double* A, int m, int n, int lda, double* R, int ldr, double* Q, int ldq,
                           hipStream_t s) {
  const int p = std::min(m, n);
  if (p <= 0) return;
  k_extract_r<<<grid_for(static_cast<size_t>(p) * n, NT), NT, 0, s>>>(A, p, n, lda, R, ldr);
  TTS_LAUNCH_CHECK();
  if (Q) {
    k_flip_q<<<grid_for(static_cast<size_t>(m) * p, NT), NT, 0, s>>>(A, m, p, lda, Q, ldq);
    TTS_LAUNCH_CHECK();
  }
}

namespace {
__global__ void k_set_info(int32_t* info, int32_t sweeps, int32_t converged) {
  info[0] = sweeps;
  info[1] = converged;
  // the block kernel keeps no largest rotated product: unknown unless converged
  *reinterpret_cast<double*>(info + 2) = converged ? 0.0 : __builtin_inf();
}

// Sweep cap of the Jacobi kernels: 80, or TTSPARSE_JACOBI_MAX_SWEEPS (1..80), which
// exists to exercise the non-convergence path from the host.
int jacobi_sweep_cap() {
  static const int cap = [] {
    const char* e = std::getenv("TTSPARSE_JACOBI_MAX_SWEEPS");
    const int v = e ? std::atoi(e) : 0;
    return (v >= 1 && v <= 80) ? v : 80;
  }();
  return cap;
}
}  // namespace

bool jacobi_svd(double* A, int rows, int c, int lda, double* V, int ldv, double* sigma, int32_t* info, hipStream_t s,
                bool lower_tri, bool want_v) {
  if (c <= 0) return false;
  const int ms = jacobi_sweep_cap();
  const size_t shm = sizeof(double) * (static_cast<size_t>(rows) * c + static_cast<size_t>(c) * c);
  // rotations left unaccumulated (triangular input of 16 < c <= 64 columns)
  const bool nov = lower_tri && rows == c && c > 16 && c <= 64 && info != nullptr;
  KTimer kt("jacobi", s, 8.0 * 2.0 * (static_cast<double>(rows) * c + static_cast<double>(c) * c),
            // per sweep: c(c-1)/2 pairs x (3 dots + 2 column updates of A, and of V when
            // accumulated); the timer multiplies it by the sweeps the launch reports in
            // info[0]
            0.5 * static_cast<double>(c) * (c - 1) * (6.0 * rows + 6.0 * rows + (nov ? 0.0 : 6.0 * c)));
  kt.flops_per_count(info);
  const size_t shm_odd = sizeof(double) * (static_cast<size_t>(rows | 1) * c + static_cast<size_t>(c | 1) * c);
  if (c > 32 && c <= 64 && rows <= 64) {
    if (nov)
      k_jacobi64h<64, false><<<1, 256, 0, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info, want_v ? 1 : 0);
    else
      k_jacobi64h<64, true><<<1, 256, 0, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info, 1);
    TTS_LAUNCH_CHECK();
    return nov;
  }
  if (c > 16 && c <= 32 && rows <= 64) {
    if (nov)
      k_jacobi64h<32, false><<<1, 256, 0, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info, want_v ? 1 : 0);
    else
      k_jacobi64h<32, true><<<1, 256, 0, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info, 1);
    TTS_LAUNCH_CHECK();
    return nov;
  }
  if (c <= 64 && rows <= 64) {
    k_jacobi64<<<1, 256, sizeof(double) * 128 * static_cast<size_t>(c), s>>>(A, rows, c, lda, V, ldv, sigma, ms,
                                                                               info);
    TTS_LAUNCH_CHECK();
    return false;
  }
  if (shm_odd <= 150 * 1024 && c <= 64 && rows <= 256) {
    if (rows <= 128)
      k_jacobi_reg<16, 8><<<1, 512, shm_odd, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info);
    else
      k_jacobi_reg<32, 8><<<1, 1024, shm_odd, s>>>(A, rows, c, lda, V, ldv, sigma, ms, info);
    TTS_LAUNCH_CHECK();
    return false;
  }
  // A and V in registers: 64 < c <= 128 columns of at most 128 rows
  if (c > 64 && c <= 128 && rows <= 128) {
    const int H = (c + 1) / 2;
    k_jacobi_oe<8><<<1, 1024, sizeof(double) * 2 * 8 * 16 * static_cast<size_t>(H), s>>>(A, rows, c, lda, V, ldv,
                                                                                         sigma, ms, info);
    TTS_LAUNCH_CHECK();
    return false;
  }
  // A in LDS with the rotations logged, then V in LDS: up to 138 columns
  if (shm > 150 * 1024 && c <= 138 && rows <= 160 && sizeof(double) * static_cast<size_t>(rows) * c <= 150 * 1024) {
    constexpr int kMaxSweeps = 80;  // the rotation log holds this many sweeps
    const int N = c + (c & 1);
    const size_t lbytes = sizeof(double2) * static_cast<size_t>(kMaxSweeps) * (N - 1) * (N / 2);
    void* lg = cached_alloc(lbytes, s);
    if (!lg) fail(TT_ERR_NOMEM, "device allocation failed");
    const size_t lshm = sizeof(double) * std::max(static_cast<size_t>(rows) * c, static_cast<size_t>(c) * c);
    k_jacobi_log<1024, 16, 10><<<1, 1024, lshm, s>>>(A, rows, c, lda, V, ldv, sigma, static_cast<double2*>(lg),
                                                      std::min(ms, kMaxSweeps), info);
    TTS_LAUNCH_CHECK();
    cached_free(lg, lbytes, s);
    return false;
  }
  // A in LDS, V in global memory: up to 160 columns
  if (shm > 150 * 1024 && c <= 160 && rows <= 160 && sizeof(double) * static_cast<size_t>(rows) * c <= 150 * 1024) {
    k_jacobi_lv<1024, 16, 10><<<1, 1024, sizeof(double) * static_cast<size_t>(rows) * c, s>>>(A, rows, c, lda, V,
                                                                                             ldv, sigma, ms, info);
    TTS_LAUNCH_CHECK();
    return false;
  }
  if (shm <= 150 * 1024 || c <= 2 * BJ_B) {
    const int use_lds = shm <= 150 * 1024;
    k_jacobi<BT, 16><<<1, BT, use_lds ? shm : 0, s>>>(A, rows, c, lda, V, ldv, sigma, use_lds, ms, info);
    TTS_LAUNCH_CHECK();
    return false;
  }
  // wide: block Jacobi, one launch per round of block pairs
  const size_t bshm = sizeof(double) * 2 * BJ_B * (static_cast<size_t>(rows) + c);
  if (bshm > 150 * 1024) fail(TT_ERR_TOO_LARGE, "Jacobi SVD: matrix too large for the block kernel");
  int nb = (c + BJ_B - 1) / BJ_B;
  nb += nb & 1;
  k_eye<<<grid_for(static_cast<size_t>(c) * c, NT), NT, 0, s>>>(V, c, ldv);
  TTS_LAUNCH_CHECK();
  int32_t* flag = static_cast<int32_t*>(cached_alloc(sizeof(int32_t), s));
  if (!flag) fail(TT_ERR_NOMEM, "device allocation failed");
  int32_t hflag = 1;
  int sweeps = 0;
  const int bcap = std::min(ms, 60);
  for (int sweep = 0; sweep < bcap && hflag; ++sweep) {
    TTS_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    for (int rd = 0; rd < nb - 1; ++rd) {
      k_bjacobi_round<<<nb / 2, NT, bshm, s>>>(A, rows, c, lda, V, ldv, nb, rd, flag);
      TTS_LAUNCH_CHECK();
    }
    {
      Readback rb(s);
      rb.add(&hflag, flag, sizeof(int32_t));
      rb.sync();
    }
    sweeps = sweep + 1;
  }
  cached_free(flag, sizeof(int32_t), s);
  k_col_norms<<<c, NT, 0, s>>>(A, rows, c, lda, sigma);
  TTS_LAUNCH_CHECK();
  if (info) {
    k_set_info<<<1, 1, 0, s>>>(info, sweeps, hflag ? 0 : 1);
    TTS_LAUNCH_CHECK();
  }
  return false;
}

void copy_matrix(const double* A, int rows, int cols, int lda, double* B, int ldb, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  k_copy<<<grid_for(static_cast<size_t>(rows) * cols, NT), NT, 0, s>>>(A, rows, cols, lda, B, ldb);
  TTS_LAUNCH_CHECK();
}

void transpose(const double* A, int rows, int cols, int lda, double* B, int ldb, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  k_transpose<<<dim3((rows + 31) / 32, (cols + 31) / 32), NT, 0, s>>>(A, rows, cols, lda, B, ldb);
  TTS_LAUNCH_CHECK();
}

void permute_cols(const double* A, int rows, int lda, const int32_t* perm, const double* scale, int cols, double* B,
                  int ldb, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  k_permute_cols<<<dim3(grid_for(rows, NT), cols), NT, 0, s>>>(A, rows, lda, perm, scale, B, ldb);
  TTS_LAUNCH_CHECK();
}

void sign_fix(double* U, int rows, int r, int ldu, double* VS, int vrows, int ldv, hipStream_t s) {
  if (r <= 0) return;
  if (rows <= kSignRows) {
    k_sign_fix<<<r, NT, 0, s>>>(U, rows, r, ldu, VS, vrows, ldv);
    TTS_LAUNCH_CHECK();
    return;
  }
  // about 2048 workgroups over r columns, slices of at least 4 NT rows
  int ns = std::max(1, std::min((rows + 4 * NT - 1) / (4 * NT), 2048 / std::max(1, r)));
  const int slice = (rows + ns - 1) / ns;
  ns = (rows + slice - 1) / slice;
  const size_t np = static_cast<size_t>(ns) * r;
  const size_t bytes = np * (2 * sizeof(double) + sizeof(int)) + sizeof(double) * r;
  char* buf = static_cast<char*>(cached_alloc(bytes, s));
  if (!buf) fail(TT_ERR_NOMEM, "device allocation failed");
  double* pabs = reinterpret_cast<double*>(buf);
  double* pval = pabs + np;
  double* sgn = pval + np;
  int* pidx = reinterpret_cast<int*>(sgn + r);
  k_colmax_slices<<<dim3(ns, r), NT, 0, s>>>(U, rows, ldu, slice, pabs, pidx, pval);
  TTS_LAUNCH_CHECK();
  k_sign_decide<<<(r + NT - 1) / NT, NT, 0, s>>>(pabs, pidx, pval, ns, r, sgn);
  TTS_LAUNCH_CHECK();
  k_apply_sign<<<grid_for(static_cast<size_t>(rows) * r, NT), NT, 0, s>>>(U, rows, r, ldu, sgn);
  TTS_LAUNCH_CHECK();
  k_apply_sign<<<grid_for(static_cast<size_t>(vrows) * r, NT), NT, 0, s>>>(VS, vrows, r, ldv, sgn);
  TTS_LAUNCH_CHECK();
  cached_free(buf, bytes, s);
}

}  // namespace tts
