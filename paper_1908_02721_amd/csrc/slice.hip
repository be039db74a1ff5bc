// Bond-2 Gram slice of the left-to-right QR sweep (TT-rounding, Alg 2 run left to
// right) on the exact sparse TT, for tensors whose second bond is too wide to
// factor on one device:
//
//   bond 1  X_1 = unfold_2(G^(1)) (n_1 x beta_1) = Q_1 R_1.  A wide X_1 leaves Q_1
//           free up to an orthogonal factor; the gauge is fixed by the SVD: Q_1 =
//           left singular vectors (sigma non-ascending, largest-magnitude entry of
//           each column positive), R_1 = Q_1^T X_1, all in FP64.  Computed as
//           CholeskyQR2 of X_1^T = Q R (Householder on breakdown), one-sided Jacobi
//           on R (R V = W Sigma, so V are the left singular vectors of X_1 and need
//           no division by sigma), then R_1 = Q_1^T X_1 on the FP64 matrix cores.
//   X_2     = unfold_2(R_1 x_1 G^(2)), block-sparse: block (j, i) is the m-vector
//           sum over the entries (rho = g n_2 + i, column j, value c) of N_2 of
//           c R_1[:, g].  Blocks are stored slot-major (by i, then j).  Nearly every
//           block is one scaled column of R_1, so this is a gather (HBM-bound on the
//           write of X_2), done on the vector units in the precision of the mode:
//           FP64; or binary32 operands / bfloat16 operands, FP32 accumulation, FP32
//           storage.
//   Gram    Gamma = X_2 diag(w_2) X_2^T, w_2 the squared row norms of the right part
//           of bond 2, FP64 on the matrix cores.  Rows are slot-major (q = i m + a);
//           block (i, i2) = sum over the columns j holding both slots of
//           w_2[j] x_{j,i} x_{j,i2}^T.  Only blocks i <= i2 are formed (symmetry),
//           stored packed, each m x m row-major.  Diagonal blocks take every block
//           of the slot; off-diagonal blocks take the (i, i2) pairs of the columns,
//           listed by one sort.  Work items of at most 2048 pairs go to one
//           512-thread workgroup each (largest first); items of a split block
//           write partial blocks summed afterwards in item order (deterministic).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "dense.hpp"
#include "linalg.hpp"
#include "prim.hpp"
#include "slice.hpp"

namespace tts {

namespace {

constexpr int NT = 256;
constexpr int kMaxM = 208;       // 13 MFMA tiles of 16
constexpr int kGramThreads = 512;
constexpr int kGramWaves = kGramThreads / 64;
constexpr int kKC = 16;          // pairs per LDS stage (four k-steps of the 16x16x4 MFMA)
constexpr int kItemPairs = 2048; // pairs per work item

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GramItem {
  int32_t kind;     // 0: diagonal block (blocks [start, start+nk) of one slot); 1: off-diagonal (pairs)
  int32_t nk;       // number of blocks / pairs
  int32_t to_part;  // 1: write to the partial buffer
  int32_t tile0;    // first output tile (row-major over the MT x MT tiles) of this item
  int64_t start;
  int64_t dst;      // element offset of the m x m destination
};

// Output tiles of a block are split over several items so that a wave holds at most
// 11 (off-diagonal) or 12 (diagonal) accumulator tiles: within the 256 registers of
// two waves per SIMD, and enough for the 91 upper tiles of a diagonal block at
// m = 208 to need no split.  Off-diagonal blocks take all MT x MT tiles; diagonal
// blocks (symmetric) only the MT (MT + 1) / 2 tiles on or above the diagonal, each
// mirrored.
constexpr int kTilesPerWave = 11;
__host__ __device__ constexpr int tiles_of(int mt, int kind) { return kind == 0 ? mt * (mt + 1) / 2 : mt * mt; }
__host__ __device__ constexpr int tiles_per_wave(int kind) { return kind == 0 ? 12 : kTilesPerWave; }
__host__ __device__ constexpr int gram_split(int mt, int kind) {
  return (tiles_of(mt, kind) + tiles_per_wave(kind) * 8 - 1) / (tiles_per_wave(kind) * 8);
}
__host__ __device__ constexpr int tiles_per_item(int mt, int kind) {
  return (tiles_of(mt, kind) + gram_split(mt, kind) - 1) / gram_split(mt, kind);
}

// X_1 (n_1 x beta_1, column-major): column b of N_1 (rows rho = i_1 since r_0 = 1)
__global__ __launch_bounds__(NT) void k_slice_x1(const int64_t* __restrict__ colptr, int ncols,
                                                 const int32_t* __restrict__ row, const double* __restrict__ val,
                                                 int n1, double* __restrict__ X1, int32_t* __restrict__ rowflag,
                                                 int32_t* __restrict__ nzrows) {
  const int b = blockIdx.x * NT + threadIdx.x;
  if (b >= ncols) return;
  for (int64_t e = colptr[b]; e < colptr[b + 1]; ++e) {
    const int r = row[e];
    X1[static_cast<size_t>(b) * n1 + r] = val[e];
    if (atomicExch(&rowflag[r], 1) == 0) atomicAdd(nzrows, 1);
  }
}

// Entries of N_2 keyed (slot, column) for the slot-major block order; value = entry index.
__global__ __launch_bounds__(NT) void k_x2_keys(const int64_t* __restrict__ colptr, int ncols,
                                                const int32_t* __restrict__ row, int n2, int cbits,
                                                uint64_t* __restrict__ key, uint64_t* __restrict__ ent) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= ncols) return;
  for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
    const uint64_t slot = static_cast<uint64_t>(row[e] % n2);
    key[e] = (slot << cbits) | static_cast<uint64_t>(j);
    ent[e] = static_cast<uint64_t>(e);
  }
}

__global__ __launch_bounds__(NT) void k_run_flags(const uint64_t* __restrict__ key, uint32_t n,
                                                  uint32_t* __restrict__ flag) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e >= n) return;
  flag[e] = (e == 0 || key[e] != key[e - 1]) ? 1u : 0u;
}

// Per block: first entry, slot and column.
__global__ __launch_bounds__(NT) void k_block_info(const uint64_t* __restrict__ key, const uint32_t* __restrict__ flag,
                                                   const uint32_t* __restrict__ pos, uint32_t n, int cbits,
                                                   uint32_t nb, int64_t* __restrict__ bstart,
                                                   int32_t* __restrict__ bslot, int32_t* __restrict__ bcol) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e == 0) bstart[nb] = n;
  if (e >= n || !flag[e]) return;
  const uint32_t b = pos[e];
  bstart[b] = e;
  bslot[b] = static_cast<int32_t>(key[e] >> cbits);
  bcol[b] = static_cast<int32_t>(key[e] & ((1ull << cbits) - 1ull));
}

// out[t] = first index i in [0, n) with a[i] >= t (a ascending), t = 0..nt-1
__global__ __launch_bounds__(NT) void k_lower_bound_i32(const int32_t* __restrict__ a, int64_t n, int64_t nt,
                                                        int64_t* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (t >= nt) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  out[t] = lo;
}

__global__ __launch_bounds__(NT) void k_lower_bound_u64(const uint64_t* __restrict__ a, int64_t n, int64_t nt,
                                                        int64_t* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (t >= nt) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < static_cast<uint64_t>(t)) lo = mid + 1;
    else hi = mid;
  }
  out[t] = lo;
}

// Operands in the precision of the mode.
template <int P>
__device__ __forceinline__ float lp(double x) {
  const float f = static_cast<float>(x);
  if (P == TT_BF16_FP32ACC) return static_cast<float>(static_cast<__bf16>(f));
  return f;
}

// X_2 blocks.  A wave takes 64 consecutive blocks at a time: lane l loads the
// metadata of block b0 + l (and, for a one-entry block, its entry), then the wave
// forms the blocks one by one from those registers, lane a of each m-vector
// sum of c R_1[:, g] (operands rounded to the mode's precision, FP32 accumulation
// in the reduced modes).  Also the block weights and each wave's partial of
// sum_b w_b ||x_b||^2, formed in FP64 from the stored values.
template <typename T, int P>
__device__ __forceinline__ T x2_term(double c, double r, T acc) {
  if (P == TT_FP64) return fma(c, r, acc);
  return fmaf(lp<P>(c), lp<P>(r), acc);
}

template <typename T, int P>
__global__ __launch_bounds__(NT) void k_x2_fill(const int64_t* __restrict__ bstart, const int32_t* __restrict__ bcol,
                                                uint32_t nb, const uint64_t* __restrict__ ent,
                                                const int32_t* __restrict__ row, const double* __restrict__ val,
                                                int n2, const double* __restrict__ R1, int m,
                                                const double* __restrict__ w2, T* __restrict__ x2,
                                                double* __restrict__ wblk, double* __restrict__ wpart) {
  constexpr int NU = (kMaxM + 63) / 64;
  const int lane = threadIdx.x & 63;
  const uint32_t wave = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const uint32_t nwaves = gridDim.x * (NT / 64);
  double sq = 0.0;
  for (uint64_t b0 = static_cast<uint64_t>(wave) * 64; b0 < nb; b0 += static_cast<uint64_t>(nwaves) * 64) {
    const uint64_t bl = b0 + lane;
    int64_t e0 = 0, e1 = 0;
    double wl = 0.0, cl = 0.0;
    int gl = 0;
    if (bl < nb) {
      e0 = bstart[bl];
      e1 = bstart[bl + 1];
      wl = w2[bcol[bl]];
      wblk[bl] = wl;
      if (e1 - e0 == 1) {
        const uint64_t oe = ent[e0];
        gl = row[oe] / n2;
        cl = val[oe];
      }
    }
    const int nbl = static_cast<int>(min(static_cast<uint64_t>(64), nb - b0));
    for (int k = 0; k < nbl; ++k) {
      const int64_t f0 = __shfl(e0, k, 64), f1 = __shfl(e1, k, 64);
      const double wb = __shfl(wl, k, 64);
      T acc[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) acc[u] = T(0);
      if (f1 - f0 == 1) {
        const int g = __shfl(gl, k, 64);
        const double c = __shfl(cl, k, 64);
        const double* Rg = R1 + static_cast<size_t>(g) * m;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int a = lane + 64 * u;
          if (a < m) acc[u] = x2_term<T, P>(c, Rg[a], acc[u]);
        }
      } else {
        for (int64_t e = f0; e < f1; ++e) {
          const uint64_t oe = ent[e];
          const int rho = row[oe];
          const double c = val[oe];
          const double* Rg = R1 + static_cast<size_t>(rho / n2) * m;
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const int a = lane + 64 * u;
            if (a < m) acc[u] = x2_term<T, P>(c, Rg[a], acc[u]);
          }
        }
      }
      T* xb = x2 + (b0 + k) * m;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int a = lane + 64 * u;
        if (a < m) {
          xb[a] = acc[u];
          const double v = static_cast<double>(acc[u]);
          sq = fma(wb * v, v, sq);
        }
      }
    }
  }
  sq = wave_sum_f64(sq);
  if (lane == 0) wpart[wave] = sq;
}

// Sum of the per-wave partials in wave order (one workgroup).
__global__ __launch_bounds__(NT) void k_sum_ordered(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double lds[NT];
  double s = 0.0;
  // thread t sums a contiguous run, then the runs are added in order
  const int per = (n + NT - 1) / NT;
  for (int i = threadIdx.x * per; i < min(n, (threadIdx.x + 1) * per); ++i) s += part[i];
  lds[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < NT; ++i) t += lds[i];
    *out = t;
  }
}

// (column, block) of every block, for a stable sort by column that keeps slot order.
__global__ __launch_bounds__(NT) void k_col_keys(const int32_t* __restrict__ bcol, uint32_t nb,
                                                 uint64_t* __restrict__ key, uint64_t* __restrict__ val) {
  const uint32_t b = blockIdx.x * NT + threadIdx.x;
  if (b >= nb) return;
  key[b] = static_cast<uint64_t>(bcol[b]);
  val[b] = b;
}

// Blocks of every column in slot order, from the slot-major blocks sorted (stably) by
// column: pairs (p < q) of a column, keyed by (slot_p, slot_q).  The 64-bit total
// guards the 32-bit scan of the counts.
__global__ __launch_bounds__(NT) void k_pair_counts(const int64_t* __restrict__ cptr, int ncols,
                                                    uint32_t* __restrict__ cnt, unsigned long long* __restrict__ total) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= ncols) return;
  const int64_t mj = cptr[j + 1] - cptr[j];
  const unsigned long long c = static_cast<unsigned long long>(mj) * static_cast<unsigned long long>(mj - 1) / 2ull;
  cnt[j] = static_cast<uint32_t>(c);
  atomicAdd(total, c);
}

__global__ __launch_bounds__(NT) void k_pair_emit(const int64_t* __restrict__ cptr, int ncols,
                                                  const uint64_t* __restrict__ cblk, const uint32_t* __restrict__ ppos,
                                                  const int32_t* __restrict__ bslot, int n2,
                                                  uint64_t* __restrict__ pkey, uint64_t* __restrict__ pval) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= ncols) return;
  const int64_t c0 = cptr[j], c1 = cptr[j + 1];
  uint32_t o = ppos[j];
  for (int64_t p = c0; p < c1; ++p) {
    const uint64_t bp = cblk[p];
    const uint64_t sp = static_cast<uint64_t>(bslot[bp]);
    for (int64_t q = p + 1; q < c1; ++q) {
      const uint64_t bq = cblk[q];
      pkey[o] = sp * static_cast<uint64_t>(n2) + static_cast<uint64_t>(bslot[bq]);
      pval[o] = (bp << 32) | bq;
      ++o;
    }
  }
}

// One k-step of NTPW accumulator tiles, starting at tile (tr, tc) of a wave's run:
// all fragments are read first, then the MFMA chain runs (reading each fragment just
// one MFMA ahead measured 4% slower: the chain then waits on LDS latency).  Tiles past
// the wave's nt live ones repeat its last live tile (valid addresses; never written
// back).
template <int MT, int NTPW>
__device__ __forceinline__ void gram_kstep(const double* __restrict__ Ak, const double* __restrict__ Bk, dbl4* acc,
                                           int tr, int tc, int nt, bool diag) {
  // software pipeline of depth one: the next tile's fragments are read before this
  // tile's MFMA is issued
  double fa[NTPW], fb[NTPW];
#pragma unroll
  for (int u = 0; u < NTPW; ++u) {
    fa[u] = Ak[tr * 16];
    fb[u] = Bk[tc * 16];
    if (u + 1 < nt && ++tc == MT) {
      ++tr;
      tc = diag ? tr : 0;
    }
  }
#pragma unroll
  for (int u = 0; u < NTPW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[u], acc[u], 0, 0, 0);
}

// One work item of the Gram per workgroup: the m x m block (padded to W = 16 MT)
// sum_k A_k B_k^T with A_k = w x_{b_k} and B_k = x_{b'_k} over the item's pairs, on
// v_mfma_f64_16x16x4 (operand lanes: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k; accumulator register v of lane l holds row 4v + l/16, column l%16).
// KIND 1 (off-diagonal blocks) takes all MT x MT tiles, KIND 0 (diagonal blocks) the
// tiles on or above the diagonal, mirrored when written; an item's tiles are split
// into contiguous runs of TPW over the 8 waves, each run a compile-time count so
// that a k-step reads all its fragments ahead of an unbranched MFMA chain.  Pairs go
// through LDS 16 at a time (double-buffered), converted to FP64 (and A scaled by w)
// as they are staged by coalesced per-wave loads; the next stage's loads are in
// flight during this stage's MFMA.
template <typename T, int MT, int KIND>
__global__ __launch_bounds__(kGramThreads) void k_slice_gram(const GramItem* __restrict__ items,
                                                             const T* __restrict__ x2, int m,
                                                             const double* __restrict__ wblk,
                                                             const uint64_t* __restrict__ pairs,
                                                             double* __restrict__ gram, double* __restrict__ part) {
  constexpr int W = 16 * MT;
  // accumulator tiles per wave; every item of a launch is of kind KIND
  constexpr int TPW = (tiles_per_item(MT, KIND) + kGramWaves - 1) / kGramWaves;
  static_assert(TPW <= tiles_per_wave(KIND), "accumulator tiles per wave");
  extern __shared__ double lds[];
  double* SA = lds;                 // [2][kKC][W]
  double* SB = lds + 2 * kKC * W;   // [2][kKC][W]
  const GramItem it = items[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  // staging: wave wv stages pairs wv + kGramWaves h of each stage, lane a of each
  // vector (coalesced); side A is stored scaled by the pair's weight, side B as is
  // (a diagonal item pairs a block with itself)
  constexpr int PPW = kKC / kGramWaves;
  constexpr int NU = (W + 63) / 64;
  static_assert(PPW * kGramWaves == kKC, "whole pairs per wave");
  T xa[PPW][NU], xb[PPW][NU];
  double wa[PPW];
  auto load = [&](int s0) {
#pragma unroll
    for (int h = 0; h < PPW; ++h) {
      const int p = s0 + wv + kGramWaves * h;
      const bool live = p < it.nk;
      int64_t ba = 0, bb = 0;
      if (live) {
        if (KIND == 0) {
          ba = bb = it.start + p;
        } else {
          const uint64_t pr = pairs[it.start + p];
          ba = static_cast<int64_t>(pr >> 32);
          bb = static_cast<int64_t>(pr & 0xffffffffull);
        }
      }
      wa[h] = live ? wblk[ba] : 0.0;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int a = lane + 64 * u;
        const bool ok = live && a < m;
        xa[h][u] = ok ? x2[static_cast<size_t>(ba) * m + a] : T(0);
        if (KIND != 0) xb[h][u] = ok ? x2[static_cast<size_t>(bb) * m + a] : T(0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < PPW; ++h) {
      double* A = SA + (buf * kKC + wv + kGramWaves * h) * W;
      double* B = SB + (buf * kKC + wv + kGramWaves * h) * W;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int a = lane + 64 * u;
        if (a < W) {
          const double x = static_cast<double>(xa[h][u]);
          A[a] = wa[h] * x;
          B[a] = KIND == 0 ? x : static_cast<double>(xb[h][u]);
        }
      }
    }
  };
  dbl4 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
  // this wave's tiles: positions tile0 + wv TPW + u of the item's tile order (row-major
  // over all tiles, or over the upper tiles of a diagonal block)
  // this wave's tiles: positions tile0 + wv TPW + u of the item's tile order (row-major
  // over all tiles, or over the upper tiles of a diagonal block): its first tile
  // (tr0, tc0) and count nt; later tiles step along the row, then to the next row
  const int ntiles = tiles_of(MT, KIND);
  const int tfirst = it.tile0 + wv * TPW;
  const int nt = max(0, min(TPW, min(ntiles, it.tile0 + tiles_per_item(MT, KIND)) - tfirst));
  int tr0 = 0, tc0 = 0;
  if (KIND == 0) {
    int rem = nt > 0 ? tfirst : 0;
    while (rem >= MT - tr0) {
      rem -= MT - tr0;
      ++tr0;
    }
    tc0 = tr0 + rem;
  } else if (nt > 0) {
    tr0 = tfirst / MT;
    tc0 = tfirst - tr0 * MT;
  }
  const int nst = (it.nk + kKC - 1) / kKC;
  load(0);
  store(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) load((st + 1) * kKC);
    const double* A = SA + buf * kKC * W;
    const double* B = SB + buf * kKC * W;
    // k-steps rolled: only one step's fragments are live at a time
#pragma unroll 1
    for (int ks = 0; ks < kKC; ks += 4) {
      const double* Ak = A + (ks + lk) * W + li;
      const double* Bk = B + (ks + lk) * W + li;
      if (nt > 0) gram_kstep<MT, TPW>(Ak, Bk, acc, tr0, tc0, nt, KIND == 0);
    }
    if (st + 1 < nst) store(buf ^ 1);
    __syncthreads();
  }
  double* dst = (it.to_part ? part : gram) + it.dst;
  int tr = tr0, tc = tc0;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    if (u >= nt) continue;
    const bool mirror = KIND == 0 && tr != tc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = tr * 16 + 4 * v + lk, c = tc * 16 + li;
      if (r < m && c < m) {
        dst[static_cast<size_t>(r) * m + c] = acc[u][v];
        if (mirror) dst[static_cast<size_t>(c) * m + r] = acc[u][v];
      }
    }
    if (++tc == MT) {
      ++tr;
      tc = KIND == 0 ? tr : 0;
    }
  }
}

// Split blocks: out = sum of the block's partials, in item order.
struct ReduceItem {
  int64_t dst;
  int64_t first;  // first partial (index of an m x m partial block)
  int32_t count;
  int32_t pad;
};

__global__ __launch_bounds__(NT) void k_reduce_parts(const ReduceItem* __restrict__ red, int m,
                                                     const double* __restrict__ part, double* __restrict__ gram) {
  const ReduceItem r = red[blockIdx.y];
  const int64_t mm = static_cast<int64_t>(m) * m;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; e < mm;
       e += static_cast<int64_t>(gridDim.x) * NT) {
    double s = 0.0;
    for (int c = 0; c < r.count; ++c) s += part[(r.first + c) * mm + e];
    gram[r.dst + e] = s;
  }
}

__global__ __launch_bounds__(NT) void k_zero_blocks(const int64_t* __restrict__ dst, int m, double* __restrict__ gram) {
  const int64_t mm = static_cast<int64_t>(m) * m;
  const int64_t base = dst[blockIdx.y];
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; e < mm;
       e += static_cast<int64_t>(gridDim.x) * NT)
    gram[base + e] = 0.0;
}

int bits_of(uint64_t n) {  // bits to hold values 0..n-1
  int b = 0;
  while (b < 64 && (n - 1) >> b) ++b;
  return b;
}

template <class X>
void to_host(std::vector<X>& h, const X* dev, size_t n, hipStream_t s) {
  h.resize(n);
  Readback rb(s);
  if (n) rb.add(h.data(), dev, sizeof(X) * n);
  rb.sync();
}

struct StageEvents {
  hipEvent_t e[5] = {};
  StageEvents() {
    for (auto& x : e) TTS_HIP(hipEventCreate(&x));
  }
  ~StageEvents() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// Packed index of the upper block (i, i2), i <= i2, of an n2 x n2 block matrix.
int64_t packed_block(int64_t i, int64_t i2, int64_t n2) { return i * n2 - i * (i - 1) / 2 + (i2 - i); }

template <typename T, int P>
void fill_x2(Allocator* A, const SliceInput& in, SliceOut& o, const DBuf<int64_t>& bstart, const DBuf<uint64_t>& ent,
             const double* w2, DBuf<double>& wblk, hipStream_t s) {
  const uint32_t nb = static_cast<uint32_t>(o.nblocks);
  const int n2 = static_cast<int>(in.dims[1]);
  o.x2.reset(A, sizeof(T) * static_cast<size_t>(nb) * o.m);
  wblk.reset(A, nb);
  const unsigned grid = std::max(1u, std::min<unsigned>((nb + 255) / 256, 8192));
  DBuf<double> wpart(A, static_cast<size_t>(grid) * (NT / 64)), wsum(A, 1);
  {
    KTimer kt("slice_x2", s,
              12.0 * in.n_nnz[1] + 8.0 * static_cast<double>(o.m) * in.betas[1] +
                  static_cast<double>(sizeof(T)) * nb * o.m,
              2.0 * static_cast<double>(in.n_nnz[1]) * o.m);
    k_x2_fill<T, P><<<grid, NT, 0, s>>>(bstart.get(), o.blk_col.get(), nb, ent.get(), in.n_row[1], in.n_val[1], n2,
                                        o.r1.get(), o.m, w2, reinterpret_cast<T*>(o.x2.get()), wblk.get(),
                                        wpart.get());
    TTS_LAUNCH_CHECK();
  }
  k_sum_ordered<<<1, NT, 0, s>>>(wpart.get(), static_cast<int>(grid * (NT / 64)), wsum.get());
  TTS_LAUNCH_CHECK();
  {
    Readback rb(s);
    rb.add(&o.wnorm2, wsum.get(), sizeof(double));
    rb.sync();
  }
}

template <typename T>
void run_gram(Allocator* A, const SliceInput& in, SliceOut& o, const double* wblk, const uint64_t* pairs,
              const std::vector<int64_t>& slot_ptr, const std::vector<int64_t>& pair_ptr, hipStream_t s) {
  const int64_t n2 = in.dims[1], m = o.m;
  const int64_t mm = m * m;
  std::vector<GramItem> items;
  std::vector<ReduceItem> reds;
  std::vector<int64_t> zeros;
  int64_t nparts = 0;
  double flops = 0.0;
  const int MT = static_cast<int>((m + 15) / 16);
  auto add_block = [&](int kind, int64_t i, int64_t i2, int64_t start, int64_t count) {
    const int64_t dst = packed_block(i, i2, n2) * mm;
    if (count == 0) {
      zeros.push_back(dst);
      return;
    }
    flops += (kind == 0 ? static_cast<double>(m) * (m + 1) : 2.0 * m * m) * count;
    const int64_t nchunk = (count + kItemPairs - 1) / kItemPairs;
    const int nsplit = gram_split(MT, kind), tpi = tiles_per_item(MT, kind);
    if (nchunk == 1) {
      for (int sp = 0; sp < nsplit; ++sp)
        items.push_back(GramItem{kind, static_cast<int32_t>(count), 0, sp * tpi, start, dst});
      return;
    }
    reds.push_back(ReduceItem{dst, nparts, static_cast<int32_t>(nchunk), 0});
    for (int64_t c = 0; c < nchunk; ++c) {
      const int64_t lo = c * kItemPairs, hi = std::min(count, lo + kItemPairs);
      for (int sp = 0; sp < nsplit; ++sp)
        items.push_back(GramItem{kind, static_cast<int32_t>(hi - lo), 1, sp * tpi, start + lo, (nparts + c) * mm});
    }
    nparts += nchunk;
  };
  for (int64_t i = 0; i < n2; ++i) {
    add_block(0, i, i, slot_ptr[i], slot_ptr[i + 1] - slot_ptr[i]);
    for (int64_t i2 = i + 1; i2 < n2; ++i2) {
      const int64_t key = i * n2 + i2;
      add_block(1, i, i2, pair_ptr[key], pair_ptr[key + 1] - pair_ptr[key]);
    }
  }
  o.gram_flops = flops;
  // largest items first
  std::stable_sort(items.begin(), items.end(), [](const GramItem& a, const GramItem& b) { return a.nk > b.nk; });
  DBuf<GramItem> ditems(A, std::max<size_t>(items.size(), 1));
  DBuf<ReduceItem> dreds(A, std::max<size_t>(reds.size(), 1));
  DBuf<int64_t> dzeros(A, std::max<size_t>(zeros.size(), 1));
  DBuf<double> part(A, std::max<int64_t>(nparts, 1) * mm);
  if (!reds.empty())
    TTS_HIP(hipMemcpyAsync(dreds.get(), reds.data(), sizeof(ReduceItem) * reds.size(), hipMemcpyHostToDevice, s));
  if (!zeros.empty())
    TTS_HIP(hipMemcpyAsync(dzeros.get(), zeros.data(), sizeof(int64_t) * zeros.size(), hipMemcpyHostToDevice, s));
  const T* x2 = reinterpret_cast<const T*>(o.x2.get());
  // diagonal items first (they are the largest), then the off-diagonal ones; one
  // launch per kind so that each has its own accumulator count per wave
  const size_t ndiag = static_cast<size_t>(
      std::stable_partition(items.begin(), items.end(), [](const GramItem& x) { return x.kind == 0; }) -
      items.begin());
  // XCD-aware order: the items that split one block's tiles read the same pairs.
  // Workgroups are dispatched to the 8 XCDs round-robin by index, so within each
  // window of 8 blocks the parts of block b are placed at b, b + 8, b + 16, ...:
  // they run on one XCD at about the same time and the later ones find the pairs'
  // vectors in that XCD's L2 instead of reading them from HBM again.
  auto xcd_order = [&](size_t first, size_t cnt, int nsplit) {
    if (nsplit <= 1 || cnt % nsplit) return;
    for (size_t u = first; u < first + cnt; u += nsplit)
      for (int sp = 1; sp < nsplit; ++sp)
        if (items[u + sp].start != items[u].start || items[u + sp].dst != items[u].dst) return;
    std::vector<GramItem> out(items.begin() + first, items.begin() + first + cnt);
    const size_t nunit = cnt / nsplit;
    for (size_t w0 = 0; w0 < nunit; w0 += 8) {
      const size_t k = std::min<size_t>(8, nunit - w0);
      for (size_t b = 0; b < k; ++b)
        for (int sp = 0; sp < nsplit; ++sp)
          out[w0 * nsplit + sp * k + b] = items[first + (w0 + b) * nsplit + sp];
    }
    std::copy(out.begin(), out.end(), items.begin() + first);
  };
  xcd_order(0, ndiag, gram_split(MT, 0));
  xcd_order(ndiag, items.size() - ndiag, gram_split(MT, 1));
  if (!items.empty())
    TTS_HIP(hipMemcpyAsync(ditems.get(), items.data(), sizeof(GramItem) * items.size(), hipMemcpyHostToDevice, s));
  if (!items.empty()) {
    KTimer kt("slice_gram", s,
              static_cast<double>(sizeof(T)) * o.nblocks * m + 8.0 * static_cast<double>(n2) * (n2 + 1) / 2 * mm,
              flops);
    const size_t shm = sizeof(double) * 4 * kKC * 16 * static_cast<size_t>(MT);
    for (int kind = 0; kind < 2; ++kind) {
      const size_t first = kind == 0 ? 0 : ndiag, cnt = kind == 0 ? ndiag : items.size() - ndiag;
      if (cnt == 0) continue;
      const unsigned g = static_cast<unsigned>(cnt);
      const GramItem* di = ditems.get() + first;
#define TTS_GRAM_CASE(MTV)                                                                                      \
  case MTV:                                                                                                     \
    if (kind == 0)                                                                                              \
      k_slice_gram<T, MTV, 0><<<g, kGramThreads, shm, s>>>(di, x2, static_cast<int>(m), wblk, pairs, o.gram.get(), \
                                                           part.get());                                         \
    else                                                                                                        \
      k_slice_gram<T, MTV, 1><<<g, kGramThreads, shm, s>>>(di, x2, static_cast<int>(m), wblk, pairs, o.gram.get(), \
                                                           part.get());                                         \
    break;
      switch (MT) {
        TTS_GRAM_CASE(1)
        TTS_GRAM_CASE(2)
        TTS_GRAM_CASE(3)
        TTS_GRAM_CASE(4)
        TTS_GRAM_CASE(5)
        TTS_GRAM_CASE(6)
        TTS_GRAM_CASE(7)
        TTS_GRAM_CASE(8)
        TTS_GRAM_CASE(9)
        TTS_GRAM_CASE(10)
        TTS_GRAM_CASE(11)
        TTS_GRAM_CASE(12)
        TTS_GRAM_CASE(13)
        default:
          fail(TT_ERR_TOO_LARGE, "bond-1 rank above 208");
      }
#undef TTS_GRAM_CASE
      TTS_LAUNCH_CHECK();
    }
  }
  if (!reds.empty()) {
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((mm + NT - 1) / NT, 64));
    k_reduce_parts<<<dim3(gx, static_cast<unsigned>(reds.size())), NT, 0, s>>>(dreds.get(), static_cast<int>(m),
                                                                               part.get(), o.gram.get());
    TTS_LAUNCH_CHECK();
  }
  if (!zeros.empty()) {
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((mm + NT - 1) / NT, 64));
    k_zero_blocks<<<dim3(gx, static_cast<unsigned>(zeros.size())), NT, 0, s>>>(dzeros.get(), static_cast<int>(m),
                                                                                o.gram.get());
    TTS_LAUNCH_CHECK();
  }
  // the host item lists must outlive their copies
  TTS_HIP(hipStreamSynchronize(s));
}

}  // namespace

void gram_slice(Allocator& al, const SliceInput& in, SliceOut& o, hipStream_t s) {
  Allocator* A = &al;
  const int d = in.d;
  if (d < 3) fail(TT_ERR_ARG, "the bond-2 slice needs d >= 3");
  const int prec = in.precision;
  if (prec != TT_FP64 && prec != TT_FP32 && prec != TT_BF16_FP32ACC) fail(TT_ERR_ARG, "unknown precision");
  const int n1 = static_cast<int>(in.dims[0]), n2 = static_cast<int>(in.dims[1]);
  const int64_t b1 = in.betas[1], b2 = in.betas[2];
  if (n1 > kMaxM) fail(TT_ERR_TOO_LARGE, "the bond-2 slice supports n_1 <= 208");
  if (b1 < n1) fail(TT_ERR_ARG, "the bond-2 slice needs a wide bond-1 unfolding (beta_1 >= n_1)");
  if (b1 > INT32_MAX || b2 > INT32_MAX) fail(TT_ERR_TOO_LARGE, "rank above 2^31");
  if (static_cast<int64_t>(n2) * n2 > (int64_t(1) << 32)) fail(TT_ERR_TOO_LARGE, "n_2^2 above 2^32");
  StageEvents ev;
  TTS_HIP(hipEventRecord(ev.e[0], s));

  // ---- bond 1: X_1 = Q_1 R_1 in the SVD gauge ----
  DBuf<double> X1(A, static_cast<size_t>(n1) * b1);
  TTS_HIP(hipMemsetAsync(X1.get(), 0, sizeof(double) * n1 * b1, s));
  DBuf<int32_t> rowflag(A, n1 + 1);
  TTS_HIP(hipMemsetAsync(rowflag.get(), 0, sizeof(int32_t) * (n1 + 1), s));
  k_slice_x1<<<grid_for(b1, NT), NT, 0, s>>>(in.n_colptr[0], static_cast<int>(b1), in.n_row[0], in.n_val[0], n1,
                                              X1.get(), rowflag.get(), rowflag.get() + n1);
  TTS_LAUNCH_CHECK();
  DBuf<double> G(A, static_cast<size_t>(b1) * n1), Qg(A, static_cast<size_t>(b1) * n1), Rg(A, static_cast<size_t>(n1) * n1);
  transpose(X1.get(), n1, static_cast<int>(b1), n1, G.get(), static_cast<int>(b1), s);
  DBuf<int32_t> ok(A, 4);
  cholqr2_async(A, G.get(), static_cast<int>(b1), n1, Qg.get(), Rg.get(), ok.get(), s);
  int32_t hok[4];
  int32_t nz = 0;
  {
    Readback rb(s);
    rb.add(hok, ok.get(), sizeof(hok));
    rb.add(&nz, rowflag.get() + n1, sizeof(int32_t));
    rb.sync();
  }
  if (!(hok[0] && hok[1] && hok[2] && hok[3]))
    qr_explicit(A, G.get(), static_cast<int>(b1), n1, static_cast<int>(b1), Qg.get(), static_cast<int>(b1), Rg.get(),
                n1, s);
  const int m = static_cast<int>(std::min<int64_t>(nz, b1));
  if (m < 1) fail(TT_ERR_EMPTY, "bond-1 unfolding is zero");
  o.m = m;
  DBuf<double> V(A, static_cast<size_t>(n1) * n1), sig(A, n1);
  DBuf<int32_t> jinfo(A, 4);
  jacobi_svd(Rg.get(), n1, n1, n1, V.get(), n1, sig.get(), jinfo.get(), s);
  alignas(8) int32_t hinfo[4] = {0, 0, 0, 0};
  std::vector<double> hs(n1);
  {
    Readback rb(s);
    rb.add(hinfo, jinfo.get(), sizeof(hinfo));
    rb.add(hs.data(), sig.get(), sizeof(double) * n1);
    rb.sync();
  }
  svd_check(hinfo, hs.data(), n1, n1);
  std::vector<int32_t> perm(n1);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) { return hs[x] > hs[y]; });
  o.sigma1.resize(m);
  for (int j = 0; j < m; ++j) o.sigma1[j] = hs[perm[j]];
  DBuf<int32_t> dperm(A, n1);
  TTS_HIP(hipMemcpyAsync(dperm.get(), perm.data(), sizeof(int32_t) * n1, hipMemcpyHostToDevice, s));
  o.q1.reset(A, static_cast<size_t>(n1) * m);
  permute_cols(V.get(), n1, n1, dperm.get(), nullptr, m, o.q1.get(), n1, s);
  sign_fix(o.q1.get(), n1, m, n1, nullptr, 0, 0, s);
  o.r1.reset(A, static_cast<size_t>(m) * b1);
  gemm(A, true, false, m, static_cast<int>(b1), n1, 1.0, o.q1.get(), n1, X1.get(), n1, 0.0, o.r1.get(), m, s);
  TTS_HIP(hipStreamSynchronize(s));  // the permutation's host copy
  X1.release();
  G.release();
  Qg.release();
  TTS_HIP(hipEventRecord(ev.e[1], s));

  // ---- right-part weights w_2 ----
  std::vector<DBuf<double>> w(d);
  w[d - 1].reset(A, in.betas[d - 1]);
  row_sumsq(in.last_core, static_cast<int>(in.betas[d - 1]), static_cast<int>(in.dims[d - 1]), w[d - 1].get(), s);
  for (int k = d - 2; k >= 2; --k) {
    w[k].reset(A, in.betas[k]);
    right_weights(A, in.n_colptr[k], in.n_row[k], in.n_val[k], static_cast<int>(in.betas[k + 1]), in.n_nnz[k],
                  static_cast<int>(in.dims[k]), static_cast<int>(in.betas[k]), w[k + 1].get(), w[k].get(), s);
  }
  const double* w2 = w[2].get();

  // ---- X_2 blocks, slot-major ----
  const uint32_t nnz2 = in.n_nnz[1];
  const int cbits = std::max(1, bits_of(static_cast<uint64_t>(b2)));
  const int kbits = cbits + std::max(1, bits_of(static_cast<uint64_t>(n2)));
  if (kbits > 64) fail(TT_ERR_TOO_LARGE, "slot-column key above 64 bits");
  DBuf<uint64_t> key(A, nnz2), ent(A, nnz2);
  {
    DBuf<uint64_t> kt(A, nnz2), vt(A, nnz2);
    k_x2_keys<<<grid_for(b2, NT), NT, 0, s>>>(in.n_colptr[1], static_cast<int>(b2), in.n_row[1], n2, cbits,
                                              key.get(), ent.get());
    TTS_LAUNCH_CHECK();
    if (radix_sort_pairs_pp(A, key.get(), ent.get(), kt.get(), vt.get(), nnz2, kbits, s)) {
      key.swap(kt);
      ent.swap(vt);
    }
  }
  DBuf<uint32_t> flag(A, nnz2), pos(A, nnz2), cnt(A, 1);
  k_run_flags<<<grid_for(nnz2, NT), NT, 0, s>>>(key.get(), nnz2, flag.get());
  TTS_LAUNCH_CHECK();
  exclusive_scan_u32(A, flag.get(), pos.get(), nnz2, cnt.get(), s);
  uint32_t nb = 0;
  {
    Readback rb(s);
    rb.add(&nb, cnt.get(), sizeof(uint32_t));
    rb.sync();
  }
  o.nblocks = nb;
  DBuf<int64_t> bstart(A, static_cast<size_t>(nb) + 1);
  DBuf<int32_t> bslot(A, nb);
  o.blk_col.reset(A, nb);
  k_block_info<<<grid_for(nnz2, NT), NT, 0, s>>>(key.get(), flag.get(), pos.get(), nnz2, cbits, nb, bstart.get(),
                                                 bslot.get(), o.blk_col.get());
  TTS_LAUNCH_CHECK();
  o.slot_ptr.reset(A, static_cast<size_t>(n2) + 1);
  k_lower_bound_i32<<<grid_for(n2 + 1, NT), NT, 0, s>>>(bslot.get(), nb, n2 + 1, o.slot_ptr.get());
  TTS_LAUNCH_CHECK();
  key.release();
  flag.release();
  pos.release();
  DBuf<double> wblk;
  if (prec == TT_FP64) {
    o.x2_dtype = TT_DTYPE_F64;
    fill_x2<double, TT_FP64>(A, in, o, bstart, ent, w2, wblk, s);
  } else {
    o.x2_dtype = TT_DTYPE_F32;
    if (prec == TT_FP32)
      fill_x2<float, TT_FP32>(A, in, o, bstart, ent, w2, wblk, s);
    else
      fill_x2<float, TT_BF16_FP32ACC>(A, in, o, bstart, ent, w2, wblk, s);
  }
  ent.release();
  bstart.release();
  TTS_HIP(hipEventRecord(ev.e[2], s));

  // ---- pair lists of the off-diagonal blocks ----
  DBuf<uint64_t> ck(A, nb), cv(A, nb);
  {
    DBuf<uint64_t> kt(A, nb), vt(A, nb);
    k_col_keys<<<grid_for(nb, NT), NT, 0, s>>>(o.blk_col.get(), nb, ck.get(), cv.get());
    TTS_LAUNCH_CHECK();
    if (radix_sort_pairs_pp(A, ck.get(), cv.get(), kt.get(), vt.get(), nb, cbits, s)) {
      ck.swap(kt);
      cv.swap(vt);
    }
  }
  DBuf<int64_t> cptr(A, static_cast<size_t>(b2) + 1);
  k_lower_bound_u64<<<grid_for(b2 + 1, NT), NT, 0, s>>>(ck.get(), nb, b2 + 1, cptr.get());
  TTS_LAUNCH_CHECK();
  ck.release();
  DBuf<uint32_t> pcnt(A, b2), ppos(A, b2), ptot(A, 1);
  DBuf<unsigned long long> ptot64(A, 1);
  TTS_HIP(hipMemsetAsync(ptot64.get(), 0, sizeof(unsigned long long), s));
  k_pair_counts<<<grid_for(b2, NT), NT, 0, s>>>(cptr.get(), static_cast<int>(b2), pcnt.get(), ptot64.get());
  TTS_LAUNCH_CHECK();
  unsigned long long np64 = 0;
  {
    Readback rb(s);
    rb.add(&np64, ptot64.get(), sizeof(np64));
    rb.sync();
  }
  if (np64 >= (1ull << 31)) fail(TT_ERR_TOO_LARGE, "more than 2^31 slot pairs in the columns of N_2");
  exclusive_scan_u32(A, pcnt.get(), ppos.get(), static_cast<uint32_t>(b2), ptot.get(), s);
  const uint32_t np = static_cast<uint32_t>(np64);
  o.npairs = np;
  DBuf<uint64_t> pk(A, std::max<uint32_t>(np, 1)), pv(A, std::max<uint32_t>(np, 1));
  k_pair_emit<<<grid_for(b2, NT), NT, 0, s>>>(cptr.get(), static_cast<int>(b2), cv.get(), ppos.get(), bslot.get(), n2,
                                              pk.get(), pv.get());
  TTS_LAUNCH_CHECK();
  const int pbits = std::max(1, bits_of(static_cast<uint64_t>(n2) * n2));
  if (np > 0) {
    DBuf<uint64_t> kt(A, np), vt(A, np);
    if (radix_sort_pairs_pp(A, pk.get(), pv.get(), kt.get(), vt.get(), np, pbits, s)) {
      pk.swap(kt);
      pv.swap(vt);
    }
  }
  const int64_t nkeys = static_cast<int64_t>(n2) * n2 + 1;
  DBuf<int64_t> pptr(A, nkeys);
  k_lower_bound_u64<<<grid_for(nkeys, NT), NT, 0, s>>>(pk.get(), np, nkeys, pptr.get());
  TTS_LAUNCH_CHECK();
  std::vector<int64_t> hslot, hpair;
  to_host(hslot, o.slot_ptr.get(), static_cast<size_t>(n2) + 1, s);
  to_host(hpair, pptr.get(), static_cast<size_t>(nkeys), s);
  cv.release();
  cptr.release();
  pk.release();
  TTS_HIP(hipEventRecord(ev.e[3], s));

  // ---- weighted Gram, packed upper blocks ----
  const size_t nblk = static_cast<size_t>(n2) * (n2 + 1) / 2;
  o.gram.reset(A, nblk * static_cast<size_t>(m) * m);
  if (prec == TT_FP64)
    run_gram<double>(A, in, o, wblk.get(), pv.get(), hslot, hpair, s);
  else
    run_gram<float>(A, in, o, wblk.get(), pv.get(), hslot, hpair, s);
  TTS_HIP(hipEventRecord(ev.e[4], s));
  TTS_HIP(hipEventSynchronize(ev.e[4]));
  for (int i = 0; i < 4; ++i) {
    float ms = 0.f;
    TTS_HIP(hipEventElapsedTime(&ms, ev.e[i], ev.e[i + 1]));
    o.ms[i] = ms;
  }
  float tot = 0.f;
  TTS_HIP(hipEventElapsedTime(&tot, ev.e[0], ev.e[4]));
  o.ms[4] = tot;
  logf("Gram slice: m %d, %lld blocks, %lld pairs; bond-1 QR %.3f ms, X_2 %.3f ms, pairs %.3f ms, Gram %.3f ms", m,
       static_cast<long long>(o.nblocks), static_cast<long long>(o.npairs), o.ms[0], o.ms[1], o.ms[2], o.ms[3]);
}

}  // namespace tts
