// Kernels of the sparse stage: per-mode sparse unfoldings and their parallel-vector
// rounding (Deparallelisation of every level's unfolding, Algorithm 3 applied in the
// TT-SVD sweep of Algorithm 1 in place of the truncated SVD).
//
// Data flow of one level k (entries of M_k sorted so that every column -- a suffix
// (i_{k+1},...,i_d) -- is one contiguous segment):
//   col_flags/col_starts : segment boundaries -> column start offsets (columns_small:
//                          the same in one workgroup for small levels)
//   canon                : one thread (canon_wave: one wave) per column: order its
//                          entries by row rho,
//                          s = value at the smallest row, c_j = v_j / s (IEEE
//                          binary64 division, optionally rounded to fewer fraction
//                          bits: the tolerant test), 64-bit hash of (m, rho_j, bits(c_j))
//   group                : open-addressing table keyed by the hash; a column that
//                          finds an occupied slot compares its full canonical key
//                          with the slot's representative column; the smallest
//                          row-major suffix key of each group is its leader
//   leaders              : leaders sorted by row-major suffix key -> group ids
//                          (first occurrence in row-major column order), N_k's
//                          column places
//   emit                 : N_k (CSC) and the next level's entries
//                          (rho' = g * n_{k+1} + i_{k+1}, value s)
#include "sparse.hpp"
#include "prim.hpp"

#include <algorithm>
#include <cmath>

namespace tts {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ uint64_t fmask(uint32_t b) { return (b >= 64) ? ~0ull : ((1ull << b) - 1ull); }

__global__ __launch_bounds__(NT) void k_ingest(const int32_t* __restrict__ idx, const double* __restrict__ val,
                                               uint32_t nnz, ModeInfo mi, uint64_t* __restrict__ keys,
                                               uint64_t* __restrict__ vbits, DevStatus* st, int vec4) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  bool zero = false;
  if (e < nnz) {
    const int32_t* c = idx + static_cast<size_t>(e) * mi.d;
    const double v = val[e];
    uint64_t key = 0;
    bool bad = false;
    // the coordinates eight at a time, each group's loads issued together (as two
    // 16-byte loads when every row is 16-byte aligned)
    for (int j0 = 0; j0 < mi.d; j0 += 8) {
      int32_t x[8];
      if (vec4) {
        const int4 a = *reinterpret_cast<const int4*>(c + j0);
        const int4 b = (j0 + 4 < mi.d) ? *reinterpret_cast<const int4*>(c + j0 + 4) : make_int4(0, 0, 0, 0);
        x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w;
        x[4] = b.x, x[5] = b.y, x[6] = b.z, x[7] = b.w;
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = c[(j0 + u < mi.d) ? j0 + u : 0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = j0 + u;
        if (j < mi.d) {
          bad |= (x[u] < 0) || (static_cast<uint32_t>(x[u]) >= mi.n[j]);
          key |= static_cast<uint64_t>(static_cast<uint32_t>(x[u])) << mi.off[j];
        }
      }
    }
    if (bad) atomicOr(&st->err, kErrIndex);
    if (!isfinite(v)) atomicOr(&st->err, kErrNonfinite);
    zero = (v == 0.0);
    keys[e] = zero ? ~0ull : key;
    vbits[e] = __double_as_longlong(v);
  }
  // explicit zeros are rare: one atomic per wave that has any (a count of kept
  // entries would need one per workgroup, all on one address)
  const uint64_t zm = __ballot(zero);
  if (zm && (threadIdx.x & 63) == 0) atomicAdd(&st->dropped, static_cast<uint32_t>(__popcll(zm)));
}

__global__ __launch_bounds__(NT) void k_col_flags(const uint64_t* __restrict__ ekey, uint32_t nE, int sh,
                                                  int level1, int long_bit, const double* __restrict__ ev,
                                                  uint32_t* __restrict__ flag, double* __restrict__ norm_part,
                                                  DevStatus* st) {
  __shared__ double red[NT / 64];
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  double sq = 0.0;
  if (e < nE) {
    const uint64_t k = ekey[e];
    const uint64_t col = k >> sh;
    const bool start = (e == 0) || ((ekey[e - 1] >> sh) != col);
    flag[e] = start ? 1u : 0u;
    if (level1) {
      if (e > 0 && ekey[e - 1] == k) atomicOr(&st->err, kErrDuplicate);
      const double v = ev[e];
      sq = v * v;
    }
    // columns are contiguous runs of the sorted entries: the one starting at e is
    // longer than kMaxLocal exactly when entry e + kMaxLocal still belongs to it
    if (long_bit >= 0 && start && nE - e > static_cast<uint32_t>(kMaxLocal) &&
        (ekey[e + kMaxLocal] >> sh) == col)
      atomicOr(&st->longmask, 1ull << long_bit);
  }
  if (level1) {
    sq = wave_sum_f64(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w];
      norm_part[blockIdx.x] = s;
    }
  }
}

// Sum of the per-workgroup partials in a fixed order: 1024 threads, each with four
// independent running sums over a strided quarter of its share (loads issued
// together), then a wave sum and the 16 wave sums in order.
constexpr int NF = 1024;
__global__ __launch_bounds__(NF) void k_norm_final(const double* __restrict__ part, uint32_t np, DevStatus* st) {
  __shared__ double red[NF / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  uint32_t i = threadIdx.x;
  for (; i + 3 * NF < np; i += 4 * NF) {
    const double a = part[i], b = part[i + NF], c = part[i + 2 * NF], e = part[i + 3 * NF];
    s0 += a;
    s1 += b;
    s2 += c;
    s3 += e;
  }
  for (; i < np; i += NF) s0 += part[i];
  double s = wave_sum_f64((s0 + s1) + (s2 + s3));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NF / 64; ++w) t += red[w];
    st->norm2 = t;
  }
}

__global__ __launch_bounds__(NT) void k_col_starts(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                                   uint32_t nE, uint32_t* __restrict__ col_start,
                                                   const uint32_t* __restrict__ d_ncols) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e < nE && flag[e]) col_start[pos[e]] = e;
  if (e == 0) col_start[*d_ncols] = nE;
}

// a3 for a level k >= 2 of at most kColsSmallMax entries in one workgroup: thread t
// takes a contiguous run of at most CS_PER entries (held in registers), counts the
// column starts in it (an entry whose suffix differs from its predecessor's), and
// after a workgroup scan writes each start's column place, and flags a column
// longer than kMaxLocal entries.  Same col_start, *d_ncols and long-column bit as
// k_col_flags, the scan and k_col_starts.
constexpr int CS_NT = 1024;
constexpr int CS_PER = static_cast<int>(kColsSmallMax / CS_NT);
__device__ __forceinline__ void columns_small_block(const uint64_t* __restrict__ ekey, uint32_t nE, int sh,
                                                    int long_bit, uint32_t* __restrict__ col_start,
                                                    uint32_t* __restrict__ d_ncols, DevStatus* st) {
  __shared__ uint32_t red[CS_NT / 64];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nE + CS_NT - 1) / CS_NT;
  const uint32_t b = min(nE, t * per), e1 = min(nE, b + per);
  uint64_t col[CS_PER];
#pragma unroll
  for (int u = 0; u < CS_PER; ++u) {
    const uint32_t e = b + u;
    col[u] = e < e1 ? (ekey[e] >> sh) : 0ull;
  }
  const uint64_t before = (b > 0 && b < e1) ? (ekey[b - 1] >> sh) : 0ull;
  uint32_t starts = 0;  // bit u: entry b + u starts a column
#pragma unroll
  for (int u = 0; u < CS_PER; ++u) {
    const uint32_t e = b + u;
    const bool st_u = e < e1 && (e == 0 || (u == 0 ? before : col[u > 0 ? u - 1 : 0]) != col[u]);
    starts |= st_u ? (1u << u) : 0u;
  }
  uint32_t tot;
  uint32_t pos = block_excl_scan_u32<CS_NT>(static_cast<uint32_t>(__popc(starts)), red, &tot);
#pragma unroll
  for (int u = 0; u < CS_PER; ++u)
    if ((starts >> u) & 1u) col_start[pos++] = b + u;
  if (t == 0) {
    col_start[tot] = nE;
    *d_ncols = tot;
  }
  if (long_bit < 0) return;
  // a column is longer than kMaxLocal exactly when the entry kMaxLocal past its start
  // still belongs to it (columns are contiguous runs of the sorted entries)
  bool lng = false;
#pragma unroll
  for (int u = 0; u < CS_PER; ++u) {
    const uint32_t e = b + u;
    if (((starts >> u) & 1u) && nE - e > static_cast<uint32_t>(kMaxLocal))
      lng = lng || (ekey[e + kMaxLocal] >> sh) == col[u];
  }
  if (lng) atomicOr(&st->longmask, 1ull << long_bit);
}
__global__ __launch_bounds__(CS_NT) void k_columns_small(const uint64_t* __restrict__ ekey, uint32_t nE, int sh,
                                                         int long_bit, uint32_t* __restrict__ col_start,
                                                         uint32_t* __restrict__ d_ncols, DevStatus* st) {
  columns_small_block(ekey, nE, sh, long_bit, col_start, d_ncols, st);
}

// a3 without flag arrays (speculative pass): two launches over tiles of ST_TILE
// entries, thread t of a tile owning ST_IPT consecutive entries.  The first counts
// each tile's column starts (an entry whose suffix differs from its predecessor's;
// on level 1 also the duplicate check and a fixed-order sum of squares per tile, on
// later levels the long-column probe); the second recomputes the starts, adds the
// counts of the tiles before its own (at most kStartsMaxTiles of them, each tile
// summing them itself) and writes every start's column place.  Same col_start,
// *d_ncols, duplicate and long-column flags as k_col_flags, the scan and k_col_starts.
constexpr int ST_IPT = 16;
constexpr uint32_t ST_TILE = NT * ST_IPT;
static_assert(kStartsMaxTiles % NT == 0, "whole thread rounds of tile counts");
// the suffixes of entries b .. b + ST_IPT - 1 (clamped loads) and of entry b - 1
__device__ __forceinline__ void tile_suffixes(const uint64_t* __restrict__ ekey, uint32_t nE, int sh, uint32_t b,
                                              uint64_t key[ST_IPT], uint64_t* before) {
#pragma unroll
  for (int u = 0; u < ST_IPT; ++u) key[u] = ekey[min(b + u, nE - 1)];
  *before = b > 0 ? ekey[b - 1] : 0ull;
}
__device__ __forceinline__ uint32_t tile_starts(const uint64_t key[ST_IPT], uint64_t before, uint32_t b, uint32_t nE,
                                                int sh) {
  uint32_t m = 0;
#pragma unroll
  for (int u = 0; u < ST_IPT; ++u) {
    const uint64_t prev = u == 0 ? before : key[u > 0 ? u - 1 : 0];
    const bool st = b + u < nE && (b + u == 0 || (prev >> sh) != (key[u] >> sh));
    m |= st ? (1u << u) : 0u;
  }
  return m;
}
__global__ __launch_bounds__(NT) void k_starts_count(const uint64_t* __restrict__ ekey, uint32_t nE, int sh,
                                                     int level1, int long_bit, const double* __restrict__ ev,
                                                     uint32_t* __restrict__ part, double* __restrict__ norm_part,
                                                     DevStatus* st) {
  __shared__ uint32_t red[NT / 64];
  __shared__ double dred[NT / 64];
  const uint32_t b = blockIdx.x * ST_TILE + threadIdx.x * ST_IPT;
  uint64_t key[ST_IPT], before;
  uint32_t m = 0;
  double sq = 0.0;
  if (b < nE) {
    tile_suffixes(ekey, nE, sh, b, key, &before);
    m = tile_starts(key, before, b, nE, sh);
    if (level1) {
      bool dup = false;
#pragma unroll
      for (int u = 0; u < ST_IPT; ++u) {
        const uint64_t prev = u == 0 ? before : key[u > 0 ? u - 1 : 0];
        dup = dup || (b + u < nE && b + u > 0 && prev == key[u]);
        const double v = (b + u < nE) ? ev[b + u] : 0.0;
        sq += v * v;
      }
      if (dup) atomicOr(&st->err, kErrDuplicate);
    }
    if (long_bit >= 0) {
      // the column starting at e is longer than kMaxLocal exactly when entry
      // e + kMaxLocal still belongs to it
      bool lng = false;
#pragma unroll
      for (int u = 0; u < ST_IPT; ++u)
        if (((m >> u) & 1u) && nE - (b + u) > static_cast<uint32_t>(kMaxLocal))
          lng = lng || (ekey[b + u + kMaxLocal] >> sh) == (key[u] >> sh);
      if (lng) atomicOr(&st->longmask, 1ull << long_bit);
    }
  }
  uint32_t tot;
  block_excl_scan_u32<NT>(static_cast<uint32_t>(__popc(m)), red, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  if (level1) {
    sq = wave_sum_f64(sq);
    if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += dred[w];
      norm_part[blockIdx.x] = s;
    }
  }
}
__global__ __launch_bounds__(NT) void k_starts_place(const uint64_t* __restrict__ ekey, uint32_t nE, int sh,
                                                     const uint32_t* __restrict__ part, uint32_t* __restrict__ col_start,
                                                     uint32_t* __restrict__ d_ncols) {
  __shared__ uint32_t red[NT / 64];
  const uint32_t tile = blockIdx.x;
  constexpr int R = static_cast<int>(kStartsMaxTiles / NT);
  uint32_t q = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t j = threadIdx.x + r * NT;
    q += j < tile ? part[j] : 0u;
  }
  uint32_t prefix;
  block_excl_scan_u32<NT>(q, red, &prefix);
  const uint32_t b = tile * ST_TILE + threadIdx.x * ST_IPT;
  uint32_t m = 0;
  if (b < nE) {
    uint64_t key[ST_IPT], before;
    tile_suffixes(ekey, nE, sh, b, key, &before);
    m = tile_starts(key, before, b, nE, sh);
  }
  uint32_t tot;
  uint32_t run = prefix + block_excl_scan_u32<NT>(static_cast<uint32_t>(__popc(m)), red, &tot);
#pragma unroll
  for (int u = 0; u < ST_IPT; ++u)
    if ((m >> u) & 1u) col_start[run++] = b + u;
  if (threadIdx.x == 0 && tile == gridDim.x - 1) {
    col_start[prefix + tot] = nE;
    *d_ncols = prefix + tot;
  }
}

// Column counts of every level from the globally sorted kept keys.  A level-k column
// (k = 1 .. d-1) is a distinct suffix key >> off[k] (modes k .. d-1), so its count is
// the number of positions where that suffix differs from the previous key's (the first
// position counts for every level).  Row y of the grid takes levels 1 + LC_PER y ..;
// per-workgroup sums go to counts[k] with one atomic each.  Also flags a duplicate
// (equal neighbouring keys).
constexpr int LC_PER = 8;
constexpr int LC_U = 8;  // runs of 64 keys per wave and loop trip
__device__ __forceinline__ uint64_t suffix_of(uint64_t key, uint32_t off) { return off >= 64 ? 0ull : key >> off; }
__global__ __launch_bounds__(NT) void k_level_counts(const uint64_t* __restrict__ keys, uint32_t n, ModeInfo mi,
                                                     uint32_t* __restrict__ counts, DevStatus* st) {
  __shared__ uint32_t red[NT / 64][LC_PER];
  const int k0 = 1 + LC_PER * static_cast<int>(blockIdx.y);
  uint32_t cnt[LC_PER];
#pragma unroll
  for (int j = 0; j < LC_PER; ++j) cnt[j] = 0u;
  bool dup = false;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // a wave takes 64 consecutive keys at a time (uniform loop), LC_U such runs with
  // all their loads issued together: each lane's predecessor comes from the lane
  // below, the first lane's from memory
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * NT;
  for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * NT + w * 64; base < n; base += LC_U * stride) {
    uint64_t kk[LC_U], pk[LC_U];
#pragma unroll
    for (int u = 0; u < LC_U; ++u) {
      const uint64_t e = base + u * stride + lane;
      kk[u] = e < n ? keys[e] : 0ull;
      pk[u] = (lane == 0 && e > 0 && e < n) ? keys[e - 1] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < LC_U; ++u) {
      const uint64_t e = base + u * stride + lane;
      const uint64_t key = kk[u];
      uint64_t prev = __shfl_up(key, 1, 64);
      if (lane == 0) prev = (e > 0) ? pk[u] : ~key;  // ~key differs from key in every bit
      if (e >= n) continue;
      dup = dup || (e > 0 && prev == key);
#pragma unroll
      for (int j = 0; j < LC_PER; ++j) {
        const int k = k0 + j;
        if (k < mi.d) cnt[j] += (suffix_of(key, mi.off[k]) != suffix_of(prev, mi.off[k])) ? 1u : 0u;
      }
    }
  }
  if (dup && blockIdx.y == 0) atomicOr(&st->err, kErrDuplicate);
#pragma unroll
  for (int j = 0; j < LC_PER; ++j) {
    uint32_t v = cnt[j];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < LC_PER) {
    const int k = k0 + static_cast<int>(threadIdx.x);
    if (k < mi.d) {
      uint32_t t = 0;
      for (int q = 0; q < NT / 64; ++q) t += red[q][threadIdx.x];
      // kLevelCountCopies copies of each count, so that the workgroups' adds do not
      // all queue on one address
      atomicAdd(&counts[static_cast<size_t>(k) * kLevelCountCopies + blockIdx.x % kLevelCountCopies], t);
    }
  }
}

__global__ __launch_bounds__(NT) void k_make_composite(const uint32_t* __restrict__ flag,
                                                       const uint32_t* __restrict__ pos,
                                                       const uint32_t* __restrict__ erho, uint32_t nE, int rbits,
                                                       uint64_t* __restrict__ ckey, uint64_t* __restrict__ cval) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e >= nE) return;
  const uint64_t colid = static_cast<uint64_t>(pos[e] + flag[e] - 1u);
  ckey[e] = (colid << rbits) | static_cast<uint64_t>(erho[e]);
  cval[e] = e;
}

__global__ __launch_bounds__(NT) void k_permute(const uint64_t* __restrict__ perm, uint32_t nE,
                                                const uint64_t* __restrict__ ekey_in,
                                                const uint32_t* __restrict__ erho_in,
                                                const double* __restrict__ ev_in, uint64_t* __restrict__ ekey_out,
                                                uint32_t* __restrict__ erho_out, double* __restrict__ ev_out) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e >= nE) return;
  const uint32_t src = static_cast<uint32_t>(perm[e]);
  ekey_out[e] = ekey_in[src];
  erho_out[e] = erho_in[src];
  ev_out[e] = ev_in[src];
}

// Hash of a canonical column: a function of its length and of every (position,
// row, canonical value), summed over the entries (mod 2^64) so that it can be formed
// in any order, also in parallel.  Only a filter: equal hashes are verified entry by
// entry before two columns are grouped.
__device__ __forceinline__ uint64_t col_hash_term(uint32_t j, uint32_t rho, double cv) {
  return mix64(mix64((static_cast<uint64_t>(j) << 32 | rho) ^ 0x9e3779b97f4a7c15ull) ^
               static_cast<uint64_t>(__double_as_longlong(cv)));
}
// Canonical value v / s, rounded to 52 - drop fraction bits when drop > 0 (round half
// to even on the magnitude's bit pattern; a carry may move into the exponent, and a
// rounding that would reach the infinity/NaN exponent truncates instead).  Columns
// parallel up to a perturbation well below that precision then share one key.
__device__ __forceinline__ double canon_value(double v, double s, int drop) {
  const double x = v / s;
  if (drop == 0) return x;
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
  const uint64_t sign = u & (1ull << 63), mag = u ^ sign;
  const uint64_t kept = mag >> drop, rest = mag & ((1ull << drop) - 1ull), half = 1ull << (drop - 1);
  const uint64_t up = kept + ((rest > half || (rest == half && (kept & 1ull))) ? 1ull : 0ull);
  uint64_t r = up << drop;
  if ((r >> 52) >= 0x7FFull) r = kept << drop;
  return __longlong_as_double(static_cast<long long>(r | sign));
}
__device__ __forceinline__ uint64_t col_hash_final(uint32_t m, uint64_t sum) {
  return mix64(sum ^ mix64(static_cast<uint64_t>(m) * 0x9e3779b97f4a7c15ull));
}

// Suffix fields of column c: its packed suffix and its row-major key.
__device__ __forceinline__ void col_keys(const CanonArgs& a, const ModeInfo& mi, uint32_t c, uint32_t st) {
  const uint64_t suf = a.ekey[st] >> a.sh;
  a.colsuf[c] = suf;
  uint64_t rm = 0;
  const uint32_t base = mi.off[a.kidx];
  for (int j = a.kidx; j < mi.d; ++j) {
    const uint64_t f = (suf >> (mi.off[j] - base)) & fmask(mi.bits[j]);
    rm = (mi.bits[j] ? (rm << mi.bits[j]) : rm) | f;
  }
  a.rmkey[c] = rm;
}

// Clears the grouping table: slots t, t + stride, ... (below tsize).
__device__ __forceinline__ void clear_table(const CanonArgs& a, uint32_t t, uint32_t stride) {
  for (uint32_t e = t; e < a.tsize; e += stride) {
    a.table[e] = 0ull;
    a.slotmin[e] = ~0ull;
    if (a.slot_gid) a.slot_gid[e] = 0u;
  }
}

// One column of at most CAP entries whose rows are not yet ordered: all its entries
// are loaded at once (clamped addresses), the places beyond the column padded with
// the largest row (rows are below 2^31).  The rows of a column are distinct, so an
// entry's place in row order is the number of smaller rows: one compare-and-add per
// pair, with no further condition.  s is the value at the smallest row, hs the
// column's hash sum.
template <int CAP>
__device__ __forceinline__ void canon_rows(const CanonArgs& a, bool active, uint32_t st, uint32_t m, double* s,
                                           uint64_t* hs) {
  uint32_t rr[CAP];
  double vv[CAP];
#pragma unroll
  for (int j = 0; j < CAP; ++j) {
    const uint32_t e = st + min(static_cast<uint32_t>(j), m > 0 ? m - 1 : 0u);
    const uint32_t r = active ? a.erho[e] : 0xffffffffu;
    rr[j] = static_cast<uint32_t>(j) < m ? r : 0xffffffffu;
    vv[j] = active ? a.ev[e] : 0.0;
  }
  uint32_t rmin = 0xffffffffu;
  double sv = 0.0;
#pragma unroll
  for (int j = 0; j < CAP; ++j) {
    const bool lt = rr[j] < rmin;
    rmin = lt ? rr[j] : rmin;
    sv = lt ? vv[j] : sv;
  }
  uint64_t h = 0;
#pragma unroll
  for (int j = 0; j < CAP; ++j) {
    uint32_t rank = 0;
#pragma unroll
    for (int l = 0; l < CAP; ++l) rank += rr[l] < rr[j] ? 1u : 0u;
    if (static_cast<uint32_t>(j) < m) {
      const double cv = canon_value(vv[j], sv, a.snap);
      a.crho[st + rank] = rr[j];
      a.cval[st + rank] = cv;
      h += col_hash_term(rank, rr[j], cv);
    }
  }
  *s = sv;
  *hs = h;
}

constexpr uint32_t CN_STAGE = 512;  // entries of a wave's columns staged in LDS
// SORT: the rows of a column are not yet ordered (a.sort_rows); the two forms are
// separate kernels so that the ordered one keeps few registers (more waves per CU).
template <bool SORT>
__global__ __launch_bounds__(NT) void k_canon(CanonArgs a, ModeInfo mi) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  clear_table(a, c, gridDim.x * NT);
  const bool active = c < a.ncols;
  const uint32_t st = active ? a.col_start[c] : 0;
  const uint32_t m = active ? a.col_start[c + 1] - st : 0;
  uint64_t hs = 0;
  double s = 0.0;
  if constexpr (!SORT) {
    // Rows already ascending.  A wave's 64 columns are consecutive, so their entries
    // are one contiguous range: when every wave's range of the workgroup fits
    // CN_STAGE entries it is staged through LDS (coalesced loads, each lane then
    // works on its own column there, coalesced stores); otherwise each lane reads its
    // column eight entries at a time (clamped addresses, loads issued together).
    __shared__ uint32_t srho[NT / 64][CN_STAGE];
    __shared__ double sval[NT / 64][CN_STAGE];
    __shared__ int fits;
    const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t cw0 = min(blockIdx.x * NT + w * 64, a.ncols), cw1 = min(cw0 + 64, a.ncols);
    const uint32_t e0 = cw0 < cw1 ? a.col_start[cw0] : 0u, e1 = cw0 < cw1 ? a.col_start[cw1] : 0u;
    if (threadIdx.x == 0) fits = 1;
    __syncthreads();
    if (lane == 0 && e1 - e0 > CN_STAGE) fits = 0;
    __syncthreads();
    if (fits) {
      for (uint32_t j = lane; j < e1 - e0; j += 64) {
        const uint32_t e = e0 + j;
        srho[w][j] = a.erho ? a.erho[e] : static_cast<uint32_t>(a.ekey[e] & a.rho_mask);
        sval[w][j] = a.ev[e];
      }
      __syncthreads();
      if (active) {
        const uint32_t o = st - e0;
        s = sval[w][o];
        for (uint32_t j = 0; j < m; ++j) {
          const double cv = canon_value(sval[w][o + j], s, a.snap);
          sval[w][o + j] = cv;  // this lane's own entries
          hs += col_hash_term(j, srho[w][o + j], cv);
        }
      }
      __syncthreads();
      for (uint32_t j = lane; j < e1 - e0; j += 64) {
        a.crho[e0 + j] = srho[w][j];
        a.cval[e0 + j] = sval[w][j];
      }
    } else if (active) {
      s = a.ev[st];
      for (uint32_t j0 = 0; j0 < m; j0 += 8) {
        uint32_t rr[8];
        double vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t e = st + min(j0 + u, m - 1);
          rr[u] = a.erho ? a.erho[e] : static_cast<uint32_t>(a.ekey[e] & a.rho_mask);
          vv[u] = a.ev[e];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t j = j0 + u;
          if (j < m) {
            const double cv = canon_value(vv[u], s, a.snap);
            a.crho[st + j] = rr[u];
            a.cval[st + j] = cv;
            hs += col_hash_term(j, rr[u], cv);
          }
        }
      }
    }
  } else {
    // at most kMaxLocal entries (checked by the host); the wave's longest column picks
    // the register arrays' size, so short columns cost no more than their length
    uint32_t mw = m;
    for (int o = 32; o > 0; o >>= 1) mw = max(mw, static_cast<uint32_t>(__shfl_xor(mw, o, 64)));
    const uint32_t mwu = __builtin_amdgcn_readfirstlane(mw);
    if (mwu <= 4)
      canon_rows<4>(a, active, st, m, &s, &hs);
    else if (mwu <= 8)
      canon_rows<8>(a, active, st, m, &s, &hs);
    else if (mwu <= 16)
      canon_rows<16>(a, active, st, m, &s, &hs);
    else
      canon_rows<kMaxLocal>(a, active, st, m, &s, &hs);
  }
  if (!active) return;
  a.colhash[c] = col_hash_final(m, hs);
  a.cols[c] = s;
  col_keys(a, mi, c, st);
}

// The same for levels of few columns whose rows are not yet ordered (at most
// kMaxLocal entries each, where one lane per column would leave most of the chip
// idle): one wave per column, one lane per entry.  An entry's place is the number of
// smaller rows among the column's (read lane by lane: the column length is uniform
// over the wave); the value at the smallest row comes from the lane of place 0, and
// the hash terms are summed over the wave.  The same results as k_canon.
constexpr int CW_COLS = NT / 64;  // columns per workgroup
__device__ __forceinline__ void canon_wave_col(const CanonArgs& a, const ModeInfo& mi, uint32_t c, uint32_t lane) {
  const uint32_t st = a.col_start[c];
  const uint32_t m = a.col_start[c + 1] - st;
  const uint32_t mw = min(m, 64u);
  const bool act = lane < mw;
  const uint32_t r = act ? a.erho[st + lane] : 0xffffffffu;
  const double v = act ? a.ev[st + lane] : 0.0;
  uint32_t rank = 0;
  for (uint32_t l = 0; l < mw; ++l)
    rank += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(r), static_cast<int>(l))) < r ? 1u : 0u;
  const int first = __ffsll(static_cast<unsigned long long>(__ballot(act && rank == 0))) - 1;
  const double s = __shfl(v, first, 64);
  uint64_t h = 0;
  if (act) {
    const double cv = canon_value(v, s, a.snap);
    a.crho[st + rank] = r;
    a.cval[st + rank] = cv;
    h = col_hash_term(rank, r, cv);
  }
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
  if (lane == 0) {
    a.colhash[c] = col_hash_final(m, h);
    a.cols[c] = s;
    col_keys(a, mi, c, st);
  }
}
__global__ __launch_bounds__(NT) void k_canon_wave(CanonArgs a, ModeInfo mi) {
  clear_table(a, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
  const uint32_t c = blockIdx.x * CW_COLS + (threadIdx.x >> 6);
  if (c < a.ncols) canon_wave_col(a, mi, c, threadIdx.x & 63);  // the same for the whole wave
}

// The same for levels whose columns are already in row order and include long ones:
// one workgroup per column, its entries spread over the threads.
__global__ __launch_bounds__(NT) void k_canon_wide(CanonArgs a, ModeInfo mi) {
  __shared__ uint64_t red[NT / 64];
  const uint32_t c = blockIdx.x;
  clear_table(a, blockIdx.x * NT + threadIdx.x, gridDim.x * NT);
  const uint32_t st = a.col_start[c], en = a.col_start[c + 1];
  const uint32_t m = en - st;
  const double s = a.ev[st];
  uint64_t hs = 0;
  for (uint32_t j = threadIdx.x; j < m; j += NT) {
    const uint32_t rho = a.erho ? a.erho[st + j] : static_cast<uint32_t>(a.ekey[st + j] & a.rho_mask);
    const double cv = canon_value(a.ev[st + j], s, a.snap);
    a.crho[st + j] = rho;
    a.cval[st + j] = cv;
    hs += col_hash_term(j, rho, cv);
  }
  for (int o = 32; o > 0; o >>= 1) hs += __shfl_xor(hs, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = hs;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    a.colhash[c] = col_hash_final(m, t);
    a.cols[c] = s;
    col_keys(a, mi, c, st);
  }
}

// Entry-by-entry equality of two canonical columns of m entries, eight entries at a
// time with each group's loads issued together (clamped addresses).
__device__ __forceinline__ bool same_column(const uint32_t* __restrict__ crho, const double* __restrict__ cval,
                                            uint32_t sa, uint32_t sb, uint32_t m) {
  for (uint32_t j0 = 0; j0 < m; j0 += 8) {
    uint32_t ra[8], rb[8];
    uint64_t va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t j = min(j0 + u, m - 1);
      ra[u] = crho[sa + j];
      rb[u] = crho[sb + j];
      va[u] = static_cast<uint64_t>(__double_as_longlong(cval[sa + j]));
      vb[u] = static_cast<uint64_t>(__double_as_longlong(cval[sb + j]));
    }
    bool eq = true;
#pragma unroll
    for (int u = 0; u < 8; ++u) eq = eq && ra[u] == rb[u] && va[u] == vb[u];
    if (!eq) return false;
  }
  return true;
}

__global__ __launch_bounds__(NT) void k_group(const uint64_t* __restrict__ colhash, const uint32_t* __restrict__ crho,
                                              const double* __restrict__ cval, const uint32_t* __restrict__ col_start,
                                              const uint64_t* __restrict__ rmkey, uint32_t ncols, uint64_t* table,
                                              uint64_t* slotmin, uint32_t tmask, uint32_t max_probe,
                                              uint32_t* over, uint32_t* __restrict__ slot,
                                              uint32_t* __restrict__ isrep) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  const bool active = c < ncols;
  const uint64_t h = active ? colhash[c] : 0;
  const uint32_t st = active ? col_start[c] : 0;
  const uint32_t m = active ? col_start[c + 1] - st : 0;
  uint32_t p = static_cast<uint32_t>(h) & tmask;
  uint32_t rep = 0;
  // A table with more slots than columns always has an empty slot within reach
  // (max_probe = its size); a smaller one (speculative pass) may not, and a column
  // that finds neither its group nor an empty slot within max_probe probes flags it.
  uint32_t probe = 0;
  for (; active && probe < max_probe; ++probe) {
    uint64_t cur = __hip_atomic_load(&table[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == 0) {
      const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(&table[p]), 0ull,
                                     static_cast<unsigned long long>(c) + 1ull);
      if (old == 0) {
        rep = 1;
        break;
      }
      cur = old;
    }
    const uint32_t r = static_cast<uint32_t>(cur - 1);
    if (colhash[r] == h) {
      const uint32_t sr = col_start[r];
      if (col_start[r + 1] - sr == m && same_column(crho, cval, sr, st, m)) break;
    }
    p = (p + 1) & tmask;
  }
  if (active && probe == max_probe && over) atomicOr(over, 1u);
  if (active) {
    slot[c] = p;
    isrep[c] = rep;
  }
  // Group leader = smallest row-major key (this kernel serves the levels of fewer
  // than 16384 columns; larger ones take k_group_local, which takes the minimum per
  // chunk first)
  const uint64_t rk = active ? rmkey[c] : ~0ull;
  if (active && rk < __hip_atomic_load(&slotmin[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMin(reinterpret_cast<unsigned long long*>(&slotmin[p]), static_cast<unsigned long long>(rk));
}

// Probe of the global table for column c (hash h, m entries from st): returns the
// slot of its group and whether c became the group's representative.
__device__ __forceinline__ uint32_t global_probe(const uint64_t* __restrict__ colhash, const uint32_t* __restrict__ crho,
                                                 const double* __restrict__ cval,
                                                 const uint32_t* __restrict__ col_start, uint64_t* table, uint32_t tmask,
                                                 uint32_t max_probe, uint32_t* over, uint32_t c, uint64_t h,
                                                 uint32_t st, uint32_t m, uint32_t* rep) {
  uint32_t p = static_cast<uint32_t>(h) & tmask;
  *rep = 0;
  for (uint32_t probe = 0; probe < max_probe; ++probe) {
    uint64_t cur = __hip_atomic_load(&table[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == 0) {
      const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(&table[p]), 0ull,
                                     static_cast<unsigned long long>(c) + 1ull);
      if (old == 0) {
        *rep = 1;
        return p;
      }
      cur = old;
    }
    const uint32_t r = static_cast<uint32_t>(cur - 1);
    if (colhash[r] == h) {
      const uint32_t sr = col_start[r];
      if (col_start[r + 1] - sr == m && same_column(crho, cval, sr, st, m)) return p;
    }
    p = (p + 1) & tmask;
  }
  if (over) atomicOr(over, 1u);
  return p;
}

// k_group for large levels, where parallel columns put many columns into few groups:
// a workgroup first groups its GL_CH columns in an LDS table (full-key verification
// against the chunk-local representative, minimum row-major key by LDS atomics),
// then only one column per chunk-local group probes the global table, and the
// group's minimum goes to memory once per chunk.  Same slots, representatives and
// minima as k_group.
// The chunk is GL_CH columns (a power of two, 256 to 2048), chosen per level so that
// the grid has at least 256 workgroups where the level allows, taken by GL_NT threads
// (up to 1024): a thread's columns are handled one after another, each a chain of
// dependent loads, so the more threads the shorter the chain.
template <int GL_CH, int GL_NT>
__global__ __launch_bounds__(GL_NT) void k_group_local(const uint64_t* __restrict__ colhash,
                                                    const uint32_t* __restrict__ crho, const double* __restrict__ cval,
                                                    const uint32_t* __restrict__ col_start,
                                                    const uint64_t* __restrict__ rmkey, uint32_t ncols, uint64_t* table,
                                                    uint64_t* slotmin, uint32_t tmask, uint32_t max_probe,
                                                    uint32_t* over, uint32_t* __restrict__ slot,
                                                    uint32_t* __restrict__ isrep) {
  constexpr int GL_TL = 2 * GL_CH, GL_PT = GL_CH / GL_NT;
  static_assert(GL_CH % GL_NT == 0 && (GL_CH & (GL_CH - 1)) == 0, "chunk of whole thread rounds, a power of two");
  __shared__ uint32_t ltab[GL_TL];   // chunk-local representative + 1, 0 = empty
  __shared__ uint32_t lglob[GL_TL];  // global slot of the local group
  __shared__ uint32_t lrep[GL_TL];   // its representative is the global one
  __shared__ unsigned long long lmin[GL_TL];
  for (int e = threadIdx.x; e < GL_TL; e += GL_NT) {
    ltab[e] = 0u;
    lmin[e] = ~0ull;
  }
  __syncthreads();
  const uint32_t c0 = blockIdx.x * GL_CH;
  uint32_t ls[GL_PT];
  // local grouping
  for (int u = 0; u < GL_PT; ++u) {
    const uint32_t c = c0 + threadIdx.x + u * GL_NT;
    ls[u] = 0xffffffffu;
    if (c >= ncols) continue;
    const uint64_t h = colhash[c];
    const uint32_t st = col_start[c];
    const uint32_t m = col_start[c + 1] - st;
    uint32_t q = static_cast<uint32_t>(h >> 32) & (GL_TL - 1);
    for (int probe = 0; probe < GL_TL; ++probe) {  // at most GL_CH of GL_TL slots are used
      uint32_t cur = ltab[q];
      if (cur == 0u) {
        const uint32_t old = atomicCAS(&ltab[q], 0u, c + 1u);
        if (old == 0u) break;
        cur = old;
      }
      const uint32_t r = cur - 1u;
      if (colhash[r] == h) {
        const uint32_t sr = col_start[r];
        if (col_start[r + 1] - sr == m && same_column(crho, cval, sr, st, m)) break;
      }
      q = (q + 1u) & (GL_TL - 1);
    }
    ls[u] = q;
    atomicMin(&lmin[q], static_cast<unsigned long long>(rmkey[c]));
  }
  __syncthreads();
  // one global probe per chunk-local group (by its local representative)
  for (int u = 0; u < GL_PT; ++u) {
    const uint32_t c = c0 + threadIdx.x + u * GL_NT;
    if (ls[u] == 0xffffffffu || ltab[ls[u]] != c + 1u) continue;
    const uint64_t h = colhash[c];
    const uint32_t st = col_start[c];
    const uint32_t m = col_start[c + 1] - st;
    uint32_t rep;
    const uint32_t p = global_probe(colhash, crho, cval, col_start, table, tmask, max_probe, over, c, h, st, m, &rep);
    lglob[ls[u]] = p;
    lrep[ls[u]] = rep;
    const unsigned long long v = lmin[ls[u]];
    if (v < __hip_atomic_load(&slotmin[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMin(reinterpret_cast<unsigned long long*>(&slotmin[p]), v);
  }
  __syncthreads();
  for (int u = 0; u < GL_PT; ++u) {
    const uint32_t c = c0 + threadIdx.x + u * GL_NT;
    if (ls[u] == 0xffffffffu) continue;
    slot[c] = lglob[ls[u]];
    isrep[c] = (ltab[ls[u]] == c + 1u) ? lrep[ls[u]] : 0u;
  }
}

__global__ __launch_bounds__(NT) void k_rep_list(const uint32_t* __restrict__ isrep, const uint32_t* __restrict__ reppos,
                                                 const uint32_t* __restrict__ slot, const uint64_t* __restrict__ slotmin,
                                                 uint32_t ncols, uint32_t cap, uint64_t* __restrict__ lkey,
                                                 uint64_t* __restrict__ lslot) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c >= ncols || !isrep[c]) return;
  const uint32_t j = reppos[c];
  if (j >= cap) return;
  const uint32_t p = slot[c];
  lkey[j] = slotmin[p];
  lslot[j] = p;
}

__global__ __launch_bounds__(NT) void k_group_ids(const uint64_t* __restrict__ lslot, uint32_t beta_arg,
                                                  const uint32_t* __restrict__ d_beta, uint32_t n,
                                                  const uint64_t* __restrict__ table,
                                                  const uint32_t* __restrict__ col_start, uint32_t* __restrict__ slot_gid,
                                                  uint32_t* __restrict__ nlen) {
  const uint32_t j = blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const uint32_t beta = d_beta ? *d_beta : beta_arg;
  // more groups than the device-count path holds: its leader list was not sorted, so
  // nothing is written (the host redoes this step with the full count)
  if (beta > n) return;
  if (j >= beta) {
    nlen[j] = 0;
    return;
  }
  const uint32_t p = static_cast<uint32_t>(lslot[j]);
  slot_gid[p] = j;
  const uint32_t r = static_cast<uint32_t>(table[p] - 1);
  nlen[j] = col_start[r + 1] - col_start[r];
}

// The leader phase of a level in one workgroup (see launch_leaders).  The rank sort:
// an element's place is the number of smaller keys, or equal ones at a lower index;
// up to 53 key bits the key and the index share one word (key << 11 | index), so one
// comparison decides.  Up to LD_NT leaders, P = 2^k threads share an element, each
// counting over a part of the keys (LDS broadcasts), the parts added by LDS atomics.
constexpr int LD_NT = 1024;
constexpr int LD_PER = static_cast<int>(kLeaderListMax / LD_NT);  // columns per thread
constexpr int LD_TPER = static_cast<int>(kLeaderTableMax / LD_NT);  // table slots per thread
__device__ __forceinline__ void leaders_block(const LeaderArgs& a) {
  __shared__ uint64_t ks[kSmallSortMax];
  __shared__ uint32_t sl[kSmallSortMax];
  __shared__ uint32_t rk[kSmallSortMax];
  __shared__ uint32_t ln[kSmallSortMax];
  __shared__ uint32_t rp[kSmallSortMax];  // representative column (list from the table)
  __shared__ uint32_t red[LD_NT / 64];
  const uint32_t t = threadIdx.x;
  const uint64_t mask = (a.nbits >= 64) ? ~0ull : ((1ull << a.nbits) - 1ull);
  const bool packed = a.nbits <= 53;
  uint32_t n;
  if (a.tscan) {
    // thread t takes a contiguous run of at most LD_TPER slots, their entries and
    // minima loaded together; the sort below orders the groups, so the list may
    // follow slot order
    const uint32_t per = (a.tsize + LD_NT - 1) / LD_NT;
    const uint32_t b = min(a.tsize, t * per), e = min(a.tsize, b + per);
    uint64_t tv[LD_TPER], mk[LD_TPER];
    uint32_t cnt = 0;
#pragma unroll
    for (int u = 0; u < LD_TPER; ++u) {
      tv[u] = (b + u < e) ? a.table[b + u] : 0ull;
      mk[u] = (b + u < e) ? a.slotmin[b + u] : 0ull;
      cnt += tv[u] ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t pos = block_excl_scan_u32<LD_NT>(cnt, red, &tot);
#pragma unroll
    for (int u = 0; u < LD_TPER; ++u) {
      if (!tv[u]) continue;
      if (pos < a.cap) {
        ks[pos] = mk[u] & mask;
        sl[pos] = b + u;
        rp[pos] = static_cast<uint32_t>(tv[u] - 1);
      }
      ++pos;
    }
    n = tot;
    if (t == 0) *a.d_beta = n;
  } else if (a.isrep) {
    // thread t takes a contiguous run of at most LD_PER columns, each step's loads
    // for the whole run issued together (flags, then slots, then slot minima)
    const uint32_t per = (a.ncols + LD_NT - 1) / LD_NT;
    const uint32_t b = min(a.ncols, t * per), e = min(a.ncols, b + per);
    uint32_t fl[LD_PER], sp[LD_PER];
    uint64_t mk[LD_PER];
    uint32_t cnt = 0;
#pragma unroll
    for (int u = 0; u < LD_PER; ++u) {
      fl[u] = (b + u < e) ? a.isrep[b + u] : 0u;
      cnt += fl[u] ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < LD_PER; ++u) sp[u] = fl[u] ? a.slot[b + u] : 0u;
#pragma unroll
    for (int u = 0; u < LD_PER; ++u) mk[u] = fl[u] ? a.slotmin[sp[u]] : 0ull;
    uint32_t tot;
    uint32_t pos = block_excl_scan_u32<LD_NT>(cnt, red, &tot);
#pragma unroll
    for (int u = 0; u < LD_PER; ++u) {
      if (!fl[u]) continue;
      a.reppos[b + u] = pos;
      if (pos < a.cap) {
        ks[pos] = mk[u] & mask;
        sl[pos] = sp[u];
      }
      ++pos;
    }
    n = tot;
    if (t == 0) *a.d_beta = n;
  } else {
    n = *a.d_beta;
    const uint32_t nl = min(n, a.cap);
    for (uint32_t i = t; i < nl; i += LD_NT) {
      ks[i] = a.lkey[i] & mask;
      sl[i] = static_cast<uint32_t>(a.lslot[i]);
    }
  }
  if (n == 0 || n > a.cap) return;  // the same for every thread
  __syncthreads();
  for (uint32_t i = t; i < n; i += LD_NT) {
    if (packed) ks[i] = (ks[i] << 11) | i;
    rk[i] = 0u;
  }
  __syncthreads();
  if (n <= static_cast<uint32_t>(LD_NT)) {
    uint32_t P = 1;
    while (P < static_cast<uint32_t>(LD_NT) && n * P * 2 <= static_cast<uint32_t>(LD_NT)) P *= 2;
    const uint32_t i = t / P, part = t % P;
    if (i < n) {
      const uint32_t len = (n + P - 1) / P, j0 = min(n, part * len), j1 = min(n, j0 + len);
      const uint64_t ki = ks[i];
      uint32_t r = 0;
#pragma unroll 8
      for (uint32_t j = j0; j < j1; ++j) {
        const uint64_t kj = ks[j];
        r += (kj < ki || (!packed && kj == ki && j < i)) ? 1u : 0u;
      }
      if (P == 1)
        rk[i] = r;
      else if (r)
        atomicAdd(&rk[i], r);
    }
  } else {
    const uint32_t i0 = t, i1 = t + LD_NT;
    const uint64_t k0 = ks[i0], k1 = i1 < n ? ks[i1] : ~0ull;
    uint32_t r0 = 0, r1 = 0;
#pragma unroll 8
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t kj = ks[j];
      r0 += (kj < k0 || (!packed && kj == k0 && j < i0)) ? 1u : 0u;
      r1 += (kj < k1 || (!packed && kj == k1 && j < i1)) ? 1u : 0u;
    }
    rk[i0] = r0;
    if (i1 < n) rk[i1] = r1;
  }
  __syncthreads();
  for (uint32_t i = t; i < n; i += LD_NT) {
    const uint32_t r = rk[i], p = sl[i];
    a.lss[r] = p;
    a.slot_gid[p] = r;
    const uint32_t rep = a.tscan ? rp[i] : static_cast<uint32_t>(a.table[p] - 1);
    ln[r] = a.col_start[rep + 1] - a.col_start[rep];
  }
  __syncthreads();
  const uint32_t per = (n + LD_NT - 1) / LD_NT;
  const uint32_t b = min(n, t * per), e = min(n, b + per);
  uint32_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += ln[i];
  uint32_t tot;
  uint32_t run = block_excl_scan_u32<LD_NT>(sum, red, &tot);
  for (uint32_t i = b; i < e; ++i) {
    a.npos[i] = run;
    run += ln[i];
  }
  if (t == 0) *a.d_nnz = tot;
}
__global__ __launch_bounds__(LD_NT) void k_leaders(LeaderArgs a) { leaders_block(a); }

// N_k's column of group j.
__device__ __forceinline__ void emit_n_group(const EmitArgs& a, uint32_t j) {
  // more groups than the launch covers (a speculative pass whose leader list was
  // capped): nothing is written, the pass is redone
  if (*a.d_beta > a.bmax) return;
  const uint32_t beta = *a.d_beta;
  if (j == 0) a.colptr[beta] = *a.d_nnz;
  if (j >= beta) return;
  const uint32_t p = static_cast<uint32_t>(a.lss[j]);
  const uint32_t r = static_cast<uint32_t>(a.table[p] - 1);
  const uint32_t s0 = a.col_start[r], m = a.col_start[r + 1] - s0;
  const uint32_t o = a.npos[j];
  a.colptr[j] = o;
  // eight entries at a time, each group's loads issued together (clamped addresses;
  // a column has at least one entry)
  for (uint32_t t0 = 0; t0 < m; t0 += 8) {
    uint32_t rr[8];
    double vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t t = min(t0 + u, m - 1);
      rr[u] = a.crho[s0 + t];
      vv[u] = a.cval[s0 + t];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t0 + u < m) {
        a.nrow[o + t0 + u] = static_cast<int32_t>(rr[u]);
        a.nval[o + t0 + u] = vv[u];
      }
  }
}

// Column c's entry of the next level (or of the last core).
__device__ __forceinline__ void emit_next_col(const EmitArgs& a, const ModeInfo& mi, uint32_t c) {
  const uint32_t g = a.slot_gid[a.slot[c]];
  const uint64_t suf = a.colsuf[c];
  const double s = a.cols[c];
  if (a.out_g) {
    int64_t lin = 0;
    const uint32_t base = mi.off[a.kidx];
    for (int j = a.kidx; j < mi.d; ++j)
      lin = lin * static_cast<int64_t>(mi.n[j]) + static_cast<int64_t>((suf >> (mi.off[j] - base)) & fmask(mi.bits[j]));
    a.out_col[c] = lin;
    a.out_g[c] = static_cast<int32_t>(g);
    a.out_s[c] = s;
  }
  const uint32_t inext = static_cast<uint32_t>(suf & fmask(mi.bits[a.kidx]));
  if (!a.last) {
    a.next_ekey[c] = suf;
    a.next_rho[c] = g * mi.n[a.kidx] + inext;
    a.next_v[c] = s;
  } else {
    a.last_core[static_cast<size_t>(g) * mi.n[a.kidx] + inext] = s;
  }
}

// The first nb_next workgroups take the columns (next level), the rest the groups (N_k).
__global__ __launch_bounds__(NT) void k_emit(EmitArgs a, ModeInfo mi, uint32_t nb_next) {
  if (blockIdx.x >= nb_next) {
    emit_n_group(a, (blockIdx.x - nb_next) * NT + threadIdx.x);
    return;
  }
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c < a.ncols) emit_next_col(a, mi, c);
}

}  // namespace

void launch_ingest(const int32_t* idx, const double* val, uint32_t nnz, const ModeInfo& mi, uint64_t* keys,
                   uint64_t* vbits, DevStatus* st, hipStream_t s) {
  if (!nnz) return;
  const int vec4 = (mi.d % 4 == 0) && (reinterpret_cast<uintptr_t>(idx) % 16 == 0);
  k_ingest<<<grid_for(nnz, NT), NT, 0, s>>>(idx, val, nnz, mi, keys, vbits, st, vec4);
  TTS_LAUNCH_CHECK();
}

uint32_t norm_partials_count(uint32_t nE) { return grid_for(nE, NT); }

void launch_col_flags(const uint64_t* ekey, uint32_t nE, int sh, bool level1, int long_bit, const double* ev,
                      uint32_t* flag, double* norm_part, DevStatus* st, hipStream_t s) {
  k_col_flags<<<grid_for(nE, NT), NT, 0, s>>>(ekey, nE, sh, level1 ? 1 : 0, long_bit, ev, flag, norm_part, st);
  TTS_LAUNCH_CHECK();
}

void launch_norm_final(const double* part, uint32_t np, DevStatus* st, hipStream_t s) {
  k_norm_final<<<1, NF, 0, s>>>(part, np, st);
  TTS_LAUNCH_CHECK();
}

void launch_columns_small(const uint64_t* ekey, uint32_t nE, int sh, int long_bit, uint32_t* col_start,
                          uint32_t* d_ncols, DevStatus* st, hipStream_t s) {
  if (nE == 0 || nE > kColsSmallMax) fail(TT_ERR_TOO_LARGE, "one-workgroup column pass beyond its capacity");
  k_columns_small<<<1, CS_NT, 0, s>>>(ekey, nE, sh, long_bit, col_start, d_ncols, st);
  TTS_LAUNCH_CHECK();
}

uint32_t starts_tiles(uint32_t nE) { return (nE + ST_TILE - 1) / ST_TILE; }

void launch_starts(const uint64_t* ekey, uint32_t nE, int sh, bool level1, int long_bit, const double* ev,
                   uint32_t* part, double* norm_part, uint32_t* col_start, uint32_t* d_ncols, DevStatus* st,
                   hipStream_t s) {
  const uint32_t nt = starts_tiles(nE);
  if (nE == 0 || nt > kStartsMaxTiles) fail(TT_ERR_TOO_LARGE, "column pass beyond its tile count");
  k_starts_count<<<nt, NT, 0, s>>>(ekey, nE, sh, level1 ? 1 : 0, long_bit, ev, part, norm_part, st);
  TTS_LAUNCH_CHECK();
  k_starts_place<<<nt, NT, 0, s>>>(ekey, nE, sh, part, col_start, d_ncols);
  TTS_LAUNCH_CHECK();
}

void launch_col_starts(const uint32_t* flag, const uint32_t* pos, uint32_t nE, uint32_t* col_start,
                       const uint32_t* d_ncols, hipStream_t s) {
  k_col_starts<<<grid_for(nE, NT), NT, 0, s>>>(flag, pos, nE, col_start, d_ncols);
  TTS_LAUNCH_CHECK();
}

void launch_level_counts(const uint64_t* keys, uint32_t n, const ModeInfo& mi, uint32_t* counts, DevStatus* st,
                         hipStream_t s) {
  if (n == 0 || mi.d < 2) return;
  const dim3 grid(std::min<unsigned>(grid_for(n, NT), 1024u), static_cast<unsigned>((mi.d - 2) / LC_PER + 1));
  k_level_counts<<<grid, NT, 0, s>>>(keys, n, mi, counts, st);
  TTS_LAUNCH_CHECK();
}

void launch_make_composite(const uint32_t* flag, const uint32_t* pos, const uint32_t* erho, uint32_t nE, int rbits,
                           uint64_t* ckey, uint64_t* cval, hipStream_t s) {
  k_make_composite<<<grid_for(nE, NT), NT, 0, s>>>(flag, pos, erho, nE, rbits, ckey, cval);
  TTS_LAUNCH_CHECK();
}

void launch_permute_entries(const uint64_t* perm, uint32_t nE, const uint64_t* ekey_in, const uint32_t* erho_in,
                            const double* ev_in, uint64_t* ekey_out, uint32_t* erho_out, double* ev_out,
                            hipStream_t s) {
  k_permute<<<grid_for(nE, NT), NT, 0, s>>>(perm, nE, ekey_in, erho_in, ev_in, ekey_out, erho_out, ev_out);
  TTS_LAUNCH_CHECK();
}

void launch_canon(const CanonArgs& a, const ModeInfo& mi, DevStatus*, bool wide, hipStream_t s) {
  if (!a.ncols) return;
  // per column: read its entries' (key, rho, value) once, write (rho, c) and the
  // column record (hash, s, suffix, row-major key) once -- the caller passes the
  // entry count through the column starts; bytes are estimated from ncols here
  KTimer kt("level_canon", s, 56.0 * a.ncols, 0.0);
  if (wide && !a.sort_rows)
    k_canon_wide<<<a.ncols, NT, 0, s>>>(a, mi);
  else if (a.sort_rows && a.ncols <= kCanonWaveMax)
    k_canon_wave<<<grid_for(a.ncols, CW_COLS), NT, 0, s>>>(a, mi);
  else if (a.sort_rows)
    k_canon<true><<<grid_for(a.ncols, NT), NT, 0, s>>>(a, mi);
  else
    k_canon<false><<<grid_for(a.ncols, NT), NT, 0, s>>>(a, mi);
  TTS_LAUNCH_CHECK();
}

void launch_group(const uint64_t* colhash, const uint32_t* crho, const double* cval, const uint32_t* col_start,
                  const uint64_t* rmkey, uint32_t ncols, uint64_t* table, uint64_t* slotmin, uint32_t tmask,
                  uint32_t max_probe, uint32_t* over, uint32_t* slot, uint32_t* isrep, hipStream_t s) {
  if (!ncols) return;
  // per column: read hash, start and row-major key, write slot and flag
  KTimer kt("level_group", s, 32.0 * ncols, 0.0);
  if (ncols >= 16384) {
    // large levels: chunk-local grouping first (see k_group_local), with chunks small
    // enough for at least 256 workgroups (down to 256 columns)
#define TTS_GROUP_LOCAL(CH)                                                                                    \
  k_group_local<CH, ((CH) < 1024 ? (CH) : 1024)><<<(ncols + (CH) - 1) / (CH), ((CH) < 1024 ? (CH) : 1024), 0, s>>>( \
      colhash, crho, cval, col_start, rmkey, ncols, table, slotmin, tmask, max_probe, over, slot, isrep)
    if (ncols >= 256u * 2048u)
      TTS_GROUP_LOCAL(2048);
    else if (ncols >= 256u * 1024u)
      TTS_GROUP_LOCAL(1024);
    else if (ncols >= 256u * 512u)
      TTS_GROUP_LOCAL(512);
    else
      TTS_GROUP_LOCAL(256);
#undef TTS_GROUP_LOCAL
  } else {
    k_group<<<grid_for(ncols, NT), NT, 0, s>>>(colhash, crho, cval, col_start, rmkey, ncols, table, slotmin, tmask,
                                               max_probe, over, slot, isrep);
  }
  TTS_LAUNCH_CHECK();
}

void launch_rep_list(const uint32_t* isrep, const uint32_t* reppos, const uint32_t* slot, const uint64_t* slotmin,
                     uint32_t ncols, uint32_t cap, uint64_t* lkey, uint64_t* lslot, hipStream_t s) {
  if (!ncols || !cap) return;
  k_rep_list<<<grid_for(ncols, NT), NT, 0, s>>>(isrep, reppos, slot, slotmin, ncols, cap, lkey, lslot);
  TTS_LAUNCH_CHECK();
}

void launch_group_ids(const uint64_t* lslot_sorted, uint32_t beta, const uint32_t* d_beta, uint32_t n,
                      const uint64_t* table, const uint32_t* col_start, uint32_t* slot_gid, uint32_t* nlen,
                      hipStream_t s) {
  if (!n) return;
  k_group_ids<<<grid_for(n, NT), NT, 0, s>>>(lslot_sorted, beta, d_beta, n, table, col_start, slot_gid, nlen);
  TTS_LAUNCH_CHECK();
}

void launch_leaders(const LeaderArgs& a, hipStream_t s) {
  if (a.cap == 0) return;
  if (a.cap > kSmallSortMax || (a.tscan && a.tsize > kLeaderTableMax) || (a.isrep && a.ncols > kLeaderListMax))
    fail(TT_ERR_TOO_LARGE, "leader phase beyond its one-workgroup capacity");
  k_leaders<<<1, LD_NT, 0, s>>>(a);
  TTS_LAUNCH_CHECK();
}

void launch_emit(const EmitArgs& a, const ModeInfo& mi, hipStream_t s) {
  const uint32_t nb_next = a.ncols ? grid_for(a.ncols, NT) : 0u;
  k_emit<<<nb_next + grid_for(a.bmax, NT), NT, 0, s>>>(a, mi, nb_next);
  TTS_LAUNCH_CHECK();
}

}  // namespace tts
