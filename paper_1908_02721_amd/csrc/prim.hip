// Device-wide exclusive scan and stable LSD radix sort, hand-written for gfx950.
//
// Radix sort: 8-bit digits, one pass per digit, three kernels per pass:
//   k_rs_hist      -- per-tile digit histogram (LDS atomics), written digit-major.
//   k_rs_scan_rows -- exclusive scan of each digit's row of tile counts, plus the
//                     digit totals.
//   k_rs_scatter   -- stable per-tile ranking (ballot match inside each wave, wave
//                     prefix over the tile), staging through LDS so that the global
//                     writes of one digit run are contiguous.
// A single tile needs only the scatter: its own offsets are the global ones.
// No inter-block waiting anywhere: every kernel only reads what earlier launches
// wrote.
#include "prim.hpp"

namespace tts {

namespace {

constexpr int SCAN_NT = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IPT;

// A thread's SCAN_IPT = 8 consecutive words: two 16-byte loads when the buffer is
// 16-byte aligned and the run is whole, guarded word loads otherwise.
__device__ __forceinline__ void load_run8(const uint32_t* in, size_t j, uint32_t n, bool vec, uint32_t v[8]) {
  if (vec && j + 8 <= n) {
    const uint4 a = *reinterpret_cast<const uint4*>(in + j);
    const uint4 b = *reinterpret_cast<const uint4*>(in + j + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (j + i < n) ? in[j + i] : 0u;
  }
}

__device__ __forceinline__ void store_run8(uint32_t* out, size_t j, uint32_t n, bool vec, const uint32_t v[8]) {
  if (vec && j + 8 <= n) {
    *reinterpret_cast<uint4*>(out + j) = make_uint4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<uint4*>(out + j + 4) = make_uint4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (j + i < n) out[j + i] = v[i];
  }
}

static_assert(SCAN_IPT == 8, "the run loads assume eight words per thread");

__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(const uint32_t* __restrict__ in, uint32_t n,
                                                         uint32_t* __restrict__ part, int vec) {
  __shared__ uint32_t lds[SCAN_NT / 64];
  const size_t base = static_cast<size_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_IPT;
  uint32_t v[SCAN_IPT];
  load_run8(in, base, n, vec != 0, v);
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) s += v[i];
  uint32_t tot;
  block_excl_scan_u32<SCAN_NT>(s, lds, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* __restrict__ part, uint32_t nb,
                                                        uint32_t* __restrict__ d_total) {
  __shared__ uint32_t lds[1024 / 64];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t j = base + threadIdx.x;
    const uint32_t x = (j < nb) ? part[j] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan_u32<1024>(x, lds, &tot);
    if (j < nb) part[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && d_total) *d_total = carry;
}

// Second pass.  With `fused`, part[] holds the raw tile sums (at most FUSED_TILES of
// them) and each tile adds up the sums before it itself; the last tile writes the
// total.  Otherwise part[] already holds the exclusive prefixes.
constexpr uint32_t FUSED_TILES = 4096;
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const uint32_t* in, uint32_t* out, uint32_t n,
                                                        const uint32_t* __restrict__ part, int fused,
                                                        uint32_t* __restrict__ d_total, int vin, int vout) {
  __shared__ uint32_t lds[SCAN_NT / 64];
  const size_t base = static_cast<size_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_IPT;
  uint32_t v[SCAN_IPT];
  load_run8(in, base, n, vin != 0, v);
  uint32_t prefix;
  if (fused) {
    constexpr int R = FUSED_TILES / SCAN_NT;
    uint32_t q[R];
    const uint32_t b = blockIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t j = threadIdx.x + r * SCAN_NT;
      q[r] = part[j < b ? j : 0u];
    }
    uint32_t p = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) p += (threadIdx.x + r * SCAN_NT < b) ? q[r] : 0u;
    block_excl_scan_u32<SCAN_NT>(p, lds, &prefix);
  } else {
    prefix = part[blockIdx.x];
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) s += v[i];
  uint32_t tot;
  uint32_t run = block_excl_scan_u32<SCAN_NT>(s, lds, &tot) + prefix;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    const uint32_t x = v[i];
    v[i] = run;
    run += x;
  }
  store_run8(out, base, n, vout != 0, v);
  if (fused && d_total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *d_total = prefix + tot;
}

// ----------------------------------------------------------------------------
constexpr int RS_NT = 256;
constexpr int RS_NW = RS_NT / 64;
constexpr int RS_IPT = 16;
constexpr int RS_TILE = RS_NT * RS_IPT;  // 4096 items per tile

// Mask of the lanes of this wave that hold the same 8-bit digit (all lanes must
// be active).
__device__ __forceinline__ uint64_t match_digit(unsigned dig) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (dig >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// Per-tile digit histogram: LDS atomic adds (integer counts, so the order of the adds
// does not matter), all of a thread's keys loaded before any add.  Written digit-major.
// Per-tile digit counts.  Each wave counts into its own 256 bins, and a row of keys
// whose digit is the same in every lane of the wave (common in the high digits of
// structured keys, where per-lane atomics on one bin would serialise) is counted by
// one lane; the bins are summed per digit at the end.
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t* __restrict__ keys, uint32_t n, int shift,
                                                   uint32_t* __restrict__ counts, uint32_t ntiles) {
  __shared__ uint32_t h[RS_NW][256];
#pragma unroll
  for (int w = 0; w < RS_NW; ++w) h[w][threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t base = static_cast<size_t>(blockIdx.x) * RS_TILE;
  unsigned dig[RS_IPT];
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const size_t i = base + static_cast<size_t>(r) * RS_NT + threadIdx.x;
    dig[r] = (i < n) ? static_cast<unsigned>((keys[i] >> shift) & 255u) : 256u;
  }
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const unsigned d0 = __builtin_amdgcn_readfirstlane(dig[r]);
    if (__ballot(dig[r] != d0) == 0ull) {  // uniform over the wave
      if (lane == 0 && d0 < 256u) atomicAdd(&h[wv][d0], 64u);
    } else if (dig[r] < 256u) {
      atomicAdd(&h[wv][dig[r]], 1u);
    }
  }
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int w = 0; w < RS_NW; ++w) t += h[w][threadIdx.x];
  counts[static_cast<size_t>(threadIdx.x) * ntiles + blockIdx.x] = t;
}

// Exclusive scan of one digit's row of per-tile counts (one workgroup per digit),
// in place; the row total goes to dtot[digit].  The scatter adds the exclusive scan
// of the 256 digit totals itself.
__global__ __launch_bounds__(RS_NT) void k_rs_scan_rows(uint32_t* __restrict__ counts, uint32_t ntiles,
                                                        uint32_t* __restrict__ dtot) {
  __shared__ uint32_t lds[RS_NW];
  constexpr int IPT = 4;
  uint32_t* row = counts + static_cast<size_t>(blockIdx.x) * ntiles;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < ntiles; base += RS_NT * IPT) {
    const uint32_t j0 = base + threadIdx.x * IPT;
    uint32_t v[IPT], s = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      v[i] = (j0 + i < ntiles) ? row[j0 + i] : 0u;
      s += v[i];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan_u32<RS_NT>(s, lds, &tot);
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      if (j0 + i < ntiles) row[j0 + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                      const uint64_t* __restrict__ vin,
                                                      uint64_t* __restrict__ kout,
                                                      uint64_t* __restrict__ vout, uint32_t n, int shift,
                                                      const uint32_t* __restrict__ offs,
                                                      const uint32_t* __restrict__ dtot, uint32_t ntiles) {
  __shared__ uint32_t wcnt[RS_NW][256];
  __shared__ uint32_t toff[256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t scan_lds[RS_NW];
  __shared__ uint64_t stage[RS_TILE];
  __shared__ uint8_t sdig[RS_TILE];

  for (int i = threadIdx.x; i < RS_NW * 256; i += RS_NT) (&wcnt[0][0])[i] = 0;
  // global offset of this tile's run of each digit; a single tile (offs == nullptr)
  // takes its own tile offsets, set below
  uint32_t gbase = 0;
  if (offs) {
    uint32_t all;
    gbase = block_excl_scan_u32<RS_NT>(dtot[threadIdx.x], scan_lds, &all) +
            offs[static_cast<size_t>(threadIdx.x) * ntiles + blockIdx.x];
  }
  __syncthreads();

  const unsigned w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t tile0 = static_cast<size_t>(blockIdx.x) * RS_TILE;
  const size_t base = tile0 + static_cast<size_t>(w) * 64 * RS_IPT;
  uint64_t k[RS_IPT], v[RS_IPT];
  uint32_t rk[RS_IPT];
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const size_t i = base + static_cast<size_t>(r) * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? kin[i] : 0ull;
    v[r] = valid ? vin[i] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const size_t i = base + static_cast<size_t>(r) * 64 + lane;
    const bool valid = i < n;
    const unsigned dig = static_cast<unsigned>((k[r] >> shift) & 255u);
    const uint64_t peers = match_digit(dig) & __ballot(valid);
    const uint32_t pre = static_cast<uint32_t>(__popcll(peers & lanemask_lt()));
    const uint32_t old = valid ? wcnt[w][dig] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && pre == 0) wcnt[w][dig] = old + static_cast<uint32_t>(__popcll(peers));
    __builtin_amdgcn_wave_barrier();
    rk[r] = old + pre;
  }
  __syncthreads();
  {
    const unsigned t = threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int ww = 0; ww < RS_NW; ++ww) {
      const uint32_t c = wcnt[ww][t];
      wcnt[ww][t] = s;
      s += c;
    }
    uint32_t tot;
    const uint32_t to = block_excl_scan_u32<RS_NT>(s, scan_lds, &tot);
    toff[t] = to;
    goff[t] = offs ? gbase : to;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const size_t i = base + static_cast<size_t>(r) * 64 + lane;
    if (i < n) {
      const unsigned dig = static_cast<unsigned>((k[r] >> shift) & 255u);
      const uint32_t pos = toff[dig] + wcnt[w][dig] + rk[r];
      stage[pos] = k[r];
      sdig[pos] = static_cast<uint8_t>(dig);
    }
  }
  __syncthreads();
  const uint32_t cnt = static_cast<uint32_t>(min(static_cast<size_t>(RS_TILE), n - tile0));
  for (uint32_t j = threadIdx.x; j < cnt; j += RS_NT) {
    const unsigned dig = sdig[j];
    kout[goff[dig] + (j - toff[dig])] = stage[j];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const size_t i = base + static_cast<size_t>(r) * 64 + lane;
    if (i < n) {
      const unsigned dig = static_cast<unsigned>((k[r] >> shift) & 255u);
      stage[toff[dig] + wcnt[w][dig] + rk[r]] = v[r];
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < cnt; j += RS_NT) {
    const unsigned dig = sdig[j];
    vout[goff[dig] + (j - toff[dig])] = stage[j];
  }
}

// Exclusive scan of up to SMALL_SCAN elements in one launch: the input is staged in
// LDS with coalesced loads, each of the 1024 threads scans a contiguous run, and the
// runs are combined with a workgroup scan.
constexpr uint32_t SMALL_SCAN = 16384;
// One workgroup: thread t scans a contiguous run of `per` elements.  The LDS copy has
// one padding word per 32, so that the runs of neighbouring threads (a power-of-two
// stride apart) fall into different banks.
__device__ __forceinline__ uint32_t scan_pad(uint32_t i) { return i + (i >> 5); }
__global__ __launch_bounds__(1024) void k_scan_single(const uint32_t* in, uint32_t* out, uint32_t n,
                                                      uint32_t* __restrict__ d_total) {
  __shared__ uint32_t buf[SMALL_SCAN + SMALL_SCAN / 32];
  __shared__ uint32_t lds[1024 / 64];
  for (uint32_t i = threadIdx.x; i < n; i += 1024) buf[scan_pad(i)] = in[i];
  __syncthreads();
  const uint32_t per = (n + 1023) / 1024;
  const uint32_t b = min(n, threadIdx.x * per), e = min(n, b + per);
  uint32_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += buf[scan_pad(i)];
  uint32_t tot;
  uint32_t run = block_excl_scan_u32<1024>(sum, lds, &tot);
  for (uint32_t i = b; i < e; ++i) {
    const uint32_t v = buf[scan_pad(i)];
    buf[scan_pad(i)] = run;
    run += v;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += 1024) out[i] = buf[scan_pad(i)];
  if (threadIdx.x == 0 && d_total) *d_total = tot;
}

// Stable sort of up to SMALL_SORT pairs by key bits [0, nbits) in one workgroup:
// each element's output position is the number of elements with a smaller masked
// key, or an equal one at a lower index.  With nbits <= 53 the key and the index are
// packed into one word (key << 11 | index), so that one comparison decides.  Up to
// 1024 elements, P = 2^k threads share an element (n P <= 1024), each counting over
// a contiguous part of the keys (staged in LDS, read as broadcasts), and the parts
// are added with LDS atomics (integers: the order does not matter).
constexpr uint32_t SMALL_SORT = kSmallSortMax;
__global__ __launch_bounds__(1024) void k_sort_small(const uint64_t* __restrict__ keys,
                                                     const uint64_t* __restrict__ vals, uint32_t n_arg, int nbits,
                                                     uint64_t* __restrict__ kout, uint64_t* __restrict__ vout,
                                                     const uint32_t* __restrict__ d_n, uint32_t cap) {
  __shared__ uint64_t ks[SMALL_SORT];
  __shared__ uint32_t rk[SMALL_SORT];
  const uint32_t n = d_n ? *d_n : n_arg;  // the count from the device when given
  if (n == 0 || n > cap) return;
  const uint64_t mask = (nbits >= 64) ? ~0ull : ((1ull << nbits) - 1ull);
  const bool packed = nbits <= 53;
  for (uint32_t i = threadIdx.x; i < n; i += 1024) {
    const uint64_t k = keys[i] & mask;
    ks[i] = packed ? ((k << 11) | i) : k;
    rk[i] = 0;
  }
  __syncthreads();
  if (n <= 1024) {
    uint32_t P = 1;
    while (P < 1024 && n * P * 2 <= 1024) P *= 2;
    const uint32_t i = threadIdx.x / P, part = threadIdx.x % P;
    if (i < n) {
      const uint32_t len = (n + P - 1) / P, j0 = part * len, j1 = min(n, j0 + len);
      const uint64_t ki = ks[i];
      uint32_t r = 0;
      if (packed) {
#pragma unroll 8
        for (uint32_t j = j0; j < j1; ++j) r += (ks[j] < ki) ? 1u : 0u;
      } else {
#pragma unroll 8
        for (uint32_t j = j0; j < j1; ++j) {
          const uint64_t kj = ks[j];
          r += (kj < ki || (kj == ki && j < i)) ? 1u : 0u;
        }
      }
      if (P == 1)
        rk[i] = r;
      else
        atomicAdd(&rk[i], r);
    }
  } else {
    constexpr int EPT = SMALL_SORT / 1024;
    uint64_t km[EPT];
    uint32_t rank[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t i = threadIdx.x + e * 1024;
      km[e] = (i < n) ? ks[i] : ~0ull;
      rank[e] = 0;
    }
#pragma unroll 8
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t kj = ks[j];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const uint32_t i = threadIdx.x + e * 1024;
        rank[e] += (packed ? (kj < km[e]) : (kj < km[e] || (kj == km[e] && j < i))) ? 1u : 0u;
      }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t i = threadIdx.x + e * 1024;
      if (i < n) rk[i] = rank[e];
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += 1024) {
    const uint32_t r = rk[i];
    kout[r] = keys[i];
    vout[r] = vals[i];
  }
}

}  // namespace

void exclusive_scan_u32(Allocator* al, const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total,
                        hipStream_t s) {
  if (n == 0) {
    if (d_total) TTS_HIP(hipMemsetAsync(d_total, 0, sizeof(uint32_t), s));
    return;
  }
  if (n <= SMALL_SCAN) {
    k_scan_single<<<1, 1024, 0, s>>>(in, out, n, d_total);
    TTS_LAUNCH_CHECK();
    return;
  }
  const uint32_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DBuf<uint32_t> part(al, nb);
  const int vin = (reinterpret_cast<uintptr_t>(in) & 15u) == 0;
  const int vout = (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  k_scan_reduce<<<nb, SCAN_NT, 0, s>>>(in, n, part.get(), vin);
  TTS_LAUNCH_CHECK();
  const int fused = nb <= FUSED_TILES;
  if (!fused) {
    k_scan_partials<<<1, 1024, 0, s>>>(part.get(), nb, d_total);
    TTS_LAUNCH_CHECK();
  }
  k_scan_apply<<<nb, SCAN_NT, 0, s>>>(in, out, n, part.get(), fused, d_total, vin, vout);
  TTS_LAUNCH_CHECK();
}

bool radix_sort_pairs_pp(Allocator* al, uint64_t* keys, uint64_t* vals, uint64_t* ktmp, uint64_t* vtmp,
                         uint32_t n, int nbits, hipStream_t s) {
  if (n <= 1 || nbits <= 0) return false;
  // the rank sort costs about 3 + n^2 / 50000 us, a radix pass over one tile about
  // 10 us (more tiles: a few us more per tile)
  const uint64_t passes_n = static_cast<uint64_t>((nbits + 7) / 8);
  if (n <= SMALL_SORT && static_cast<uint64_t>(n) * n <= 40000ull * (10 * passes_n - 3)) {
    k_sort_small<<<1, 1024, 0, s>>>(keys, vals, n, nbits, ktmp, vtmp, nullptr, SMALL_SORT);
    TTS_LAUNCH_CHECK();
    return true;
  }
  const uint32_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  const int passes = (nbits + 7) / 8;
  DBuf<uint32_t> counts(al, ntiles > 1 ? static_cast<size_t>(256) * ntiles + 256 : 1);
  uint32_t* dtot = counts.get() + static_cast<size_t>(256) * ntiles;
  uint64_t *ki = keys, *vi = vals, *ko = ktmp, *vo = vtmp;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    if (ntiles > 1) {
      k_rs_hist<<<ntiles, RS_NT, 0, s>>>(ki, n, shift, counts.get(), ntiles);
      TTS_LAUNCH_CHECK();
      k_rs_scan_rows<<<256, RS_NT, 0, s>>>(counts.get(), ntiles, dtot);
      TTS_LAUNCH_CHECK();
    }
    {
      // algorithmic bytes of one pass: read and write every (key, value) pair once
      KTimer kt("sort_scatter", s, 32.0 * n, 0.0);
      k_rs_scatter<<<ntiles, RS_NT, 0, s>>>(ki, vi, ko, vo, n, shift, ntiles > 1 ? counts.get() : nullptr,
                                            ntiles > 1 ? dtot : nullptr, ntiles);
      TTS_LAUNCH_CHECK();
    }
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  return ki != keys;
}

void radix_sort_pairs(Allocator* al, uint64_t* keys, uint64_t* vals, uint64_t* ktmp, uint64_t* vtmp,
                      uint32_t n, int nbits, hipStream_t s) {
  if (radix_sort_pairs_pp(al, keys, vals, ktmp, vtmp, n, nbits, s)) {
    TTS_HIP(hipMemcpyAsync(keys, ktmp, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    TTS_HIP(hipMemcpyAsync(vals, vtmp, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace tts
