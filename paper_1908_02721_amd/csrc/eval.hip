// Sampled-entry evaluation of a TT (entry formula of Sec. 2.3) and its gradient.
//
// Forward: one group of LPE lanes per entry (LPE = 32 when every rank <= 32, else
// 64); the running row vector lives in LDS, lane j computes output j of
// v * G_k[:, i_k, :] reading row a of the slice (coalesced across lanes).
//
// Backward of L = sum_n gy[n] y_n:
//   dL/dG_k[a, i, b] = sum_{n : i_k^n = i} gy[n] * l_k^n[a] * r_{k+1}^n[b],
// l_k = G_0[i_0]...G_{k-1}[i_{k-1}], r_{k+1} = G_{k+1}[i_{k+1}]...G_{d-1}[i_{d-1}].
// The left and right partial products of every entry are stored once; then, per
// core, the entries are bucketed by i_k (stable radix sort), and every (i, chunk of
// the bucket) workgroup forms the small product (gy*L)^T R of its chunk in
// registers from LDS-staged rows.  Chunk partials are summed in a fixed order, so
// the gradient is bitwise reproducible.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "prim.hpp"

namespace tts {
namespace {

constexpr int NT = 256;
constexpr int RMAX = 256;

struct EvalDesc {
  int32_t d;
  int32_t n[TT_MAX_D];
  int32_t r[TT_MAX_D + 1];
  const void* core[TT_MAX_D];
  int64_t loff[TT_MAX_D + 1];  // offset (in elements per entry) of l_k, k = 1..d-1
  int64_t roff[TT_MAX_D + 1];  // offset of r_k, k = 1..d-1
  int64_t lsum, rsum;          // sum_{k=1}^{d-1} r_k
};

// Left chain: y[n] and (optionally) l_k for k = 1..d-1 into L[n * lsum + loff[k] + a].
template <typename T, int LPE>
__global__ __launch_bounds__(NT) void k_eval_left(EvalDesc ed, int64_t m, const int32_t* __restrict__ idx,
                                                  T* __restrict__ y, T* __restrict__ L, uint32_t* __restrict__ err) {
  constexpr int EPW = 64 / LPE;  // entries per wave
  __shared__ T buf[NT / 64][EPW][2][RMAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LPE, l = lane % LPE;
  T* va = buf[wv][sub][0];
  T* vb = buf[wv][sub][1];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (NT / 64) * EPW;
  for (int64_t n = (static_cast<int64_t>(blockIdx.x) * (NT / 64) + wv) * EPW + sub; n < m + (EPW - 1); n += stride) {
    const bool live = n < m;
    int32_t coord = 0;
    if (live && l < ed.d) coord = idx[n * ed.d + l];
    bool bad = live && l < ed.d && (coord < 0 || coord >= ed.n[l]);
    if (bad) atomicOr(err, 1u);
    if (l == 0) va[0] = T(1);
    __builtin_amdgcn_wave_barrier();
    for (int k = 0; k < ed.d; ++k) {
      const int ik = __shfl(coord, k, LPE);
      const int r0 = ed.r[k], r1 = ed.r[k + 1];
      const int ok = (ik >= 0 && ik < ed.n[k]) ? 1 : 0;
      const T* G = static_cast<const T*>(ed.core[k]) + static_cast<int64_t>(ok ? ik : 0) * r1;
      const int64_t rs = static_cast<int64_t>(ed.n[k]) * r1;
      for (int j = l; j < r1; j += LPE) {
        T acc = T(0);
        if (live)
          for (int a = 0; a < r0; ++a) acc = fma(va[a], G[a * rs + j], acc);
        vb[j] = acc;
        if (L && live && k < ed.d - 1) L[n * ed.lsum + ed.loff[k + 1] + j] = acc;
      }
      __builtin_amdgcn_wave_barrier();
      T* t = va;
      va = vb;
      vb = t;
    }
    if (live && l == 0) y[n] = va[0];
    __builtin_amdgcn_wave_barrier();
  }
}

// Right chain: r_k for k = d-1..1 into R[n * rsum + roff[k] + a]; r_k has length r[k].
template <typename T, int LPE>
__global__ __launch_bounds__(NT) void k_eval_right(EvalDesc ed, int64_t m, const int32_t* __restrict__ idx,
                                                   T* __restrict__ R) {
  constexpr int EPW = 64 / LPE;
  __shared__ T buf[NT / 64][EPW][2][RMAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LPE, l = lane % LPE;
  T* va = buf[wv][sub][0];
  T* vb = buf[wv][sub][1];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (NT / 64) * EPW;
  for (int64_t n = (static_cast<int64_t>(blockIdx.x) * (NT / 64) + wv) * EPW + sub; n < m + (EPW - 1); n += stride) {
    const bool live = n < m;
    int32_t coord = 0;
    if (live && l < ed.d) coord = idx[n * ed.d + l];
    if (l == 0) va[0] = T(1);
    __builtin_amdgcn_wave_barrier();
    for (int k = ed.d - 1; k >= 1; --k) {
      const int ik = __shfl(coord, k, LPE);
      const int r0 = ed.r[k], r1 = ed.r[k + 1];
      const int ok = (ik >= 0 && ik < ed.n[k]) ? 1 : 0;
      const T* G = static_cast<const T*>(ed.core[k]) + static_cast<int64_t>(ok ? ik : 0) * r1;
      const int64_t rs = static_cast<int64_t>(ed.n[k]) * r1;
      for (int a = l; a < r0; a += LPE) {
        T acc = T(0);
        if (live)
          for (int b = 0; b < r1; ++b) acc = fma(G[a * rs + b], va[b], acc);
        vb[a] = acc;
        if (live) R[n * ed.rsum + ed.roff[k] + a] = acc;
      }
      __builtin_amdgcn_wave_barrier();
      T* t = va;
      va = vb;
      vb = t;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(NT) void k_bucket_keys(const int32_t* __restrict__ idx, int64_t m, int d, int k,
                                                    uint64_t* __restrict__ key, uint64_t* __restrict__ val) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (n >= m) return;
  key[n] = static_cast<uint64_t>(idx[n * d + k]);
  val[n] = static_cast<uint64_t>(n);
}

__global__ __launch_bounds__(NT) void k_bucket_offsets(const uint64_t* __restrict__ skey, int64_t m, int nk,
                                                       int64_t* __restrict__ off) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i > nk) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (skey[mid] < static_cast<uint64_t>(i))
      lo = mid + 1;
    else
      hi = mid;
  }
  off[i] = lo;
}

// Partial gradient of core k for one (bucket i, chunk c, output tile) workgroup.
// Output tile: rows a in [a0, a0+64), columns b in [b0, b0+64); thread owns a 4x4
// register tile (rows ty + 16u, columns tx + 16v).
template <typename T, int KC>
__global__ __launch_bounds__(NT) void k_grad_partial(int r0, int r1, int nk, const uint64_t* __restrict__ perm,
                                                     const int64_t* __restrict__ off, const T* __restrict__ gy,
                                                     const T* __restrict__ L, int64_t lsum, int64_t loff,
                                                     const T* __restrict__ R, int64_t rsum, int64_t roff,
                                                     int64_t chunk, T* __restrict__ part) {
  __shared__ T Ls[KC][65];
  __shared__ T Rs[KC][65];
  const int i = blockIdx.x;
  const int c = blockIdx.y;
  const int tA = (r0 + 63) / 64;
  const int a0 = (blockIdx.z % tA) * 64, b0 = (blockIdx.z / tA) * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t beg = off[i] + static_cast<int64_t>(c) * chunk;
  const int64_t end = min(off[i + 1], beg + chunk);
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
  for (int64_t s0 = beg; s0 < end; s0 += KC) {
    const int cnt = static_cast<int>(min(static_cast<int64_t>(KC), end - s0));
    for (int e = threadIdx.x; e < KC * 64; e += NT) {
      const int t = e / 64, j = e % 64;
      T lv = T(0), rv = T(0);
      if (t < cnt) {
        const int64_t n = static_cast<int64_t>(perm[s0 + t]);
        const int a = a0 + j, b = b0 + j;
        if (a < r0) lv = (loff < 0 ? T(1) : L[n * lsum + loff + a]) * gy[n];
        if (b < r1) rv = (roff < 0 ? T(1) : R[n * rsum + roff + b]);
      }
      Ls[t][j] = lv;
      Rs[t][j] = rv;
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      T av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = Ls[t][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = Rs[t][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  // partial of chunk c, laid out like the core: [a][i][b]
  const int64_t csz = static_cast<int64_t>(r0) * nk * r1;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a = a0 + ty + 16 * u;
    if (a >= r0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = b0 + tx + 16 * v;
      if (b >= r1) continue;
      part[static_cast<int64_t>(c) * csz + (static_cast<int64_t>(a) * nk + i) * r1 + b] = acc[u][v];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_grad_reduce(int64_t csz, int nchunk, const T* __restrict__ part,
                                                    T* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= csz) return;
  T s = T(0);
  for (int c = 0; c < nchunk; ++c) s += part[static_cast<int64_t>(c) * csz + e];
  out[e] = s;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_zero(T* __restrict__ p, int64_t n) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e < n) p[e] = T(0);
}

tt_status check_args(int32_t d, const int64_t* dims, const int64_t* ranks, const void* const* cores, int32_t dtype,
                     int64_t m, const int32_t* idx, EvalDesc& ed) {
  if (d < 1 || d > TT_MAX_D || !dims || !ranks || !cores || m < 0 || (m > 0 && !idx)) return TT_ERR_ARG;
  if (dtype != TT_DTYPE_F64 && dtype != TT_DTYPE_F32) return TT_ERR_ARG;
  if (ranks[0] != 1 || ranks[d] != 1) return TT_ERR_ARG;
  ed = EvalDesc{};
  ed.d = d;
  for (int k = 0; k <= d; ++k) {
    if (ranks[k] < 1 || ranks[k] > RMAX) return TT_ERR_ARG;
    ed.r[k] = static_cast<int32_t>(ranks[k]);
  }
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1 || dims[k] > INT32_MAX || !cores[k]) return TT_ERR_ARG;
    ed.n[k] = static_cast<int32_t>(dims[k]);
    ed.core[k] = cores[k];
  }
  int64_t lo = 0;
  for (int k = 1; k < d; ++k) {
    ed.loff[k] = lo;
    ed.roff[k] = lo;
    lo += ranks[k];
  }
  ed.lsum = ed.rsum = lo;
  return TT_OK;
}

int max_rank_of(const EvalDesc& ed) {
  int r = 1;
  for (int k = 0; k <= ed.d; ++k) r = std::max(r, static_cast<int>(ed.r[k]));
  return r;
}

template <typename T>
void launch_left(const EvalDesc& ed, int64_t m, const int32_t* idx, T* y, T* L, uint32_t* err, hipStream_t s) {
  const bool narrow = max_rank_of(ed) <= 32 && ed.d <= 32;
  const int64_t per_block = (NT / 64) * (narrow ? 2 : 1);
  const int64_t blocks = std::min<int64_t>((m + per_block - 1) / per_block, 256 * 64);
  if (narrow)
    k_eval_left<T, 32><<<static_cast<unsigned>(std::max<int64_t>(blocks, 1)), NT, 0, s>>>(ed, m, idx, y, L, err);
  else
    k_eval_left<T, 64><<<static_cast<unsigned>(std::max<int64_t>(blocks, 1)), NT, 0, s>>>(ed, m, idx, y, L, err);
  TTS_LAUNCH_CHECK();
}

template <typename T>
void launch_right(const EvalDesc& ed, int64_t m, const int32_t* idx, T* R, hipStream_t s) {
  const bool narrow = max_rank_of(ed) <= 32 && ed.d <= 32;
  const int64_t per_block = (NT / 64) * (narrow ? 2 : 1);
  const int64_t blocks = std::min<int64_t>((m + per_block - 1) / per_block, 256 * 64);
  if (narrow)
    k_eval_right<T, 32><<<static_cast<unsigned>(std::max<int64_t>(blocks, 1)), NT, 0, s>>>(ed, m, idx, R);
  else
    k_eval_right<T, 64><<<static_cast<unsigned>(std::max<int64_t>(blocks, 1)), NT, 0, s>>>(ed, m, idx, R);
  TTS_LAUNCH_CHECK();
}

void* dalloc(size_t bytes, hipStream_t s) {
  void* p = nullptr;
  if (bytes == 0) return nullptr;
  if (hipMallocAsync(&p, bytes, s) != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(TT_ERR_NOMEM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

struct DevMem {
  hipStream_t s;
  std::vector<void*> ps;
  explicit DevMem(hipStream_t st) : s(st) {}
  template <class X>
  X* get(size_t n) {
    void* p = dalloc(n * sizeof(X), s);
    ps.push_back(p);
    return static_cast<X*>(p);
  }
  ~DevMem() {
    for (void* p : ps)
      if (p) (void)hipFreeAsync(p, s);
  }
};

template <typename T>
tt_status eval_impl(const EvalDesc& ed, int64_t m, const int32_t* idx, void* y_out, hipStream_t s) {
  DevMem mem(s);
  uint32_t* err = mem.get<uint32_t>(1);
  TTS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
  if (m > 0) launch_left<T>(ed, m, idx, static_cast<T*>(y_out), nullptr, err, s);
  uint32_t h = 0;
  TTS_HIP(hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s));
  TTS_HIP(hipStreamSynchronize(s));
  if (h) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  return TT_OK;
}

template <typename T>
tt_status grad_impl(const EvalDesc& ed, int64_t m, const int32_t* idx, const T* gy, void* const* grads,
                    hipStream_t s) {
  DevMem mem(s);
  Allocator al;
  al.stream = s;
  const int d = ed.d;
  uint32_t* err = mem.get<uint32_t>(1);
  TTS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
  T* y = mem.get<T>(std::max<int64_t>(m, 1));
  T* L = ed.lsum ? mem.get<T>(static_cast<size_t>(m) * ed.lsum + 1) : nullptr;
  T* R = ed.rsum ? mem.get<T>(static_cast<size_t>(m) * ed.rsum + 1) : nullptr;
  if (m > 0) {
    launch_left<T>(ed, m, idx, y, L, err, s);
    if (R) launch_right<T>(ed, m, idx, R, s);
  }
  uint32_t h = 0;
  TTS_HIP(hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s));
  TTS_HIP(hipStreamSynchronize(s));
  if (h) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  uint64_t* key = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* perm = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* kt = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* vt = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  constexpr int KC = sizeof(T) == 8 ? 64 : 128;
  for (int k = 0; k < d; ++k) {
    const int nk = ed.n[k], r0 = ed.r[k], r1 = ed.r[k + 1];
    const int64_t csz = static_cast<int64_t>(r0) * nk * r1;
    T* gout = static_cast<T*>(grads[k]);
    if (m == 0) {
      k_zero<T><<<grid_for(csz, NT), NT, 0, s>>>(gout, csz);
      TTS_LAUNCH_CHECK();
      continue;
    }
    k_bucket_keys<<<grid_for(m, NT), NT, 0, s>>>(idx, m, d, k, key, perm);
    TTS_LAUNCH_CHECK();
    int bits = 0;
    while (bits < 31 && (static_cast<int64_t>(nk) - 1) >> bits) ++bits;
    radix_sort_pairs(&al, key, perm, kt, vt, static_cast<uint32_t>(m), bits, s);
    int64_t* off = mem.get<int64_t>(nk + 1);
    k_bucket_offsets<<<grid_for(nk + 1, NT), NT, 0, s>>>(key, m, nk, off);
    TTS_LAUNCH_CHECK();
    std::vector<int64_t> hoff(nk + 1);
    TTS_HIP(hipMemcpyAsync(hoff.data(), off, sizeof(int64_t) * (nk + 1), hipMemcpyDeviceToHost, s));
    TTS_HIP(hipStreamSynchronize(s));
    int64_t maxb = 0;
    for (int i = 0; i < nk; ++i) maxb = std::max(maxb, hoff[i + 1] - hoff[i]);
    // chunks of the largest bucket: at most 512 per bucket, each a multiple of KC
    const int64_t iters = std::max<int64_t>(1, (maxb + KC * 512 - 1) / (KC * 512));
    const int64_t chunk = KC * iters;
    const int nchunk = static_cast<int>(std::max<int64_t>(1, (maxb + chunk - 1) / chunk));
    const int tiles = ((r0 + 63) / 64) * ((r1 + 63) / 64);
    T* part = mem.get<T>(static_cast<size_t>(nchunk) * csz);
    const int64_t lo = (k >= 1) ? ed.loff[k] : -1;              // l_k (k >= 1); l_0 = 1
    const int64_t ro = (k + 1 <= d - 1) ? ed.roff[k + 1] : -1;  // r_{k+1}; r_d = 1
    k_grad_partial<T, KC><<<dim3(nk, nchunk, tiles), NT, 0, s>>>(r0, r1, nk, perm, off, gy, L, ed.lsum, lo, R,
                                                                 ed.rsum, ro, chunk, part);
    TTS_LAUNCH_CHECK();
    k_grad_reduce<T><<<grid_for(csz, NT), NT, 0, s>>>(csz, nchunk, part, gout);
    TTS_LAUNCH_CHECK();
  }
  TTS_HIP(hipStreamSynchronize(s));
  return TT_OK;
}

}  // namespace
}  // namespace tts

using namespace tts;

extern "C" tt_status tt_eval_entries(int32_t d, const int64_t* dims, const int64_t* ranks, const void* const* cores,
                                     int32_t dtype, int64_t m, const int32_t* idx, void* y_out, void* stream) {
  EvalDesc ed;
  tt_status st = check_args(d, dims, ranks, cores, dtype, m, idx, ed);
  if (st != TT_OK) return st;
  if (m > 0 && !y_out) return TT_ERR_ARG;
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dtype == TT_DTYPE_F64 ? eval_impl<double>(ed, m, idx, y_out, s) : eval_impl<float>(ed, m, idx, y_out, s);
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}

extern "C" tt_status tt_eval_entries_backward(int32_t d, const int64_t* dims, const int64_t* ranks,
                                              const void* const* cores, int32_t dtype, int64_t m, const int32_t* idx,
                                              const void* grad_y, void* const* grad_cores, void* stream) {
  EvalDesc ed;
  tt_status st = check_args(d, dims, ranks, cores, dtype, m, idx, ed);
  if (st != TT_OK) return st;
  if ((m > 0 && !grad_y) || !grad_cores) return TT_ERR_ARG;
  for (int k = 0; k < d; ++k)
    if (!grad_cores[k]) return TT_ERR_ARG;
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dtype == TT_DTYPE_F64
               ? grad_impl<double>(ed, m, idx, static_cast<const double*>(grad_y), grad_cores, s)
               : grad_impl<float>(ed, m, idx, static_cast<const float*>(grad_y), grad_cores, s);
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}
