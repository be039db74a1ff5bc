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
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include <mutex>

#include "common.hpp"
#include "prim.hpp"

// Scratch of the allocation-free evaluation (tt_eval_entries_noalloc): word 0 is the
// coordinate-check flag of the per-entry kernel.  One copy per device, held until
// the process ends.  Host code never passes this name to a kernel or a copy: it
// takes the device address from hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) uint32_t scratch[64];

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

// Bucket keys of the depth-t trie nodes: key = mode index, value = node index in the
// low 32 bits and its parent's index in the high 32 bits (so that consumers reach
// the parent vector with one load fewer).
__global__ __launch_bounds__(NT) void k_bucket_keys_u32(const uint32_t* __restrict__ coord,
                                                        const uint32_t* __restrict__ parent, int64_t m,
                                                        uint64_t* __restrict__ key, uint64_t* __restrict__ val) {
  const int64_t n = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (n >= m) return;
  key[n] = static_cast<uint64_t>(coord[n]);
  val[n] = (static_cast<uint64_t>(parent[n]) << 32) | static_cast<uint64_t>(n);
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


// out[a][i][b] = sum over the chunks c of bucket i of part[c][a][b], in chunk order
// (four interleaved partial sums keep four loads in flight; the order is fixed).
template <typename T>
__global__ __launch_bounds__(NT) void k_grad_reduce(int r0, int nk, int r1, const int64_t* __restrict__ cstart,
                                                    const T* __restrict__ part, T* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  const int64_t csz = static_cast<int64_t>(r0) * nk * r1;
  if (e >= csz) return;
  const int b = static_cast<int>(e % r1);
  const int i = static_cast<int>((e / r1) % nk);
  const int a = static_cast<int>(e / (static_cast<int64_t>(r1) * nk));
  const int64_t O = static_cast<int64_t>(r0) * r1;
  const T* p = part + a * r1 + b;
  const int64_t c1 = cstart[i + 1];
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
  int64_t c = cstart[i];
  for (; c + 3 < c1; c += 4) {
    s0 += p[c * O];
    s1 += p[(c + 1) * O];
    s2 += p[(c + 2) * O];
    s3 += p[(c + 3) * O];
  }
  for (; c < c1; ++c) s0 += p[c * O];
  out[e] = (s0 + s1) + (s2 + s3);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_zero(T* __restrict__ p, int64_t n) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e < n) p[e] = T(0);
}

tt_status check_core_args(int32_t d, const int64_t* dims, const int64_t* ranks, const void* const* cores,
                          int32_t dtype, EvalDesc& ed) {
  auto bad = [](const char* why) {
    set_last_error(why);
    return TT_ERR_ARG;
  };
  if (d < 1 || d > TT_MAX_D) return bad("d must be in [1, TT_MAX_D]");
  if (!dims || !ranks || !cores) return bad("dims, ranks and cores must not be NULL");
  if (dtype != TT_DTYPE_F64 && dtype != TT_DTYPE_F32) return bad("unknown dtype");
  if (ranks[0] != 1 || ranks[d] != 1) return bad("ranks[0] and ranks[d] must be 1");
  ed = EvalDesc{};
  ed.d = d;
  for (int k = 0; k <= d; ++k) {
    if (ranks[k] < 1 || ranks[k] > RMAX) return bad("every rank must be in [1, 256]");
    ed.r[k] = static_cast<int32_t>(ranks[k]);
  }
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1 || dims[k] > INT32_MAX) return bad("every mode size must be in [1, 2^31 - 1]");
    if (!cores[k]) return bad("a core pointer is NULL");
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

tt_status check_args(int32_t d, const int64_t* dims, const int64_t* ranks, const void* const* cores, int32_t dtype,
                     int64_t m, const int32_t* idx, EvalDesc& ed) {
  if (m < 0 || (m > 0 && !idx)) {
    set_last_error("m must be >= 0 and idx non-NULL when m > 0");
    return TT_ERR_ARG;
  }
  return check_core_args(d, dims, ranks, cores, dtype, ed);
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

struct DevMem {
  hipStream_t s;
  std::vector<std::pair<void*, size_t>> ps;
  explicit DevMem(hipStream_t st) : s(st) {}
  template <class X>
  X* get(size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(X);
    void* p = cached_alloc(bytes, s);
    if (!p) fail(TT_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    ps.emplace_back(p, bytes);
    return static_cast<X*>(p);
  }
  ~DevMem() {
    for (auto& pb : ps) cached_free(pb.first, pb.second, s);
  }
};

// ---------------------------------------------------------------------------
// Prefix-trie evaluation.  Entries are sorted by their coordinates (mode 0 most
// significant); the distinct prefixes (i_0..i_{t-1}) of depth t are the nodes of a
// trie whose depth-d nodes are the distinct coordinates.  Left products are
// computed once per node (top-down), the "up" vectors
//   U_t[q] = sum over leaves n below q of gy_n * G_t[i_t^n] ... G_{d-1}[i_{d-1}^n]
// once per node (bottom-up), and
//   dL/dG_t[a, i, b] = sum over children c (depth t+1, i_t(c) = i) of L_t[parent(c)][a] U_{t+1}[c][b].
// The work is sum_t P_t r_{t-1} r_t instead of m sum_t r_{t-1} r_t.
// ---------------------------------------------------------------------------
struct TrieGeom {
  int32_t d;
  uint32_t bits[TT_MAX_D];
  uint32_t off[TT_MAX_D];  // mode 0 most significant: off[k] = sum_{j>k} bits[j]
  int32_t n[TT_MAX_D];
};

__global__ __launch_bounds__(NT) void k_tri_keys(const int32_t* __restrict__ idx, int64_t m, TrieGeom g,
                                                 uint64_t* __restrict__ key, uint64_t* __restrict__ val,
                                                 uint32_t* __restrict__ err) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= m) return;
  uint64_t k = 0;
  bool bad = false;
  for (int j = 0; j < g.d; ++j) {
    const int32_t c = idx[e * g.d + j];
    bad |= (c < 0) || (c >= g.n[j]);
    k |= static_cast<uint64_t>(static_cast<uint32_t>(c)) << g.off[j];
  }
  if (bad) atomicOr(err, 1u);
  key[e] = bad ? 0ull : k;
  val[e] = static_cast<uint64_t>(e);
}

__global__ __launch_bounds__(NT) void k_tri_flags(const uint64_t* __restrict__ key, int64_t m, int sh,
                                                  uint32_t* __restrict__ flag) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= m) return;
  flag[e] = (e == 0 || (key[e] >> sh) != (key[e - 1] >> sh)) ? 1u : 0u;
}

__global__ __launch_bounds__(NT) void k_tri_nodes(const uint64_t* __restrict__ key, const uint32_t* __restrict__ flag,
                                                  const uint32_t* __restrict__ pos, int64_t m,
                                                  const uint32_t* __restrict__ prev_id, int csh, uint64_t cmask,
                                                  uint32_t* __restrict__ cur_id, uint32_t* __restrict__ parent,
                                                  uint32_t* __restrict__ coord, uint32_t* __restrict__ start) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= m) return;
  const uint32_t id = pos[e] + flag[e] - 1u;
  cur_id[e] = id;
  if (flag[e]) {
    parent[id] = prev_id ? prev_id[e] : 0u;
    coord[id] = static_cast<uint32_t>((key[e] >> csh) & cmask);
    if (start) start[id] = static_cast<uint32_t>(e);
  }
}

__global__ __launch_bounds__(NT) void k_tri_child_ranges(const uint32_t* __restrict__ parent, int64_t pc,
                                                         int64_t pq, uint32_t* __restrict__ cbeg) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (c == 0) cbeg[pq] = static_cast<uint32_t>(pc);
  if (c >= pc) return;
  if (c == 0 || parent[c] != parent[c - 1]) cbeg[parent[c]] = static_cast<uint32_t>(c);
}

// Matrix-core tile step for the evaluation kernels: v_mfma_f64_16x16x4 (FP64) or
// v_mfma_f32_16x16x4_f32 (FP32).  Operands: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator register v of lane l holds row row(l, v), column l%16
// (the two instructions order their accumulator rows differently).
typedef double evd4 __attribute__((ext_vector_type(4)));
typedef float evf4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef evd4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <>
struct Mfma<float> {
  typedef evf4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// One chunk of a bucket: nodes [beg, beg + cnt) of the bucket order, all with last
// mode index i.
struct ChunkDesc {
  int64_t beg;
  uint32_t i, cnt;
};
struct ChunkList {
  const ChunkDesc* d = nullptr;
  int64_t n = 0;
  const int64_t* cstart = nullptr;
};

// Bucketed row-times-slice product over the nodes of one trie depth grouped by their
// last mode index: workgroup (chunk, tile) takes the chunk's NB nodes q (index i),
// gathers their input rows src[parent(q)] (forward; src[q] when parent is null),
// multiplies them by the r0 x r1 slice S_i (S_i[a][b] = G[i*sI + a*sK + b], staged
// in LDS 32 rows at a time) and writes dst[q][b0:b0+TW]: a small gather-GEMM-scatter
// on the matrix cores, each of the 4 waves owning a 32 x 32 block of the NB x TW tile
// as 2 x 2 MFMA blocks (NB = 64: TW = 64; NB = 128 for slices at most 32 wide:
// TW = 32).  Only non-empty chunks are launched.  Forward: S_i = G[:, i, :].  Up
// pass: S_i = G[:, i, :]^T, rows = the children's up vectors.
template <typename T, int NB>
__global__ __launch_bounds__(NT) void k_tri_fwd_bucket_mfma(int r0, int r1, int64_t sK, int64_t sI,
                                                            const ChunkDesc* __restrict__ chunks,
                                                            const uint64_t* __restrict__ perm,
                                                            const uint32_t* __restrict__ parent,
                                                            const T* __restrict__ Lprev, const T* __restrict__ G,
                                                            T* __restrict__ Lcur) {
  static_assert(NB == 64 || NB == 128, "64- or 128-node chunks");
  constexpr int TW = NB == 64 ? 64 : 32;
  constexpr int AK = 32;
  __shared__ T Vs[AK][NB + 1];
  __shared__ T Ss[AK][TW + 1];
  __shared__ uint32_t qid[NB], pid[NB];
  const ChunkDesc cd = chunks[blockIdx.x];
  const int i = static_cast<int>(cd.i);
  const int64_t beg = cd.beg;
  const int cnt = static_cast<int>(cd.cnt);
  const int b0 = blockIdx.y * TW;
  for (int e = threadIdx.x; e < NB; e += NT) {
    const uint64_t pv = (e < cnt) ? perm[beg + e] : 0ull;
    const uint32_t q = static_cast<uint32_t>(pv);
    qid[e] = q;
    pid[e] = parent ? static_cast<uint32_t>(pv >> 32) : q;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = NB == 64 ? (w & 1) * 32 : w * 32, wn = NB == 64 ? (w >> 1) * 32 : 0;
  const int li = lane & 15, lk = lane >> 4;
  typename Mfma<T>::acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::zero();
  // 16 x 16 blocks that lie wholly outside the nodes or the columns are skipped
  // (uniform per wave): skinny slices (r1 <= 32) and short last chunks
  const bool act0 = wm < cnt, act1 = wm + 16 < cnt;
  const bool actc0 = b0 + wn < r1, actc1 = b0 + wn + 16 < r1;
  const T* Gi = G + static_cast<int64_t>(i) * sI;
  // staging: all loads of a K-stage in flight together (clamped addresses, masked
  // afterwards); the next stage's loads are issued before this stage's MFMA
  constexpr int PV = AK * NB / NT, PS = AK * TW / NT;
  T vv[PV], sv[PS];
  auto load_stage = [&](int a0) {
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      const int a = e % AK, nn = e / AK;
      const bool ok = nn < cnt && a0 + a < r0;
      vv[u] = Lprev[ok ? static_cast<int64_t>(pid[nn]) * r0 + a0 + a : 0];
    }
#pragma unroll
    for (int u = 0; u < PS; ++u) {
      const int e = threadIdx.x + u * NT;
      const int b = e % TW, a = e / TW;
      const bool ok = a0 + a < r0 && b0 + b < r1;
      sv[u] = Gi[ok ? (a0 + a) * sK + b0 + b : 0];
    }
  };
  load_stage(0);
  for (int a0 = 0; a0 < r0; a0 += AK) {
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      const int a = e % AK, nn = e / AK;
      Vs[a][nn] = (nn < cnt && a0 + a < r0) ? vv[u] : T(0);
    }
#pragma unroll
    for (int u = 0; u < PS; ++u) {
      const int e = threadIdx.x + u * NT;
      const int b = e % TW, a = e / TW;
      Ss[a][b] = (a0 + a < r0 && b0 + b < r1) ? sv[u] : T(0);
    }
    __syncthreads();
    if (a0 + AK < r0) load_stage(a0 + AK);
    const int kk = ((min(AK, r0 - a0) + 3) / 4) * 4;
    if (act0 && actc0) {
      for (int k4 = 0; k4 < kk; k4 += 4) {
        const T x0 = Vs[k4 + lk][wm + li], x1 = Vs[k4 + lk][wm + 16 + li];
        const T y0 = Ss[k4 + lk][wn + li], y1 = Ss[k4 + lk][wn + 16 + li];
        acc[0][0] = Mfma<T>::mma(x0, y0, acc[0][0]);
        if (actc1) acc[0][1] = Mfma<T>::mma(x0, y1, acc[0][1]);
        if (act1) acc[1][0] = Mfma<T>::mma(x1, y0, acc[1][0]);
        if (act1 && actc1) acc[1][1] = Mfma<T>::mma(x1, y1, acc[1][1]);
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
        const int nn = wm + 16 * x + Mfma<T>::row(lane, v);
        const int b = b0 + wn + 16 * y + li;
        if (nn < cnt && b < r1) Lcur[static_cast<int64_t>(qid[nn]) * r1 + b] = acc[x][y][v];
      }
}

// Partial gradient slice of one (bucket, chunk, tile): sum over the chunk's entries t
// (all with mode index i) of Lrow_t[a] * Rrow_t[b] (Lrow scaled by grad_y when given),
// a 64 x 64 tile of MFMA blocks contracting over the entries staged KC at a time;
// written to part[chunk] laid out like the core, [a][i][b].
template <typename T, int KC>
__global__ __launch_bounds__(NT) void k_grad_partial_mfma(int r0, int r1, const ChunkDesc* __restrict__ chunks,
                                                          const uint64_t* __restrict__ perm, const T* __restrict__ gy,
                                                          const T* __restrict__ L, int64_t lsum, int64_t loff,
                                                          const T* __restrict__ R, int64_t rsum, int64_t roff,
                                                          T* __restrict__ part, const uint32_t* __restrict__ lidx) {
  __shared__ T Ls[KC][65];
  __shared__ T Rs[KC][65];
  const ChunkDesc cd = chunks[blockIdx.x];
  const int tA = (r0 + 63) / 64;
  const int a0 = (blockIdx.y % tA) * 64, b0 = (blockIdx.y / tA) * 64;
  const int64_t beg = cd.beg;
  const int64_t end = beg + cd.cnt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // 16 x 16 blocks wholly outside r0 x r1 are skipped (uniform per wave)
  const bool act0 = a0 + wm < r0, act1 = a0 + wm + 16 < r0;
  const bool actc0 = b0 + wn < r1, actc1 = b0 + wn + 16 < r1;
  typename Mfma<T>::acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::zero();
  // staging: thread (tb, j) loads column j of entries tb, tb + 4, ...; all index loads
  // of a stage are issued before its data loads (clamped addresses, masked
  // afterwards, no branches between them), so a stage costs two memory round trips
  // rather than two per entry
  constexpr int PER = KC * 64 / NT;
  const int j = threadIdx.x & 63, tb = threadIdx.x >> 6;
  const int a = a0 + j, b = b0 + j;
  for (int64_t s0 = beg; s0 < end; s0 += KC) {
    const int cnt = static_cast<int>(min(static_cast<int64_t>(KC), end - s0));
    uint64_t pv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = tb + 4 * u;
      pv[u] = (t < cnt) ? perm[s0 + t] : 0ull;
    }
    T lv[PER], rv[PER];
    if (loff >= 0) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int64_t nl =
            lidx ? static_cast<int64_t>(pv[u] >> 32) : static_cast<int64_t>(static_cast<uint32_t>(pv[u]));
        lv[u] = L[(a < r0) ? nl * lsum + loff + a : 0];
      }
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) lv[u] = T(1);
    }
    if (roff >= 0) {
#pragma unroll
      for (int u = 0; u < PER; ++u)
        rv[u] = R[(b < r1) ? static_cast<int64_t>(static_cast<uint32_t>(pv[u])) * rsum + roff + b : 0];
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) rv[u] = T(1);
    }
    if (gy) {
#pragma unroll
      for (int u = 0; u < PER; ++u) lv[u] *= gy[static_cast<uint32_t>(pv[u])];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const bool live = tb + 4 * u < cnt;
      Ls[tb + 4 * u][j] = (live && a < r0) ? lv[u] : T(0);
      Rs[tb + 4 * u][j] = (live && b < r1) ? rv[u] : T(0);
    }
    __syncthreads();
    const int kk = ((cnt + 3) / 4) * 4;
    if (act0 && actc0) {
      for (int k4 = 0; k4 < kk; k4 += 4) {
        const T x0 = Ls[k4 + lk][wm + li], x1 = Ls[k4 + lk][wm + 16 + li];
        const T y0 = Rs[k4 + lk][wn + li], y1 = Rs[k4 + lk][wn + 16 + li];
        acc[0][0] = Mfma<T>::mma(x0, y0, acc[0][0]);
        if (actc1) acc[0][1] = Mfma<T>::mma(x0, y1, acc[0][1]);
        if (act1) acc[1][0] = Mfma<T>::mma(x1, y0, acc[1][0]);
        if (act1 && actc1) acc[1][1] = Mfma<T>::mma(x1, y1, acc[1][1]);
      }
    }
    __syncthreads();
  }
  T* pc = part + static_cast<int64_t>(blockIdx.x) * r0 * r1;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = a0 + wm + 16 * x + Mfma<T>::row(lane, v);
        const int b = b0 + wn + 16 * y + li;
        if (a < r0 && b < r1) pc[a * r1 + b] = acc[x][y][v];
      }
}


// Forward for narrow outputs (r1 < 16): one thread per (node, output column); the
// node's parent vector is read from global memory, the slice column from LDS.
template <typename T>
__global__ __launch_bounds__(NT) void k_tri_fwd_narrow(int r0, int r1, int64_t sK, int64_t sI,
                                                       const uint64_t* __restrict__ perm,
                                                       const int64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ parent,
                                                       const T* __restrict__ Lprev, const T* __restrict__ G,
                                                       T* __restrict__ Lcur) {
  __shared__ T Ss[RMAX * 16];
  const int i = blockIdx.x;
  const int per = NT / r1;  // nodes per pass
  const int64_t beg = off[i] + static_cast<int64_t>(blockIdx.y) * per * 8;
  const int64_t end = min(off[i + 1], beg + static_cast<int64_t>(per) * 8);
  if (beg >= end) return;
  const T* Gi = G + static_cast<int64_t>(i) * sI;
  for (int e = threadIdx.x; e < r0 * r1; e += NT) {
    const int a = e / r1, b = e % r1;
    Ss[a * r1 + b] = Gi[a * sK + b];
  }
  __syncthreads();
  const int b = threadIdx.x % r1, nn = threadIdx.x / r1;
  if (nn >= per) return;
  for (int64_t t = beg + nn; t < end; t += per) {
    const uint64_t pv = perm[t];
    const int64_t q = static_cast<int64_t>(static_cast<uint32_t>(pv));
    const T* v = Lprev + (parent ? static_cast<int64_t>(pv >> 32) : q) * r0;
    T acc = T(0);
    for (int a = 0; a < r0; ++a) acc = fma(v[a], Ss[a * r1 + b], acc);
    Lcur[q * r1 + b] = acc;
  }
}

// Gradient partial for small outputs (r0 * r1 <= 256): thread t owns output
// o = t % O for the entries t / O, t / O + NT / O, ... of its chunk; the per-thread
// sums are then added in a fixed order.
template <typename T>
__global__ __launch_bounds__(NT) void k_grad_small(int r0, int r1, const ChunkDesc* __restrict__ chunks,
                                                   const uint64_t* __restrict__ perm, const T* __restrict__ L,
                                                   int64_t loff, const T* __restrict__ R,
                                                   const uint32_t* __restrict__ lidx, T* __restrict__ part) {
  __shared__ T red[NT];
  const ChunkDesc cd = chunks[blockIdx.x];
  const int O = r0 * r1;
  const int lanes = NT / O;
  const int o = threadIdx.x % O, l = threadIdx.x / O;
  const int a = o / r1, b = o % r1;
  const int64_t beg = cd.beg;
  const int64_t end = beg + cd.cnt;
  T acc = T(0);
  if (l < lanes) {
    // four entries per iteration so that their loads overlap
    int64_t t = beg + l;
    for (; t + 3 * lanes < end; t += 4 * lanes) {
      uint64_t pv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pv[u] = perm[t + u * lanes];
      T lv[4], rv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        lv[u] = (loff < 0) ? T(1) : L[static_cast<int64_t>(pv[u] >> 32) * r0 + a];
        rv[u] = R[static_cast<int64_t>(static_cast<uint32_t>(pv[u])) * r1 + b];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(lv[u], rv[u], acc);
    }
    for (; t < end; t += lanes) {
      const uint64_t pv = perm[t];
      const int64_t n = static_cast<int64_t>(static_cast<uint32_t>(pv));
      const T lv = (loff < 0) ? T(1) : L[static_cast<int64_t>(pv >> 32) * r0 + a];
      acc = fma(lv, R[n * r1 + b], acc);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < O) {
    T s2 = T(0);
    for (int ll = 0; ll < lanes; ++ll) s2 += red[ll * O + threadIdx.x];
    part[static_cast<int64_t>(blockIdx.x) * O + a * r1 + b] = s2;
  }
}

// Up vectors of depth-t nodes from their children (depth t+1).  GT is the core
// with its slices transposed: GT[(i * r1 + b) * r0 + a] = G[a, i, b].
template <typename T, int LPE>
__global__ __launch_bounds__(NT) void k_tri_up(int64_t P, const uint32_t* __restrict__ cbeg,
                                               const uint32_t* __restrict__ ccoord, const T* __restrict__ Unext,
                                               int r0, int r1, const T* __restrict__ GT, T* __restrict__ Ucur) {
  constexpr int EPW = 64 / LPE;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LPE, l = lane % LPE;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (NT / 64) * EPW;
  for (int64_t q = (static_cast<int64_t>(blockIdx.x) * (NT / 64) + wv) * EPW + sub; q < P; q += stride) {
    const int64_t c0 = cbeg[q], c1 = cbeg[q + 1];
    T acc[RMAX / LPE];
#pragma unroll
    for (int s2 = 0; s2 < RMAX / LPE; ++s2) acc[s2] = T(0);
    // children four at a time: their indices and up vectors (r1 <= 4) are loaded
    // together, then the slice entries; clamped addresses, masked contributions
    for (int64_t c = c0; c < c1; c += 4) {
      uint32_t co[4];
      T uv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t cc = (c + u < c1) ? c + u : c;
        co[u] = ccoord[cc];
#pragma unroll
        for (int b = 0; b < 4; ++b) uv[u][b] = (b < r1 && c + u < c1) ? Unext[cc * r1 + b] : T(0);
      }
#pragma unroll
      for (int s2 = 0; s2 < RMAX / LPE; ++s2) {
        const int a = l + s2 * LPE;
        if (a < r0) {
          T x = acc[s2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const T* base = GT + static_cast<int64_t>(co[u]) * r1 * r0 + a;
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (b < r1) x = fma(base[b * r0], uv[u][b], x);
          }
          acc[s2] = x;
        }
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < RMAX / LPE; ++s2) {
      const int a = l + s2 * LPE;
      if (a < r0) Ucur[q * r0 + a] = acc[s2];
    }
  }
}

// Up vectors as k_tri_up, for a core that fits in LDS: workgroup per QB consecutive
// parents, whose children are consecutive too (trie order).  The transposed core, the
// parents' child ranges and the children's indices and up vectors (r1 <= 4) are
// staged in LDS with coalesced loads (the children in pieces of UP_CH), then thread
// (q, a) sums over the children of q from LDS and the rows are stored coalesced.
constexpr int UP_CH = 512;
template <typename T>
__global__ __launch_bounds__(NT) void k_tri_up_seg(int64_t P, int QB, const uint32_t* __restrict__ cbeg,
                                                   const uint32_t* __restrict__ ccoord, const T* __restrict__ Unext,
                                                   int r0, int r1, int nk, const T* __restrict__ GT,
                                                   T* __restrict__ Ucur) {
  extern __shared__ unsigned char up_sm[];
  T* gs = reinterpret_cast<T*>(up_sm);                       // r0 * nk * r1
  const int csz = r0 * nk * r1;
  T* su = gs + csz;                                          // UP_CH * 4
  uint32_t* sco = reinterpret_cast<uint32_t*>(su + UP_CH * 4);  // UP_CH
  uint32_t* scb = sco + UP_CH;                               // QB + 1
  const int64_t q0 = static_cast<int64_t>(blockIdx.x) * QB;
  const int nq = static_cast<int>(min(static_cast<int64_t>(QB), P - q0));
  for (int e = threadIdx.x; e <= nq; e += NT) scb[e] = cbeg[q0 + e];
  for (int e = threadIdx.x; e < csz; e += NT) gs[e] = GT[e];
  __syncthreads();
  const uint32_t clo = scb[0], chi = scb[nq];
  constexpr int PT = 8;  // (parent, row) pairs per thread: QB * r0 <= PT * NT
  T acc[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) acc[j] = T(0);
  for (uint32_t p0 = clo; p0 < chi; p0 += UP_CH) {
    const int pc = static_cast<int>(min(static_cast<uint32_t>(UP_CH), chi - p0));
    if (p0 != clo) __syncthreads();  // the previous piece is no longer read
    for (int e = threadIdx.x; e < pc; e += NT) sco[e] = ccoord[p0 + e];
    for (int e = threadIdx.x; e < pc * r1; e += NT) su[e] = Unext[static_cast<int64_t>(p0) * r1 + e];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int e = threadIdx.x + j * NT;
      const int qq = e / r0, a = e % r0;
      if (qq < nq) {
        const uint32_t c0 = max(scb[qq], p0), c1 = min(scb[qq + 1], p0 + static_cast<uint32_t>(pc));
        T x = acc[j];
        for (uint32_t c = c0; c < c1; ++c) {
          const int cl = static_cast<int>(c - p0);
          const T* g = gs + static_cast<int64_t>(sco[cl]) * r1 * r0 + a;
          for (int b = 0; b < r1; ++b) x = fma(g[b * r0], su[cl * r1 + b], x);
        }
        acc[j] = x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int e = threadIdx.x + j * NT;
    if (e / r0 < nq) Ucur[q0 * r0 + e] = acc[j];
  }
}

// Forward of a depth whose r1 is small, in trie order: one thread per (node, b),
// L[q][b] = sum_a Lprev[parent(q)][a] G[a][coord(q)][b], the whole core staged in
// LDS.  Siblings are adjacent in trie order, so their shared parent vector is read
// once from memory and then from cache (bucket order would scatter them).
template <typename T>
__global__ __launch_bounds__(NT) void k_tri_fwd_trie(int64_t P, int r0, int r1, int nk,
                                                     const uint32_t* __restrict__ parent,
                                                     const uint32_t* __restrict__ coord, const T* __restrict__ Lprev,
                                                     const T* __restrict__ G, T* __restrict__ Lcur) {
  extern __shared__ unsigned char tri_smem[];
  T* Gs = reinterpret_cast<T*>(tri_smem);
  const int csz = r0 * nk * r1;
  for (int e = threadIdx.x; e < csz; e += NT) Gs[e] = G[e];
  __syncthreads();
  const int64_t items = P * r1;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; e < items;
       e += static_cast<int64_t>(gridDim.x) * NT) {
    const int64_t q = e / r1;
    const int b = static_cast<int>(e - q * r1);
    const T* v = Lprev + static_cast<int64_t>(parent[q]) * r0;
    const T* g = Gs + static_cast<int64_t>(coord[q]) * r1 + b;
    const int64_t ga = static_cast<int64_t>(nk) * r1;
    T acc = T(0);
#pragma unroll 8
    for (int a = 0; a < r0; ++a) acc = fma(v[a], g[a * ga], acc);
    Lcur[e] = acc;
  }
}

// Up vector of each parent as the fixed-order sum of its children's products:
// U[q][a] = sum_{c in [cbeg[q], cbeg[q+1])} V[c][a].  One thread per (q, a).
template <typename T>
__global__ __launch_bounds__(NT) void k_tri_segsum(int64_t P, int r0, const uint32_t* __restrict__ cbeg,
                                                   const T* __restrict__ V, T* __restrict__ U) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= P * r0) return;
  const int64_t q = e / r0;
  const int a = static_cast<int>(e - q * r0);
  const int64_t c0 = cbeg[q], c1 = cbeg[q + 1];
  T acc = T(0);
  int64_t c = c0;
  for (; c + 3 < c1; c += 4) {  // four loads in flight, summed in child order
    const T v0 = V[c * r0 + a], v1 = V[(c + 1) * r0 + a], v2 = V[(c + 2) * r0 + a], v3 = V[(c + 3) * r0 + a];
    acc += v0;
    acc += v1;
    acc += v2;
    acc += v3;
  }
  for (; c < c1; ++c) acc += V[c * r0 + a];
  U[e] = acc;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_tri_leaf_up(int64_t P, const uint32_t* __restrict__ start, int64_t m,
                                                    const uint64_t* __restrict__ perm, const T* __restrict__ gy,
                                                    T* __restrict__ U) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (q >= P) return;
  const int64_t e1 = (q + 1 < P) ? static_cast<int64_t>(start[q + 1]) : m;
  T s = T(0);
  for (int64_t e = start[q]; e < e1; ++e) s += gy[perm[e]];
  U[q] = s;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_tri_out(int64_t m, const uint32_t* __restrict__ leaf,
                                                const uint64_t* __restrict__ perm, const T* __restrict__ Ld,
                                                T* __restrict__ y) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= m) return;
  y[perm[e]] = Ld[leaf[e]];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_slice_transpose(const T* __restrict__ G, int r0, int nk, int r1,
                                                        T* __restrict__ GT) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  const int64_t tot = static_cast<int64_t>(r0) * nk * r1;
  if (e >= tot) return;
  const int b = static_cast<int>(e % r1);
  const int i = static_cast<int>((e / r1) % nk);
  const int a = static_cast<int>(e / (static_cast<int64_t>(r1) * nk));
  GT[(static_cast<int64_t>(i) * r1 + b) * r0 + a] = G[e];
}

// The same transpose through 32 x 32 LDS tiles of one slice i: the tile of G[a][i][b]
// is read along b and written along a, so both sides are coalesced.  blockIdx.x =
// (i * ta + ta_index) * tb + tb_index with ta = ceil(r0 / 32), tb = ceil(r1 / 32).
template <typename T>
__global__ __launch_bounds__(256) void k_slice_transpose_tiled(const T* __restrict__ G, int r0, int nk, int r1,
                                                               int ta, int tb, T* __restrict__ GT) {
  __shared__ T tile[32][33];
  const int64_t blk = blockIdx.x;
  const int jb = static_cast<int>(blk % tb);
  const int64_t q = blk / tb;
  const int ja = static_cast<int>(q % ta);
  const int i = static_cast<int>(q / ta);
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8 threads
  const int a0 = ja * 32, b0 = jb * 32;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a = a0 + ty + 8 * u, b = b0 + tx;
    if (a < r0 && b < r1) tile[ty + 8 * u][tx] = G[(static_cast<int64_t>(a) * nk + i) * r1 + b];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int b = b0 + ty + 8 * u, a = a0 + tx;
    if (a < r0 && b < r1) GT[(static_cast<int64_t>(i) * r1 + b) * r0 + a] = tile[tx][ty + 8 * u];
  }
}

template <typename T>
__global__ void k_one(T* p) {
  *p = T(1);
}

struct Trie {
  int64_t m = 0;
  std::vector<uint64_t*> bperm;           // per depth t = 1..d: nodes sorted by their last index
  std::vector<int64_t*> boff;             // bucket offsets (n_{t-1} + 1)
  std::vector<int64_t> bmax;              // largest bucket
  std::vector<int64_t> P;                 // P[t], t = 0..d (P[0] = 1)
  std::vector<uint32_t*> parent, coord;   // per depth t = 1..d
  uint32_t* leaf = nullptr;               // per sorted entry: depth-d node
  uint32_t* start = nullptr;              // per depth-d node: first sorted entry
  uint64_t* perm = nullptr;               // sorted position -> entry
  std::vector<std::vector<int64_t>> hoff; // host copy of boff
  DevMem* owner = nullptr;                // memory of the chunk lists, built on first use
  mutable std::map<std::pair<int, int64_t>, ChunkList> chunks;
};

// Non-empty chunks of at most `cl` entries of every bucket, bucket by bucket: d[c]
// for c < n, the chunks of bucket i at [cstart[i], cstart[i + 1]).  The host counts
// the chunks of each bucket from the bucket offsets (one value per bucket); the
// descriptors themselves are written on the device.
void chunk_starts_host(const std::vector<int64_t>& off, int64_t cl, std::vector<int64_t>& cs) {
  cs.assign(off.size(), 0);
  int64_t n = 0;
  for (size_t i = 0; i + 1 < off.size(); ++i) {
    cs[i] = n;
    n += (off[i + 1] - off[i] + cl - 1) / cl;
  }
  cs.back() = n;
}

__global__ __launch_bounds__(NT) void k_fill_chunks(const int64_t* __restrict__ off,
                                                    const int64_t* __restrict__ cstart, int64_t cl,
                                                    ChunkDesc* __restrict__ d) {
  const int i = blockIdx.x;
  const int64_t c0 = cstart[i], c1 = cstart[i + 1], o0 = off[i], o1 = off[i + 1];
  for (int64_t c = c0 + threadIdx.x; c < c1; c += NT) {
    const int64_t b = o0 + (c - c0) * cl;
    d[c] = ChunkDesc{b, static_cast<uint32_t>(i), static_cast<uint32_t>(min(cl, o1 - b))};
  }
}

// Builds the missing chunk lists among `keys` (depth, chunk length): their chunk
// starts go up in one small host-to-device copy, the descriptors are filled on the
// device.  The lists are kept with the trie.
void ensure_chunk_lists(const Trie& tr, const std::vector<std::pair<int, int64_t>>& keys, hipStream_t s) {
  std::vector<std::pair<int, int64_t>> todo;
  for (const auto& k : keys)
    if (tr.chunks.find(k) == tr.chunks.end() && std::find(todo.begin(), todo.end(), k) == todo.end())
      todo.push_back(k);
  if (todo.empty()) return;
  std::vector<int64_t> host, cs;
  std::vector<size_t> at(todo.size());
  std::vector<int64_t> nch(todo.size());
  for (size_t j = 0; j < todo.size(); ++j) {
    chunk_starts_host(tr.hoff[todo[j].first], todo[j].second, cs);
    at[j] = host.size();
    nch[j] = cs.back();
    host.insert(host.end(), cs.begin(), cs.end());
  }
  int64_t* dev = tr.owner->get<int64_t>(host.size());
  // a pageable-memory copy has consumed its source when the call returns
  TTS_HIP(hipMemcpyAsync(dev, host.data(), sizeof(int64_t) * host.size(), hipMemcpyHostToDevice, s));
  for (size_t j = 0; j < todo.size(); ++j) {
    const int t = todo[j].first;
    const int nk = static_cast<int>(tr.hoff[t].size()) - 1;
    ChunkDesc* d = tr.owner->get<ChunkDesc>(std::max<int64_t>(nch[j], 1));
    if (nch[j] > 0) {
      k_fill_chunks<<<nk, NT, 0, s>>>(tr.boff[t], dev + at[j], todo[j].second, d);
      TTS_LAUNCH_CHECK();
    }
    tr.chunks.emplace(todo[j], ChunkList{d, nch[j], dev + at[j]});
  }
}

// One chunk list for the bucket offsets `off` (device) and `hoff` (host), in `mem`
// (entry-by-entry path, no trie).
ChunkList make_chunk_list(const int64_t* off, const std::vector<int64_t>& hoff, int64_t cl, DevMem& mem,
                          hipStream_t s) {
  std::vector<int64_t> cs;
  chunk_starts_host(hoff, cl, cs);
  int64_t* cptr = mem.get<int64_t>(cs.size());
  TTS_HIP(hipMemcpyAsync(cptr, cs.data(), sizeof(int64_t) * cs.size(), hipMemcpyHostToDevice, s));
  ChunkDesc* d = mem.get<ChunkDesc>(std::max<int64_t>(cs.back(), 1));
  if (cs.back() > 0) {
    k_fill_chunks<<<static_cast<unsigned>(hoff.size() - 1), NT, 0, s>>>(off, cptr, cl, d);
    TTS_LAUNCH_CHECK();
  }
  return ChunkList{d, cs.back(), cptr};
}

// Chunk length of a bucket product with O output columns (0: the narrow kernel,
// which takes no chunk list).
int64_t bucket_chunk(int O) { return O < 16 ? 0 : (O <= 32 ? 128 : 64); }

// The chunk list of depth t for chunk length cl (built and uploaded on first use).
ChunkList chunk_list(const Trie& tr, int t, int64_t cl, hipStream_t s) {
  ensure_chunk_lists(tr, {std::make_pair(t, cl)}, s);
  return tr.chunks.find(std::make_pair(t, cl))->second;
}

int lpe_for(const EvalDesc& ed) { return max_rank_of(ed) <= 32 ? 32 : 64; }

// Chunk length of the gradient kernels over P entries: a multiple of kc near
// P * tiles / 2048, so that the launch has about 2048 workgroups of equal work (plus
// at most one short chunk per bucket).
int64_t grad_chunk_len(int64_t P, int tiles, int kc) {
  const int64_t c = std::max<int64_t>(kc, (P * tiles + 2047) / 2048);
  return ((c + kc - 1) / kc) * kc;
}
// k_grad_small (few lanes per output entry): about 4096 chunks, at least 256 entries
int64_t grad_chunk_small(int64_t P) {
  const int64_t c = std::max<int64_t>(256, (P + 4095) / 4096);
  return ((c + 63) / 64) * 64;
}
// The gradient of an r0 x r1 core slice takes k_grad_small when an output entry has
// few lanes of work, the matrix-core kernel otherwise.
bool grad_is_small(int r0, int r1) { return r0 * r1 <= NT && (r0 < 16 || r1 < 16); }
int64_t grad_chunk(int r0, int r1, int64_t P, int kc) {
  const int tiles = ((r0 + 63) / 64) * ((r1 + 63) / 64);
  return grad_is_small(r0, r1) ? grad_chunk_small(P) : grad_chunk_len(P, tiles, kc);
}

// One pass over the items (no grid-stride repetition): every item's dependent loads
// are in flight at once rather than one after another within a workgroup.
unsigned blocks_for(int64_t items, int lpe) {
  const int64_t per_block = (NT / 64) * (64 / lpe);
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((items + per_block - 1) / per_block, 1 << 30)));
}

bool trie_possible(const EvalDesc& ed) {
  int bits = 0;
  for (int k = 0; k < ed.d; ++k) {
    int b = 0;
    while (b < 31 && (static_cast<int64_t>(ed.n[k]) - 1) >> b) ++b;
    bits += b;
  }
  return bits <= 63;
}

// Sorts the entries and builds the node arrays of every depth.  Returns false on a
// coordinate out of range.
// The arrays the trie keeps come from `mem`, temporaries from `scratch` (which may
// be the same object).
bool build_trie(const EvalDesc& ed, int64_t m, const int32_t* idx, DevMem& mem, DevMem& scratch, Allocator* al,
                Trie& tr, hipStream_t s) {
  const int d = ed.d;
  tr.owner = &mem;
  TrieGeom g{};
  g.d = d;
  int total = 0;
  for (int k = d - 1; k >= 0; --k) {
    int b = 0;
    while (b < 31 && (static_cast<int64_t>(ed.n[k]) - 1) >> b) ++b;
    g.bits[k] = b;
    g.off[k] = total;
    g.n[k] = ed.n[k];
    total += b;
  }
  tr.m = m;
  uint64_t* key = scratch.get<uint64_t>(m);
  uint64_t* val = mem.get<uint64_t>(m);
  uint64_t* kt = scratch.get<uint64_t>(m);
  uint64_t* vt = mem.get<uint64_t>(m);
  // counts[0]: index error flag; counts[t]: nodes at depth t (read back once, at the end)
  uint32_t* counts = scratch.get<uint32_t>(d + 1);
  TTS_HIP(hipMemsetAsync(counts, 0, sizeof(uint32_t) * (d + 1), s));
  k_tri_keys<<<grid_for(m, NT), NT, 0, s>>>(idx, m, g, key, val, counts);
  TTS_LAUNCH_CHECK();
  // The keys of out-of-range coordinates are garbage, but nothing below reads a core:
  // the build only touches arrays of length m, and the error is checked before any
  // use of the trie.
  if (radix_sort_pairs_pp(al, key, val, kt, vt, static_cast<uint32_t>(m), total, s)) {
    std::swap(key, kt);
    std::swap(val, vt);
  }
  tr.perm = val;
  uint32_t* flag = scratch.get<uint32_t>(m);
  uint32_t* pos = scratch.get<uint32_t>(m);
  uint32_t* ida = mem.get<uint32_t>(m);
  uint32_t* idb = mem.get<uint32_t>(m);
  tr.P.assign(d + 1, 1);
  tr.parent.assign(d + 1, nullptr);
  tr.coord.assign(d + 1, nullptr);
  uint32_t* prev = nullptr;
  for (int t = 1; t <= d; ++t) {
    // prefix (i_0..i_{t-1}) = key >> off[t-1]; mode t-1's field sits at off[t-1].
    // Node arrays are sized by m (an upper bound), so no count is read back here.
    const int psh = static_cast<int>(g.off[t - 1]);
    k_tri_flags<<<grid_for(m, NT), NT, 0, s>>>(key, m, psh, flag);
    TTS_LAUNCH_CHECK();
    exclusive_scan_u32(al, flag, pos, static_cast<uint32_t>(m), counts + t, s);
    tr.parent[t] = mem.get<uint32_t>(m);
    tr.coord[t] = mem.get<uint32_t>(m);
    uint32_t* st = nullptr;
    if (t == d) st = tr.start = mem.get<uint32_t>(m);
    uint32_t* cur = (t & 1) ? ida : idb;
    const uint64_t cmask = g.bits[t - 1] >= 64 ? ~0ull : ((1ull << g.bits[t - 1]) - 1ull);
    k_tri_nodes<<<grid_for(m, NT), NT, 0, s>>>(key, flag, pos, m, prev, psh, cmask, cur, tr.parent[t], tr.coord[t],
                                               st);
    TTS_LAUNCH_CHECK();
    prev = cur;
  }
  std::vector<uint32_t> hc(d + 1);
  {
    Readback rb(s);
    rb.add(hc.data(), counts, sizeof(uint32_t) * (d + 1));
    rb.sync();
  }
  if (hc[0]) return false;
  for (int t = 1; t <= d; ++t) tr.P[t] = hc[t];
  tr.leaf = prev;
  return true;
}

// Buckets of the depth-t nodes by their last index (stable radix sort).
void build_buckets(const EvalDesc& ed, Trie& tr, DevMem& mem, DevMem& scratch, Allocator* al, hipStream_t s) {
  const int d = ed.d;
  tr.bperm.assign(d + 1, nullptr);
  tr.boff.assign(d + 1, nullptr);
  tr.bmax.assign(d + 1, 0);
  const int64_t pmax = *std::max_element(tr.P.begin(), tr.P.end());
  uint64_t* key = scratch.get<uint64_t>(pmax);
  uint64_t* kt = scratch.get<uint64_t>(pmax);
  uint64_t* vt = mem.get<uint64_t>(pmax);
  std::vector<std::vector<int64_t>>& hoff = tr.hoff;
  hoff.assign(d + 1, {});
  Readback rb(s);
  for (int t = 1; t <= d; ++t) {
    const int nk = ed.n[t - 1];
    const int64_t P = tr.P[t];
    tr.bperm[t] = mem.get<uint64_t>(P);
    k_bucket_keys_u32<<<grid_for(P, NT), NT, 0, s>>>(tr.coord[t], tr.parent[t], P, key, tr.bperm[t]);
    TTS_LAUNCH_CHECK();
    int bits = 0;
    while (bits < 31 && (static_cast<int64_t>(nk) - 1) >> bits) ++bits;
    if (radix_sort_pairs_pp(al, key, tr.bperm[t], kt, vt, static_cast<uint32_t>(P), bits, s)) {
      std::swap(key, kt);
      tr.bperm[t] = vt;                  // the sorted permutation stays with depth t
      vt = mem.get<uint64_t>(pmax);      // fresh scratch for the next depth
    }
    tr.boff[t] = mem.get<int64_t>(nk + 1);
    k_bucket_offsets<<<grid_for(nk + 1, NT), NT, 0, s>>>(key, P, nk, tr.boff[t]);
    TTS_LAUNCH_CHECK();
    hoff[t].resize(nk + 1);
    rb.add(hoff[t].data(), tr.boff[t], sizeof(int64_t) * (nk + 1));
  }
  rb.sync();
  for (int t = 1; t <= d; ++t)
    for (int i = 0; i < ed.n[t - 1]; ++i) tr.bmax[t] = std::max(tr.bmax[t], hoff[t][i + 1] - hoff[t][i]);
}

// dst[q] = src[parent(q) or q] * S_{coord(q)} for every depth-t node q (see
// k_tri_fwd_bucket_mfma); K x O slices with strides sK (rows) and sI (index).
template <typename T>
void bucket_product(const Trie& tr, int t, int nk, int K, int O, int64_t sK, int64_t sI, const uint32_t* parent,
                    const T* src, const T* G, T* dst, hipStream_t s) {
  if (O < 16) {
    const int64_t per = (NT / O) * 8;
    const int64_t nchunk = std::max<int64_t>(1, (tr.bmax[t] + per - 1) / per);
    if (nchunk > 65535) fail(TT_ERR_TOO_LARGE, "evaluation bucket too large");
    k_tri_fwd_narrow<T><<<dim3(nk, static_cast<unsigned>(nchunk)), NT, 0, s>>>(K, O, sK, sI, tr.bperm[t], tr.boff[t],
                                                                                parent, src, G, dst);
  } else if (bucket_chunk(O) == 128) {
    const ChunkList cl = chunk_list(tr, t, 128, s);
    if (cl.n > 0)
      k_tri_fwd_bucket_mfma<T, 128><<<dim3(static_cast<unsigned>(cl.n), (O + 31) / 32), NT, 0, s>>>(
          K, O, sK, sI, cl.d, tr.bperm[t], parent, src, G, dst);
  } else {
    const ChunkList cl = chunk_list(tr, t, 64, s);
    if (cl.n > 0)
      k_tri_fwd_bucket_mfma<T, 64><<<dim3(static_cast<unsigned>(cl.n), (O + 63) / 64), NT, 0, s>>>(
          K, O, sK, sI, cl.d, tr.bperm[t], parent, src, G, dst);
  }
  TTS_LAUNCH_CHECK();
}

// The chunk lists a backward uses: the up pass's bucket products and the gradients.
template <typename T>
void backward_chunk_keys(const EvalDesc& ed, const Trie& tr, std::vector<std::pair<int, int64_t>>& keys) {
  constexpr int KC = sizeof(T) == 8 ? 32 : 64;
  const int d = ed.d;
  for (int t = d - 1; t >= 1; --t)
    if (ed.r[t + 1] > 4 && bucket_chunk(ed.r[t]) > 0) keys.emplace_back(t + 1, bucket_chunk(ed.r[t]));
  for (int t = 0; t < d; ++t) keys.emplace_back(t + 1, grad_chunk(ed.r[t], ed.r[t + 1], tr.P[t + 1], KC));
}

template <typename T>
void trie_forward(const EvalDesc& ed, Trie& tr, DevMem& mem, Allocator* al, std::vector<T*>& Lv, hipStream_t s) {
  const int d = ed.d;
  if (tr.bperm.empty()) build_buckets(ed, tr, mem, mem, al, s);
  {  // the chunk lists of this pass and of a backward, uploaded together
    std::vector<std::pair<int, int64_t>> keys;
    for (int t = 1; t <= d; ++t) {
      const int r0 = ed.r[t - 1], r1 = ed.r[t];
      const size_t core_bytes = sizeof(T) * static_cast<size_t>(r0) * ed.n[t - 1] * r1;
      if (!(r1 < 16 && core_bytes <= 48 * 1024) && bucket_chunk(r1) > 0) keys.emplace_back(t, bucket_chunk(r1));
    }
    backward_chunk_keys<T>(ed, tr, keys);
    ensure_chunk_lists(tr, keys, s);
  }
  Lv.assign(d + 1, nullptr);
  Lv[0] = mem.get<T>(1);
  k_one<T><<<1, 1, 0, s>>>(Lv[0]);
  TTS_LAUNCH_CHECK();
  for (int t = 1; t <= d; ++t) {
    const int r0 = ed.r[t - 1], r1 = ed.r[t], nk = ed.n[t - 1];
    const int64_t P = tr.P[t];
    Lv[t] = mem.get<T>(static_cast<size_t>(P) * r1);
    KTimer kt("eval_forward", s,
              static_cast<double>(P) * (r1 + 8) * sizeof(T) + static_cast<double>(tr.P[t - 1]) * r0 * sizeof(T) +
                  static_cast<double>(r0) * nk * r1 * sizeof(T),
              2.0 * static_cast<double>(P) * r0 * r1);
    const size_t core_bytes = sizeof(T) * static_cast<size_t>(r0) * nk * r1;
    if (r1 < 16 && core_bytes <= 48 * 1024) {
      const int64_t items = P * r1;
      const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((items + NT - 1) / NT, 4096));
      k_tri_fwd_trie<T><<<blocks, NT, core_bytes, s>>>(P, r0, r1, nk, tr.parent[t], tr.coord[t], Lv[t - 1],
                                                       static_cast<const T*>(ed.core[t - 1]), Lv[t]);
      TTS_LAUNCH_CHECK();
    } else {
      bucket_product<T>(tr, t, nk, r0, r1, static_cast<int64_t>(nk) * r1, r1, tr.parent[t], Lv[t - 1],
                        static_cast<const T*>(ed.core[t - 1]), Lv[t], s);
    }
  }
}

template <typename T>
tt_status trie_eval(const EvalDesc& ed, int64_t m, const int32_t* idx, T* y, hipStream_t s) {
  DevMem mem(s);
  Allocator al;
  al.stream = s;
  Trie tr;
  if (!build_trie(ed, m, idx, mem, mem, &al, tr, s)) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  std::vector<T*> Lv;
  trie_forward<T>(ed, tr, mem, &al, Lv, s);
  k_tri_out<T><<<grid_for(m, NT), NT, 0, s>>>(m, tr.leaf, tr.perm, Lv[ed.d], y);
  TTS_LAUNCH_CHECK();
  TTS_HIP(hipStreamSynchronize(s));
  return TT_OK;
}

// Up vectors (bottom-up) and the gradient of every core, from the left products of
// trie_forward.
template <typename T>
void trie_backward(const EvalDesc& ed, const Trie& tr, const std::vector<T*>& Lv, const T* gy, void* const* grads,
                   DevMem& mem, hipStream_t s) {
  const int d = ed.d;
  const int64_t m = tr.m;
  constexpr int KC = sizeof(T) == 8 ? 32 : 64;  // 33 KB of LDS: four workgroups per CU
  {  // the chunk lists of the up pass and the gradients (normally uploaded by the forward)
    std::vector<std::pair<int, int64_t>> keys;
    backward_chunk_keys<T>(ed, tr, keys);
    ensure_chunk_lists(tr, keys, s);
  }
  // up vectors, bottom-up
  std::vector<T*> Uv(d + 1, nullptr);
  Uv[d] = mem.get<T>(tr.P[d]);
  k_tri_leaf_up<T><<<grid_for(tr.P[d], NT), NT, 0, s>>>(tr.P[d], tr.start, m, tr.perm, gy, Uv[d]);
  TTS_LAUNCH_CHECK();
  std::vector<uint32_t*> cbeg(d + 1, nullptr);
  for (int t = d - 1; t >= 1; --t) {
    const int r0 = ed.r[t], r1 = ed.r[t + 1], nk = ed.n[t];
    const int64_t P = tr.P[t], Pc = tr.P[t + 1];
    cbeg[t] = mem.get<uint32_t>(P + 1);
    k_tri_child_ranges<<<grid_for(Pc, NT), NT, 0, s>>>(tr.parent[t + 1], Pc, P, cbeg[t]);
    TTS_LAUNCH_CHECK();
    T* GT = mem.get<T>(static_cast<size_t>(r0) * nk * r1);
    {
      const int ta = (r0 + 31) / 32, tb = (r1 + 31) / 32;
      if (r0 >= 16 && static_cast<int64_t>(nk) * ta * tb < (int64_t(1) << 31))
        k_slice_transpose_tiled<T><<<static_cast<unsigned>(static_cast<int64_t>(nk) * ta * tb), 256, 0, s>>>(
            static_cast<const T*>(ed.core[t]), r0, nk, r1, ta, tb, GT);
      else
        k_slice_transpose<T><<<grid_for(static_cast<size_t>(r0) * nk * r1, NT), NT, 0, s>>>(
            static_cast<const T*>(ed.core[t]), r0, nk, r1, GT);
      TTS_LAUNCH_CHECK();
    }
    Uv[t] = mem.get<T>(static_cast<size_t>(P) * r0);
    KTimer kt("eval_up", s, static_cast<double>(Pc) * (r1 + 8) * sizeof(T) + static_cast<double>(P) * r0 * sizeof(T),
              2.0 * static_cast<double>(Pc) * r0 * r1);
    const size_t up_lds = sizeof(T) * (static_cast<size_t>(r0) * nk * r1 + UP_CH * 4) + sizeof(uint32_t) * UP_CH;
    if (r1 <= 4 && r0 <= 256 && up_lds + sizeof(uint32_t) * (8 * NT / r0 + 1) <= 40 * 1024) {
      // short contraction, core in LDS: segments of consecutive parents
      const int QB = 8 * NT / r0;
      k_tri_up_seg<T><<<static_cast<unsigned>((P + QB - 1) / QB), NT, up_lds + sizeof(uint32_t) * (QB + 1), s>>>(
          P, QB, cbeg[t], tr.coord[t + 1], Uv[t + 1], r0, r1, nk, GT, Uv[t]);
      TTS_LAUNCH_CHECK();
    } else if (r1 <= 4) {
      // short contraction: each parent walks its children directly
      if (r0 <= 32)
        k_tri_up<T, 32><<<blocks_for(P, 32), NT, 0, s>>>(P, cbeg[t], tr.coord[t + 1], Uv[t + 1], r0, r1, GT, Uv[t]);
      else
        k_tri_up<T, 64><<<blocks_for(P, 64), NT, 0, s>>>(P, cbeg[t], tr.coord[t + 1], Uv[t + 1], r0, r1, GT, Uv[t]);
      TTS_LAUNCH_CHECK();
    } else {
      // children bucketed by index: V[c] = G[:, i_c, :] U[c] as gather-GEMMs, then the
      // fixed-order sum over each parent's children
      T* V = mem.get<T>(static_cast<size_t>(Pc) * r0);
      bucket_product<T>(tr, t + 1, nk, r1, r0, r0, static_cast<int64_t>(r1) * r0, nullptr, Uv[t + 1], GT, V, s);
      k_tri_segsum<T><<<grid_for(static_cast<size_t>(P) * r0, NT), NT, 0, s>>>(P, r0, cbeg[t], V, Uv[t]);
      TTS_LAUNCH_CHECK();
    }
  }
  // gradients: core t pairs parents at depth t with children at depth t+1
  for (int t = 0; t < d; ++t) {
    const int nk = ed.n[t], r0 = ed.r[t], r1 = ed.r[t + 1];
    const int64_t Pc = tr.P[t + 1];
    const int64_t csz = static_cast<int64_t>(r0) * nk * r1;
    const int tiles = ((r0 + 63) / 64) * ((r1 + 63) / 64);
    const bool small = grad_is_small(r0, r1);
    const ChunkList ch = chunk_list(tr, t + 1, grad_chunk(r0, r1, Pc, KC), s);
    T* part = mem.get<T>(static_cast<size_t>(std::max<int64_t>(ch.n, 1)) * r0 * r1);
    {
      KTimer ktm("eval_grad", s,
                 static_cast<double>(Pc) * (r0 + r1 + 8) * sizeof(T) + static_cast<double>(ch.n) * r0 * r1 * sizeof(T),
                 2.0 * static_cast<double>(Pc) * r0 * r1);
      if (ch.n > 0) {
        if (small)
          k_grad_small<T><<<static_cast<unsigned>(ch.n), NT, 0, s>>>(r0, r1, ch.d, tr.bperm[t + 1], Lv[t],
                                                                     t == 0 ? -1 : 0, Uv[t + 1], tr.parent[t + 1], part);
        else
          k_grad_partial_mfma<T, KC><<<dim3(static_cast<unsigned>(ch.n), tiles), NT, 0, s>>>(
              r0, r1, ch.d, tr.bperm[t + 1], nullptr, Lv[t], r0, t == 0 ? -1 : 0, Uv[t + 1], r1, 0, part,
              tr.parent[t + 1]);
        TTS_LAUNCH_CHECK();
      }
    }
    k_grad_reduce<T><<<grid_for(csz, NT), NT, 0, s>>>(r0, nk, r1, ch.cstart, part, static_cast<T*>(grads[t]));
    TTS_LAUNCH_CHECK();
  }
}

template <typename T>
tt_status trie_grad(const EvalDesc& ed, int64_t m, const int32_t* idx, const T* gy, void* const* grads,
                    hipStream_t s) {
  DevMem mem(s);
  Allocator al;
  al.stream = s;
  Trie tr;
  if (!build_trie(ed, m, idx, mem, mem, &al, tr, s)) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  std::vector<T*> Lv;
  trie_forward<T>(ed, tr, mem, &al, Lv, s);
  trie_backward<T>(ed, tr, Lv, gy, grads, mem, s);
  TTS_HIP(hipStreamSynchronize(s));
  return TT_OK;
}

bool trie_usable(const EvalDesc& ed, int64_t m) { return m > 0 && m < (int64_t(1) << 31) && trie_possible(ed); }

// Entry-by-entry evaluation (no trie): the fallback for coordinates too wide to pack.
template <typename T>
tt_status direct_eval(const EvalDesc& ed, int64_t m, const int32_t* idx, void* y_out, hipStream_t s) {
  DevMem mem(s);
  uint32_t* err = mem.get<uint32_t>(1);
  TTS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
  if (m > 0) launch_left<T>(ed, m, idx, static_cast<T*>(y_out), nullptr, err, s);
  uint32_t h = 0;
  {
    Readback rb(s);
    rb.add(&h, err, sizeof(h));
    rb.sync();
  }
  if (h) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  return TT_OK;
}

template <typename T>
tt_status direct_grad(const EvalDesc& ed, int64_t m, const int32_t* idx, const T* gy, void* const* grads,
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
  {
    Readback rb(s);
    rb.add(&h, err, sizeof(h));
    rb.sync();
  }
  if (h) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  uint64_t* key = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* perm = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* kt = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  uint64_t* vt = mem.get<uint64_t>(std::max<int64_t>(m, 1));
  constexpr int KC = sizeof(T) == 8 ? 32 : 64;  // 33 KB of LDS: four workgroups per CU
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
    if (radix_sort_pairs_pp(&al, key, perm, kt, vt, static_cast<uint32_t>(m), bits, s)) {
      std::swap(key, kt);
      std::swap(perm, vt);
    }
    int64_t* off = mem.get<int64_t>(nk + 1);
    k_bucket_offsets<<<grid_for(nk + 1, NT), NT, 0, s>>>(key, m, nk, off);
    TTS_LAUNCH_CHECK();
    std::vector<int64_t> hoff(nk + 1);
    {
      Readback rb(s);
      rb.add(hoff.data(), off, sizeof(int64_t) * (nk + 1));
      rb.sync();
    }
    const int tiles = ((r0 + 63) / 64) * ((r1 + 63) / 64);
    const ChunkList ch = make_chunk_list(off, hoff, grad_chunk_len(m, tiles, KC), mem, s);
    T* part = mem.get<T>(static_cast<size_t>(std::max<int64_t>(ch.n, 1)) * r0 * r1);
    const int64_t lo = (k >= 1) ? ed.loff[k] : -1;              // l_k (k >= 1); l_0 = 1
    const int64_t ro = (k + 1 <= d - 1) ? ed.roff[k + 1] : -1;  // r_{k+1}; r_d = 1
    if (ch.n > 0) {
      k_grad_partial_mfma<T, KC><<<dim3(static_cast<unsigned>(ch.n), tiles), NT, 0, s>>>(
          r0, r1, ch.d, perm, gy, L, ed.lsum, lo, R, ed.rsum, ro, part, nullptr);
      TTS_LAUNCH_CHECK();
    }
    k_grad_reduce<T><<<grid_for(csz, NT), NT, 0, s>>>(r0, nk, r1, ch.cstart, part, gout);
    TTS_LAUNCH_CHECK();
  }
  TTS_HIP(hipStreamSynchronize(s));
  return TT_OK;
}

template <typename T>
tt_status eval_impl(const EvalDesc& ed, int64_t m, const int32_t* idx, void* y_out, hipStream_t s) {
  if (trie_usable(ed, m)) return trie_eval<T>(ed, m, idx, static_cast<T*>(y_out), s);
  return direct_eval<T>(ed, m, idx, y_out, s);
}

template <typename T>
tt_status grad_impl(const EvalDesc& ed, int64_t m, const int32_t* idx, const T* gy, void* const* grads,
                    hipStream_t s) {
  if (trie_usable(ed, m)) return trie_grad<T>(ed, m, idx, gy, grads, s);
  return direct_grad<T>(ed, m, idx, gy, grads, s);
}

__global__ __launch_bounds__(NT) void k_check_coords(const int32_t* __restrict__ idx, int64_t m, EvalDesc ed,
                                                     uint32_t* __restrict__ err) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
  if (e >= m * ed.d) return;
  const int k = static_cast<int>(e % ed.d);
  const int32_t c = idx[e];
  if (c < 0 || c >= ed.n[k]) *err = 1u;
}

}  // namespace
}  // namespace tts

using namespace tts;

extern "C" tt_status tt_eval_entries(int32_t d, const int64_t* dims, const int64_t* ranks, const void* const* cores,
                                     int32_t dtype, int64_t m, const int32_t* idx, void* y_out, void* stream) {
  EvalDesc ed;
  tt_status st = check_args(d, dims, ranks, cores, dtype, m, idx, ed);
  if (st != TT_OK) return st;
  if (m > 0 && !y_out) {
    set_last_error("y_out must not be NULL when m > 0");
    return TT_ERR_ARG;
  }
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
  if ((m > 0 && !grad_y) || !grad_cores) {
    set_last_error("grad_y (when m > 0) and grad_cores must not be NULL");
    return TT_ERR_ARG;
  }
  for (int k = 0; k < d; ++k)
    if (!grad_cores[k]) {
      set_last_error("a gradient core pointer is NULL");
      return TT_ERR_ARG;
    }
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

// ---------------------------------------------------------------------------
// Evaluation plans: the trie (or, for coordinates too wide to pack, a copy of the
// coordinates) is built once and serves any number of forward and backward calls;
// a forward may keep its left products for the backward that follows.
// ---------------------------------------------------------------------------
struct tt_eval_plan_s {
  int32_t d = 0;
  int64_t dims[TT_MAX_D] = {};
  int64_t m = 0;
  bool trie = false;
  hipStream_t stream = nullptr;    // the creation stream: calls on it are stream-ordered
  tts::DevMem mem;                 // trie arrays, or the copy of the coordinates
  tts::Trie tr;
  const int32_t* idx = nullptr;    // direct path: the plan's copy of the coordinates
  std::unique_ptr<tts::DevMem> saved;  // left products of the last saving forward
  std::vector<void*> Lv;
  int32_t saved_dtype = -1;
  int64_t saved_ranks[TT_MAX_D + 1] = {};
  explicit tt_eval_plan_s(hipStream_t s) : mem(s) {}
};

namespace tts {
namespace {

template <typename T>
tt_status plan_forward(tt_eval_plan_s& p, const EvalDesc& ed, T* y, bool save, hipStream_t s) {
  if (!p.trie) return direct_eval<T>(ed, p.m, p.idx, y, s);
  auto mem = std::make_unique<DevMem>(s);
  Allocator al;
  al.stream = s;
  std::vector<T*> Lv;
  trie_forward<T>(ed, p.tr, *mem, &al, Lv, s);
  k_tri_out<T><<<grid_for(p.m, NT), NT, 0, s>>>(p.m, p.tr.leaf, p.tr.perm, Lv[ed.d], y);
  TTS_LAUNCH_CHECK();
  if (save) {
    p.saved = std::move(mem);
    p.Lv.assign(Lv.begin(), Lv.end());
  }
  return TT_OK;
}

template <typename T>
tt_status plan_backward(tt_eval_plan_s& p, const EvalDesc& ed, const T* gy, void* const* grads, bool use_saved,
                        hipStream_t s) {
  if (!p.trie) return direct_grad<T>(ed, p.m, p.idx, gy, grads, s);
  DevMem mem(s);
  std::vector<T*> Lv;
  if (use_saved) {
    for (void* v : p.Lv) Lv.push_back(static_cast<T*>(v));
  } else {
    Allocator al;
    al.stream = s;
    trie_forward<T>(ed, p.tr, mem, &al, Lv, s);
  }
  trie_backward<T>(ed, p.tr, Lv, gy, grads, mem, s);
  return TT_OK;
}

// A call on another stream than the plan's waits for the plan's stream first and for
// its own work at the end, so that memory freed to either stream's cache is idle.
struct StreamGuard {
  hipStream_t s;
  bool other;
  StreamGuard(const tt_eval_plan_s& p, hipStream_t call) : s(call), other(call != p.stream) {
    if (other) TTS_HIP(hipStreamSynchronize(p.stream));
  }
  void finish() {
    if (other) TTS_HIP(hipStreamSynchronize(s));
  }
};

}  // namespace
}  // namespace tts

extern "C" tt_status tt_eval_plan_create(int32_t d, const int64_t* dims, int64_t m, const int32_t* idx, void* stream,
                                         tt_eval_plan* plan) {
  auto bad = [](const char* why) {
    set_last_error(why);
    return TT_ERR_ARG;
  };
  if (!plan) return bad("plan must not be NULL");
  *plan = nullptr;
  if (d < 1 || d > TT_MAX_D) return bad("d must be in [1, TT_MAX_D]");
  if (!dims) return bad("dims must not be NULL");
  if (m < 0 || (m > 0 && !idx)) return bad("m must be >= 0 and idx non-NULL when m > 0");
  EvalDesc ed{};
  ed.d = d;
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1 || dims[k] > INT32_MAX) return bad("every mode size must be in [1, 2^31 - 1]");
    ed.n[k] = static_cast<int32_t>(dims[k]);
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto p = std::make_unique<tt_eval_plan_s>(s);
    p->stream = s;
    p->d = d;
    for (int k = 0; k < d; ++k) p->dims[k] = dims[k];
    p->m = m;
    p->trie = trie_usable(ed, m);
    if (p->trie) {
      DevMem scratch(s);
      Allocator al;
      al.stream = s;
      if (!build_trie(ed, m, idx, p->mem, scratch, &al, p->tr, s)) {
        set_last_error("a coordinate is outside its mode range");
        return TT_ERR_INDEX;
      }
      build_buckets(ed, p->tr, p->mem, scratch, &al, s);
    } else if (m > 0) {
      int32_t* c = p->mem.get<int32_t>(static_cast<size_t>(m) * d);
      TTS_HIP(hipMemcpyAsync(c, idx, sizeof(int32_t) * static_cast<size_t>(m) * d, hipMemcpyDeviceToDevice, s));
      DevMem scratch(s);
      uint32_t* err = scratch.get<uint32_t>(1);
      TTS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
      k_check_coords<<<grid_for(m * d, NT), NT, 0, s>>>(c, m, ed, err);
      TTS_LAUNCH_CHECK();
      uint32_t h = 0;
      {
        Readback rb(s);
        rb.add(&h, err, sizeof(h));
        rb.sync();
      }
      if (h) {
        set_last_error("a coordinate is outside its mode range");
        return TT_ERR_INDEX;
      }
      p->idx = c;
    }
    TTS_HIP(hipStreamSynchronize(s));
    *plan = p.release();
    return TT_OK;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}

extern "C" tt_status tt_eval_plan_forward(tt_eval_plan plan, const int64_t* ranks, const void* const* cores,
                                          int32_t dtype, void* y_out, int32_t save, void* stream) {
  if (!plan) {
    set_last_error("plan must not be NULL");
    return TT_ERR_ARG;
  }
  EvalDesc ed;
  tt_status st = check_core_args(plan->d, plan->dims, ranks, cores, dtype, ed);
  if (st != TT_OK) return st;
  if (plan->m > 0 && !y_out) {
    set_last_error("y_out must not be NULL when m > 0");
    return TT_ERR_ARG;
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamGuard guard(*plan, s);
    if (save) {
      plan->saved.reset();
      plan->Lv.clear();
      plan->saved_dtype = -1;
    }
    st = dtype == TT_DTYPE_F64 ? plan_forward<double>(*plan, ed, static_cast<double*>(y_out), save != 0, s)
                               : plan_forward<float>(*plan, ed, static_cast<float*>(y_out), save != 0, s);
    guard.finish();
    if (st == TT_OK && save) {
      plan->saved_dtype = dtype;
      for (int k = 0; k <= plan->d; ++k) plan->saved_ranks[k] = ranks[k];
    }
    return st;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}

extern "C" tt_status tt_eval_plan_backward(tt_eval_plan plan, const int64_t* ranks, const void* const* cores,
                                           int32_t dtype, const void* grad_y, void* const* grad_cores,
                                           int32_t use_saved, void* stream) {
  if (!plan) {
    set_last_error("plan must not be NULL");
    return TT_ERR_ARG;
  }
  EvalDesc ed;
  tt_status st = check_core_args(plan->d, plan->dims, ranks, cores, dtype, ed);
  if (st != TT_OK) return st;
  if ((plan->m > 0 && !grad_y) || !grad_cores) {
    set_last_error("grad_y (when m > 0) and grad_cores must not be NULL");
    return TT_ERR_ARG;
  }
  for (int k = 0; k < plan->d; ++k)
    if (!grad_cores[k]) {
      set_last_error("a gradient core pointer is NULL");
      return TT_ERR_ARG;
    }
  if (use_saved) {
    bool same = plan->saved_dtype == dtype;
    for (int k = 0; same && k <= plan->d; ++k) same = plan->saved_ranks[k] == ranks[k];
    if (!same) {
      set_last_error("use_saved needs a saving forward with the same ranks and dtype");
      return TT_ERR_ARG;
    }
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamGuard guard(*plan, s);
    st = dtype == TT_DTYPE_F64
             ? plan_backward<double>(*plan, ed, static_cast<const double*>(grad_y), grad_cores, use_saved != 0, s)
             : plan_backward<float>(*plan, ed, static_cast<const float*>(grad_y), grad_cores, use_saved != 0, s);
    guard.finish();
    return st;
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}

extern "C" void tt_eval_plan_free(tt_eval_plan plan) { delete plan; }

// ---------------------------------------------------------------------------
// Allocation-free evaluation: the per-entry chain kernel (as tt_eval_entries uses
// for coordinates it cannot pack), with its one word of scratch taken from the
// static `scratch` array instead of an allocation.
// ---------------------------------------------------------------------------
namespace tts {
namespace {

// The call needs one 4-byte word (the flag) whatever m and the ranks, so no input
// size can exceed the array.
static_assert(sizeof(uint32_t) <= sizeof(::scratch), "scratch too small");

__global__ void k_clear_flag(uint32_t* __restrict__ f) { *f = 0u; }

// Device address of `scratch` on the current device, looked up once per device with
// that device current.
uint32_t* noalloc_scratch() {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  TTS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(TT_ERR_DEVICE, "device ordinal outside [0, 64)");
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    TTS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
    if (!p) fail(TT_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    ptr[dev] = p;
  }
  return static_cast<uint32_t*>(ptr[dev]);
}

template <typename T>
tt_status noalloc_eval(const EvalDesc& ed, int64_t m, const int32_t* idx, T* y, hipStream_t s) {
  uint32_t* flag = noalloc_scratch();
  k_clear_flag<<<1, 1, 0, s>>>(flag);  // the array keeps the last call's contents
  TTS_LAUNCH_CHECK();
  if (m > 0) launch_left<T>(ed, m, idx, y, nullptr, flag, s);
  uint32_t h = 0;
  {
    Readback rb(s);
    rb.add(&h, flag, sizeof(h));
    rb.sync();
  }
  if (h) {
    set_last_error("a coordinate is outside its mode range");
    return TT_ERR_INDEX;
  }
  return TT_OK;
}

}  // namespace
}  // namespace tts

extern "C" tt_status tt_eval_entries_noalloc(int32_t d, const int64_t* dims, const int64_t* ranks,
                                             const void* const* cores, int32_t dtype, int64_t m, const int32_t* idx,
                                             void* y_out, void* stream) {
  EvalDesc ed;
  tt_status st = check_args(d, dims, ranks, cores, dtype, m, idx, ed);
  if (st != TT_OK) return st;
  if (m > 0 && !y_out) {
    set_last_error("y_out must not be NULL when m > 0");
    return TT_ERR_ARG;
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dtype == TT_DTYPE_F64 ? noalloc_eval<double>(ed, m, idx, static_cast<double*>(y_out), s)
                                 : noalloc_eval<float>(ed, m, idx, static_cast<float*>(y_out), s);
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  }
}
