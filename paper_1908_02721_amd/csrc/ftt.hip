// Fiber-trie FastTT (Algorithms 4-7 and 9) on gfx950.
//
// Exact TT (Algorithm 4 with Algorithm 5 as Depar).  For a quasi-permutation matrix
// Depar keeps each nonzero row once, numbered by increasing row index.  Left of core
// p the row of spl_2(G^(k)) is (prefix id of i_1..i_{k-1}) n_k + i_k, so the bond-k
// index of an entry is the rank of its pair (prefix id, i_k) among the distinct pairs:
// one radix sort of nnz keys, segment flags and a scan per level.  Right of core p
// the row of spl_1^T(G^(k)) is i_k r_k + (suffix id of i_{k+1}..i_d), ranked the same
// way from the last mode inwards.  The middle core holds the values at
// [prefix id][i_p][suffix id]; sorting those keys also finds duplicate coordinates.
// The entries' distinct prefixes and suffixes are exactly the fibers' ones, so the
// fibers are never formed (their number R, for reporting, is one more count).
//
// Rounding (Algorithm 6): a truncated-SVD sweep from core p to the right, a QR sweep
// back to core p, and a truncated-SVD sweep from core p to the left, all on dense
// cores with the library's FP64 kernels (CholeskyQR2 / Householder, one-sided
// Jacobi, f64 MFMA GEMM).
#include "ftt.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "linalg.hpp"
#include "prim.hpp"

namespace tts {
namespace {

constexpr int FT = 256;
constexpr uint32_t kNormChunk = 2048;  // entries per fixed-order partial sum of squares

struct ModeSizes {
  uint32_t n[TT_MAX_D];
};
struct FiberPack {
  uint32_t off[TT_MAX_D];  // bit offset of each mode in the fiber key (unused for the skipped mode)
};

uint32_t bits_of(uint64_t n) {  // bits to hold 0..n-1
  uint32_t b = 0;
  while (b < 64 && (uint64_t(1) << b) < n) ++b;
  return b;
}

unsigned grid_for(uint32_t n) { return static_cast<unsigned>((n + FT - 1) / FT); }

// bit 0: index out of range, bit 1: non-finite value; keep = finite, in range, nonzero
__global__ __launch_bounds__(FT) void k_ftt_check(const int32_t* __restrict__ idx, const double* __restrict__ val,
                                                  uint32_t nnz, int d, ModeSizes ms, uint32_t* __restrict__ keep,
                                                  uint32_t* __restrict__ err) {
  const uint32_t e = blockIdx.x * FT + threadIdx.x;
  if (e >= nnz) return;
  uint32_t bad = 0;
  for (int k = 0; k < d; ++k) {
    const int32_t x = idx[static_cast<size_t>(e) * d + k];
    if (x < 0 || static_cast<uint32_t>(x) >= ms.n[k]) bad |= 1u;
  }
  const double v = val[e];
  if (!isfinite(v)) bad |= 2u;
  keep[e] = (bad == 0 && v != 0.0) ? 1u : 0u;
  if (bad) atomicOr(err, bad);
}

__global__ __launch_bounds__(FT) void k_ftt_compact(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ pos,
                                                    uint32_t nnz, uint32_t* __restrict__ list) {
  const uint32_t e = blockIdx.x * FT + threadIdx.x;
  if (e < nnz && keep[e]) list[pos[e]] = e;
}

// key = id[j] * mul + i_mode (left: id = prefix id, mul = n_k) or i_mode * mul + id
// (right: id = suffix id, mul = r_k); id == null means 0.  val = j.
__global__ __launch_bounds__(FT) void k_ftt_key(const uint32_t* __restrict__ list, const int32_t* __restrict__ idx,
                                                int d, int mode, const uint32_t* __restrict__ id, uint64_t mul,
                                                bool right, uint32_t m, uint64_t* __restrict__ key,
                                                uint64_t* __restrict__ val) {
  const uint32_t j = blockIdx.x * FT + threadIdx.x;
  if (j >= m) return;
  const uint64_t i = static_cast<uint64_t>(idx[static_cast<size_t>(list[j]) * d + mode]);
  const uint64_t a = id ? id[j] : 0u;
  key[j] = right ? i * mul + a : a * mul + i;
  val[j] = j;
}

// middle key ((prefix id) n_p + i_p) r_p + suffix id, and the fiber key prefix id * r_p + suffix id
__global__ __launch_bounds__(FT) void k_ftt_key_mid(const uint32_t* __restrict__ list, const int32_t* __restrict__ idx,
                                                    int d, int mode, const uint32_t* __restrict__ pid,
                                                    const uint32_t* __restrict__ sid, uint64_t np, uint64_t rr,
                                                    uint32_t m, uint64_t* __restrict__ key, uint64_t* __restrict__ val,
                                                    uint64_t* __restrict__ fkey) {
  const uint32_t j = blockIdx.x * FT + threadIdx.x;
  if (j >= m) return;
  const uint64_t i = static_cast<uint64_t>(idx[static_cast<size_t>(list[j]) * d + mode]);
  const uint64_t a = pid ? pid[j] : 0u, b = sid ? sid[j] : 0u;
  key[j] = (a * np + i) * rr + b;
  val[j] = j;
  fkey[j] = a * rr + b;
}

// packed coordinates without mode `skip` (Algorithm 9's fiber counts)
__global__ __launch_bounds__(FT) void k_ftt_fiber_key(const uint32_t* __restrict__ list,
                                                      const int32_t* __restrict__ idx, int d, int skip, FiberPack fp,
                                                      uint32_t m, uint64_t* __restrict__ key) {
  const uint32_t j = blockIdx.x * FT + threadIdx.x;
  if (j >= m) return;
  uint64_t x = 0;
  for (int k = 0; k < d; ++k)
    if (k != skip) x |= static_cast<uint64_t>(idx[static_cast<size_t>(list[j]) * d + k]) << fp.off[k];
  key[j] = x;
}

__global__ __launch_bounds__(FT) void k_ftt_flags(const uint64_t* __restrict__ key, uint32_t m,
                                                  uint32_t* __restrict__ f) {
  const uint32_t t = blockIdx.x * FT + threadIdx.x;
  if (t < m) f[t] = (t == 0 || key[t] != key[t - 1]) ? 1u : 0u;
}

// id of sorted position t = (number of distinct keys before it, itself included) - 1;
// newid[j] = id for the entry j at t; the first entry of each distinct key sets the
// core's 1: left  (key = a n_k + i):  core[key * r_new + id]
//           right (key = i r_k + c):  core[id * block + key], block = n_k r_k
__global__ __launch_bounds__(FT) void k_ftt_assign(const uint64_t* __restrict__ key, const uint64_t* __restrict__ val,
                                                   const uint32_t* __restrict__ f, const uint32_t* __restrict__ ex,
                                                   uint32_t m, bool right, uint64_t mul, uint32_t* __restrict__ newid,
                                                   double* __restrict__ core) {
  const uint32_t t = blockIdx.x * FT + threadIdx.x;
  if (t >= m) return;
  const uint32_t id = ex[t] + f[t] - 1u;
  newid[val[t]] = id;
  if (f[t]) core[right ? static_cast<uint64_t>(id) * mul + key[t] : key[t] * mul + id] = 1.0;
}

// middle core values; equal adjacent keys are a repeated coordinate (bit 2)
__global__ __launch_bounds__(FT) void k_ftt_middle(const uint64_t* __restrict__ key, const uint64_t* __restrict__ val,
                                                   uint32_t m, const uint32_t* __restrict__ list,
                                                   const double* __restrict__ v, double* __restrict__ core,
                                                   uint32_t* __restrict__ err) {
  const uint32_t t = blockIdx.x * FT + threadIdx.x;
  if (t >= m) return;
  core[key[t]] = v[list[val[t]]];
  if (t > 0 && key[t] == key[t - 1]) atomicOr(err, 4u);
}

// sum of squares of kNormChunk consecutive kept values per workgroup, in a fixed order
__global__ __launch_bounds__(FT) void k_ftt_sumsq(const uint32_t* __restrict__ list, const double* __restrict__ v,
                                                  uint32_t m, double* __restrict__ part) {
  __shared__ double red[FT];
  const uint32_t base = blockIdx.x * kNormChunk;
  double acc = 0.0;
  for (uint32_t u = threadIdx.x; u < kNormChunk; u += FT) {
    const uint32_t j = base + u;
    if (j < m) {
      const double x = v[list[j]];
      acc = fma(x, x, acc);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = FT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <class T>
T read1(const T* dev, hipStream_t s) {
  T h{};
  {
    Readback rb(s);
    rb.add(&h, dev, sizeof(T));
    rb.sync();
  }
  return h;
}

// Validated, zero-free entry list (indices into the input), on the device.
struct Kept {
  DBuf<uint32_t> list;
  uint32_t m = 0;
};

void ftt_kept(Allocator* al, const int32_t* idx, const double* val, uint32_t nnz, const std::vector<int64_t>& dims,
              Kept& out, hipStream_t s) {
  const int d = static_cast<int>(dims.size());
  ModeSizes ms{};
  for (int k = 0; k < d; ++k) ms.n[k] = static_cast<uint32_t>(dims[k]);
  DBuf<uint32_t> keep(al, nnz), pos(al, nnz), st(al, 2);
  TTS_HIP(hipMemsetAsync(st.get(), 0, 2 * sizeof(uint32_t), s));
  k_ftt_check<<<grid_for(nnz), FT, 0, s>>>(idx, val, nnz, d, ms, keep.get(), st.get());
  TTS_LAUNCH_CHECK();
  exclusive_scan_u32(al, keep.get(), pos.get(), nnz, st.get() + 1, s);
  uint32_t h[2];
  {
    Readback rb(s);
    rb.add(h, st.get(), sizeof(h));
    rb.sync();
  }
  if (h[0] & 1u) fail(TT_ERR_INDEX, "a coordinate lies outside [0, n_k)");
  if (h[0] & 2u) fail(TT_ERR_NONFINITE, "a value is NaN or infinite");
  if (h[1] == 0) fail(TT_ERR_EMPTY, "no nonzero left after dropping explicit zeros");
  out.m = h[1];
  out.list.reset(al, out.m);
  k_ftt_compact<<<grid_for(nnz), FT, 0, s>>>(keep.get(), pos.get(), nnz, out.list.get());
  TTS_LAUNCH_CHECK();
}

// Sort (key, val) and count the distinct keys; flags and their exclusive scan are
// left in f / ex.  Returns the count (one read-back).
uint32_t sort_and_count(Allocator* al, DBuf<uint64_t>& key, DBuf<uint64_t>& val, uint32_t m, uint64_t key_range,
                        DBuf<uint32_t>& f, DBuf<uint32_t>& ex, hipStream_t s) {
  DBuf<uint64_t> kt(al, m), vt(al, m);
  radix_sort_pairs(al, key.get(), val.get(), kt.get(), vt.get(), m, static_cast<int>(std::max(1u, bits_of(key_range))),
                   s);
  DBuf<uint32_t> tot(al, 1);
  k_ftt_flags<<<grid_for(m), FT, 0, s>>>(key.get(), m, f.get());
  TTS_LAUNCH_CHECK();
  exclusive_scan_u32(al, f.get(), ex.get(), m, tot.get(), s);
  return read1(tot.get(), s);
}

void check_core(int64_t r0, int64_t n, int64_t r1, int k) {
  if (r0 > 16384 || r1 > 16384 || static_cast<double>(r0) * n * r1 > 4.0e9)
    fail(TT_ERR_TOO_LARGE, "exact fiber-trie TT too large to round on one device (core " + std::to_string(k) + ")");
}

}  // namespace

void ftt_exact(Allocator* al, const int32_t* idx, const double* val, uint32_t nnz, const std::vector<int64_t>& dims,
               int p, FttExact& out, hipStream_t s) {
  const int d = static_cast<int>(dims.size());
  Kept kp;
  ftt_kept(al, idx, val, nnz, dims, kp, s);
  const uint32_t m = kp.m;
  out.nnz = m;
  // ||A||_F: fixed-order partial sums, added on the host in order
  {
    const uint32_t np = (m + kNormChunk - 1) / kNormChunk;
    DBuf<double> part(al, np);
    k_ftt_sumsq<<<np, FT, 0, s>>>(kp.list.get(), val, m, part.get());
    TTS_LAUNCH_CHECK();
    std::vector<double> h(np);
    {
      Readback rb(s);
      rb.add(h.data(), part.get(), sizeof(double) * np);
      rb.sync();
    }
    double ss = 0.0;
    for (double x : h) ss += x;
    out.norm = std::sqrt(ss);
  }
  out.ranks.assign(d + 1, 1);
  out.cores.clear();
  out.cores.resize(d);
  DBuf<uint64_t> key(al, m), v(al, m);
  DBuf<uint32_t> f(al, m), ex(al, m);
  // prefix ids, k = 1..p-1 (core k, 1-based)
  DBuf<uint32_t> pid, pnew;
  for (int k = 1; k < p; ++k) {
    const uint64_t nk = static_cast<uint64_t>(dims[k - 1]), r0 = static_cast<uint64_t>(out.ranks[k - 1]);
    k_ftt_key<<<grid_for(m), FT, 0, s>>>(kp.list.get(), idx, d, k - 1, k > 1 ? pid.get() : nullptr, nk, false, m,
                                         key.get(), v.get());
    TTS_LAUNCH_CHECK();
    const uint32_t rk = sort_and_count(al, key, v, m, r0 * nk, f, ex, s);
    check_core(static_cast<int64_t>(r0), static_cast<int64_t>(nk), rk, k);
    out.ranks[k] = rk;
    const size_t ne = static_cast<size_t>(r0) * nk * rk;
    out.cores[k - 1].reset(al, sizeof(double) * ne);
    TTS_HIP(hipMemsetAsync(out.cores[k - 1].get(), 0, sizeof(double) * ne, s));
    pnew.reset(al, m);
    k_ftt_assign<<<grid_for(m), FT, 0, s>>>(key.get(), v.get(), f.get(), ex.get(), m, false, rk, pnew.get(),
                                            reinterpret_cast<double*>(out.cores[k - 1].get()));
    TTS_LAUNCH_CHECK();
    std::swap(pid, pnew);
  }
  // suffix ids, k = d..p+1
  DBuf<uint32_t> sid, snew;
  for (int k = d; k > p; --k) {
    const uint64_t nk = static_cast<uint64_t>(dims[k - 1]), r1 = static_cast<uint64_t>(out.ranks[k]);
    k_ftt_key<<<grid_for(m), FT, 0, s>>>(kp.list.get(), idx, d, k - 1, k < d ? sid.get() : nullptr, r1, true, m,
                                         key.get(), v.get());
    TTS_LAUNCH_CHECK();
    const uint32_t rk = sort_and_count(al, key, v, m, nk * r1, f, ex, s);
    check_core(rk, static_cast<int64_t>(nk), static_cast<int64_t>(r1), k);
    out.ranks[k - 1] = rk;
    const size_t ne = static_cast<size_t>(rk) * nk * r1;
    out.cores[k - 1].reset(al, sizeof(double) * ne);
    TTS_HIP(hipMemsetAsync(out.cores[k - 1].get(), 0, sizeof(double) * ne, s));
    snew.reset(al, m);
    k_ftt_assign<<<grid_for(m), FT, 0, s>>>(key.get(), v.get(), f.get(), ex.get(), m, true, nk * r1, snew.get(),
                                            reinterpret_cast<double*>(out.cores[k - 1].get()));
    TTS_LAUNCH_CHECK();
    std::swap(sid, snew);
  }
  // middle core p: values, duplicates, and the fiber count R
  {
    const uint64_t np = static_cast<uint64_t>(dims[p - 1]);
    const uint64_t r0 = static_cast<uint64_t>(out.ranks[p - 1]), r1 = static_cast<uint64_t>(out.ranks[p]);
    check_core(static_cast<int64_t>(r0), static_cast<int64_t>(np), static_cast<int64_t>(r1), p);
    DBuf<uint64_t> fkey(al, m), fval(al, m);
    k_ftt_key_mid<<<grid_for(m), FT, 0, s>>>(kp.list.get(), idx, d, p - 1, p > 1 ? pid.get() : nullptr,
                                             p < d ? sid.get() : nullptr, np, r1, m, key.get(), v.get(), fkey.get());
    TTS_LAUNCH_CHECK();
    {
      DBuf<uint64_t> kt(al, m), vt(al, m);
      radix_sort_pairs(al, key.get(), v.get(), kt.get(), vt.get(), m,
                       static_cast<int>(std::max(1u, bits_of(r0 * np * r1))), s);
    }
    const size_t ne = static_cast<size_t>(r0) * np * r1;
    out.cores[p - 1].reset(al, sizeof(double) * ne);
    TTS_HIP(hipMemsetAsync(out.cores[p - 1].get(), 0, sizeof(double) * ne, s));
    DBuf<uint32_t> err(al, 1);
    TTS_HIP(hipMemsetAsync(err.get(), 0, sizeof(uint32_t), s));
    k_ftt_middle<<<grid_for(m), FT, 0, s>>>(key.get(), v.get(), m, kp.list.get(), val,
                                            reinterpret_cast<double*>(out.cores[p - 1].get()), err.get());
    TTS_LAUNCH_CHECK();
    if (read1(err.get(), s) & 4u) fail(TT_ERR_DUPLICATE, "the same coordinate appears twice among the nonzeros");
    TTS_HIP(hipMemsetAsync(fval.get(), 0, sizeof(uint64_t) * m, s));
    out.fibers = sort_and_count(al, fkey, fval, m, r0 * r1, f, ex, s);
  }
}

int ftt_select_p(Allocator* al, const int32_t* idx, const double* val, uint32_t nnz, const std::vector<int64_t>& dims,
                 std::vector<double>* costs_out, hipStream_t s) {
  const int d = static_cast<int>(dims.size());
  Kept kp;
  ftt_kept(al, idx, val, nnz, dims, kp, s);
  const uint32_t m = kp.m;
  DBuf<uint64_t> key(al, m), v(al, m);
  DBuf<uint32_t> f(al, m), ex(al, m);
  std::vector<double> costs(d);
  for (int p = 1; p <= d; ++p) {
    FiberPack fp{};
    uint32_t total = 0;
    for (int k = 0; k < d; ++k) {
      if (k == p - 1) continue;
      fp.off[k] = total;
      total += bits_of(static_cast<uint64_t>(dims[k]));
    }
    if (total > 63) fail(TT_ERR_TOO_LARGE, "packed fiber key needs more than 63 bits");
    uint64_t R = 1;
    if (d > 1) {
      k_ftt_fiber_key<<<grid_for(m), FT, 0, s>>>(kp.list.get(), idx, d, p - 1, fp, m, key.get());
      TTS_LAUNCH_CHECK();
      TTS_HIP(hipMemsetAsync(v.get(), 0, sizeof(uint64_t) * m, s));
      R = sort_and_count(al, key, v, m, total >= 64 ? ~0ull : (uint64_t(1) << total), f, ex, s);
    }
    // rank bounds of Algorithm 4 (saturated at R), then the estimate of Sec. 3.6 with
    // f_SVD(m, n) = m n min(m, n) and both rank sets set to the bounds
    std::vector<uint64_t> rb(d + 1, 1);
    for (int k = 1; k < d; ++k) {
      uint64_t prod = 1;
      if (k < p) {
        for (int i = 0; i < k && prod < R; ++i) prod *= static_cast<uint64_t>(dims[i]);
      } else {
        for (int i = k; i < d && prod < R; ++i) prod *= static_cast<uint64_t>(dims[i]);
      }
      rb[k] = std::min<uint64_t>(R, prod);
    }
    auto fsvd = [](double a, double b) { return a * b * std::min(a, b); };
    auto n = [&](int i) { return static_cast<double>(dims[i - 1]); };  // 1-based
    auto rr = [&](int i) { return static_cast<double>(rb[i]); };
    double fcost = fsvd(rr(p - 1) * n(p), rr(p));
    for (int i = p + 1; i <= d - 1; ++i) fcost += fsvd(rr(i - 1) * n(i), rr(i));
    for (int i = 2; i <= p; ++i) fcost += fsvd(rr(i - 1), n(i) * rr(i));
    costs[p - 1] = fcost;
  }
  int best = 0;
  for (int p = 1; p < d; ++p)
    if (costs[p] < costs[best]) best = p;
  if (costs_out) *costs_out = costs;
  return best + 1;
}

void ftt_round(Allocator* al, const std::vector<int64_t>& dims, int p, double eps, double norm, int max_rank,
               bool dynamic, int prec, std::vector<DBuf<char>>& cores, std::vector<int64_t>& r, RoundOutput& out,
               hipEvent_t mid, hipStream_t s) {
  const int d = static_cast<int>(dims.size());
  const double den = std::sqrt(static_cast<double>(p - 1)) + std::sqrt(static_cast<double>(d - p));
  const double delta = eps * norm / den;
  // Algorithm 8: budgets of the sweep right of p and of the sweep left of p; a bond
  // gets the remaining budget shared by the bonds still to come in its sweep, and the
  // budget then loses what the bond discarded
  const double right = std::sqrt(static_cast<double>(d - p)) / den * eps * norm;
  const double left = std::sqrt(static_cast<double>(p - 1)) / den * eps * norm;
  double right2 = right * right, left2 = left * left;
  out.sigma.assign(d - 1, {});
  out.tail.assign(d - 1, 0.0);
  out.bond_delta.assign(d - 1, delta);
  auto core = [&](int k) { return reinterpret_cast<double*>(cores[k - 1].get()); };
  // first SVD sweep, k = p..d-1: spl_2(G^(k)) ((r0 n) x r1) = U S V^T, core k := U,
  // G^(k+1) := (S V^T) x_1 G^(k+1)
  for (int k = p; k <= d - 1; ++k) {
    const int r0 = static_cast<int>(r[k - 1]), n = static_cast<int>(dims[k - 1]), r1 = static_cast<int>(r[k]);
    const int m = r0 * n;
    DBuf<double> G(al, static_cast<size_t>(m) * r1);
    transpose(core(k), r1, m, r1, G.get(), m, s);  // stored [r0][n][r1] = column-major r1 x m
    const double dk = dynamic ? std::sqrt(right2 / static_cast<double>(d - k)) : delta;
    out.bond_delta[k - 1] = dk;
    SvdPart sv;
    truncated_svd(al, prec, G.get(), m, r1, dk * dk, max_rank, sv, s);
    const int rk = sv.rank;
    out.sigma[k - 1] = std::move(sv.sigma);
    out.tail[k - 1] = sv.tail;
    right2 = std::max(0.0, right2 - sv.tail);
    DBuf<char> Ck(al, sizeof(double) * static_cast<size_t>(m) * rk);
    transpose(reinterpret_cast<const double*>(sv.U.get()), m, rk, m, reinterpret_cast<double*>(Ck.get()), rk, s);
    // core k+1 stored as column-major (n' r1') x r1 = spl_1^T; times VS (r1 x rk)
    const int m2 = static_cast<int>(dims[k]) * static_cast<int>(r[k + 1]);
    DBuf<char> Cn(al, sizeof(double) * static_cast<size_t>(m2) * rk);
    gemm_prec(al, prec, false, false, m2, rk, r1, 1.0, core(k + 1), m2, sv.VS.get(), r1, 0.0,
         reinterpret_cast<double*>(Cn.get()), m2, s);
    cores[k - 1] = std::move(Ck);
    cores[k] = std::move(Cn);
    r[k] = rk;
  }
  // QR sweep, k = d..p+1: spl_1^T(G^(k)) ((n r1) x r0) = Q R, core k := Q^T,
  // G^(k-1) := G^(k-1) x_3 R^T
  for (int k = d; k >= p + 1; --k) {
    const int r0 = static_cast<int>(r[k - 1]), n = static_cast<int>(dims[k - 1]), r1 = static_cast<int>(r[k]);
    const int m = n * r1, q = std::min(m, r0);
    DBuf<double> Rm(al, static_cast<size_t>(q) * r0);
    DBuf<char> Q(al, sizeof(double) * static_cast<size_t>(m) * q);
    bool done = false;
    if (m >= r0) {  // CholeskyQR2, checked; Householder when a factor breaks down
      DBuf<int32_t> ok(al, 4);
      cholqr2_async(al, core(k), m, r0, reinterpret_cast<double*>(Q.get()), Rm.get(), ok.get(), s);
      int32_t h[4];
      {
        Readback rb(s);
        rb.add(h, ok.get(), sizeof(h));
        rb.sync();
      }
      done = h[0] && h[1] && h[2] && h[3];
    }
    if (!done) qr_explicit(al, core(k), m, r0, m, reinterpret_cast<double*>(Q.get()), m, Rm.get(), q, s);
    // core k-1 stored as column-major r0 x (r0' n') = spl_2^T; new = R (q x r0) times it
    const int cols = static_cast<int>(r[k - 2]) * static_cast<int>(dims[k - 2]);
    DBuf<char> Cp(al, sizeof(double) * static_cast<size_t>(q) * cols);
    gemm_prec(al, prec, false, false, q, cols, r0, 1.0, Rm.get(), q, core(k - 1), r0, 0.0, reinterpret_cast<double*>(Cp.get()),
         q, s);
    cores[k - 1] = std::move(Q);  // column-major m x q = [q][n][r1]
    cores[k - 2] = std::move(Cp);
    r[k - 1] = q;
  }
  out.qr_ranks = r;
  TTS_HIP(hipEventRecord(mid, s));
  // second SVD sweep, k = p..2: spl_1^T(G^(k)) ((n r1) x r0) = U S V^T, core k := U^T,
  // G^(k-1) := G^(k-1) x_3 (V S)
  for (int k = p; k >= 2; --k) {
    const int r0 = static_cast<int>(r[k - 1]), n = static_cast<int>(dims[k - 1]), r1 = static_cast<int>(r[k]);
    const int m = n * r1;
    const double dk = dynamic ? std::sqrt(left2 / static_cast<double>(k - 1)) : delta;
    out.bond_delta[k - 2] = dk;
    SvdPart sv;
    truncated_svd(al, prec, core(k), m, r0, dk * dk, max_rank, sv, s);
    const int rk = sv.rank;
    out.sigma[k - 2] = std::move(sv.sigma);
    out.tail[k - 2] = sv.tail;
    left2 = std::max(0.0, left2 - sv.tail);
    const int rows2 = static_cast<int>(r[k - 2]) * static_cast<int>(dims[k - 2]);
    DBuf<char> Pn(al, sizeof(double) * static_cast<size_t>(rows2) * rk);
    gemm_prec(al, prec, true, false, rk, rows2, r0, 1.0, sv.VS.get(), r0, core(k - 1), r0, 0.0,
         reinterpret_cast<double*>(Pn.get()), rk, s);
    cores[k - 1] = std::move(sv.U);
    cores[k - 2] = std::move(Pn);
    r[k - 1] = rk;
  }
  out.ranks = r;
  out.dtype = TT_DTYPE_F64;
  if (prec != TT_FP64) {  // reduced-precision results are handed out in binary32
    for (int k = 0; k < d; ++k) {
      const size_t ne = static_cast<size_t>(r[k]) * dims[k] * r[k + 1];
      DBuf<char> c32(al, sizeof(float) * ne);
      to_f32(reinterpret_cast<const double*>(cores[k].get()), ne, reinterpret_cast<float*>(c32.get()), s);
      cores[k] = std::move(c32);
    }
    out.dtype = TT_DTYPE_F32;
  }
}

}  // namespace tts
