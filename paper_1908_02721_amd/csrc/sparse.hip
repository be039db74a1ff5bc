// Kernels of the sparse stage: per-mode sparse unfoldings and their parallel-vector
// rounding (Deparallelisation of every level's unfolding, Algorithm 3 applied in the
// TT-SVD sweep of Algorithm 1 in place of the truncated SVD).
//
// Data flow of one level k (entries of M_k sorted so that every column -- a suffix
// (i_{k+1},...,i_d) -- is one contiguous segment):
//   col_flags/col_starts : segment boundaries -> column start offsets
//   canon                : one thread per column: order its entries by row rho,
//                          s = value at the smallest row, c_j = v_j / s (IEEE
//                          binary64 division), 64-bit hash of (m, rho_j, bits(c_j))
//   group                : open-addressing table keyed by the hash; a column that
//                          finds an occupied slot compares its full canonical key
//                          with the slot's representative column; the smallest
//                          row-major suffix key of each group is its leader
//   rep_list + sort      : leaders sorted by row-major suffix key -> group ids
//                          (first occurrence in row-major column order)
//   emit_n / emit_next   : N_k (CSC) and the next level's entries
//                          (rho' = g * n_{k+1} + i_{k+1}, value s)
#include "sparse.hpp"

#include <cmath>

namespace tts {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ uint64_t fmask(uint32_t b) { return (b >= 64) ? ~0ull : ((1ull << b) - 1ull); }

__global__ __launch_bounds__(NT) void k_ingest(const int32_t* __restrict__ idx, const double* __restrict__ val,
                                               uint32_t nnz, ModeInfo mi, uint64_t* __restrict__ keys,
                                               uint64_t* __restrict__ vbits, DevStatus* st) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  bool zero = false;
  if (e < nnz) {
    const int32_t* c = idx + static_cast<size_t>(e) * mi.d;
    const double v = val[e];
    uint64_t key = 0;
    bool bad = false;
    // the coordinates eight at a time, each group's loads issued together
    for (int j0 = 0; j0 < mi.d; j0 += 8) {
      int32_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = c[(j0 + u < mi.d) ? j0 + u : 0];
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
                                                  int level1, int check_long, const double* __restrict__ ev,
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
    if (check_long && start) {
      uint32_t j = e + 1;
      const uint32_t lim = (nE - e > static_cast<uint32_t>(kMaxLocal) + 1) ? e + kMaxLocal + 1 : nE;
      while (j < lim && (ekey[j] >> sh) == col) ++j;
      if (j - e > static_cast<uint32_t>(kMaxLocal)) atomicOr(&st->longcol, 1u);
    }
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

__global__ __launch_bounds__(NT) void k_norm_final(const double* __restrict__ part, uint32_t np, DevStatus* st) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < np; i += NT) s += part[i];
  s = wave_sum_f64(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    st->norm2 = t;
  }
}

__global__ __launch_bounds__(NT) void k_col_starts(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                                   uint32_t nE, uint32_t* __restrict__ col_start,
                                                   const DevStatus* st) {
  const uint32_t e = blockIdx.x * NT + threadIdx.x;
  if (e < nE && flag[e]) col_start[pos[e]] = e;
  if (e == 0) col_start[st->ncols] = nE;
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

__global__ __launch_bounds__(NT) void k_canon(CanonArgs a, ModeInfo mi) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c >= a.ncols) return;
  const uint32_t st = a.col_start[c], en = a.col_start[c + 1];
  const uint32_t m = en - st;
  uint64_t h = mix64(static_cast<uint64_t>(m) * 0x9e3779b97f4a7c15ull);
  double s;
  if (!a.sort_rows) {
    s = a.ev[st];
    for (uint32_t j = 0; j < m; ++j) {
      const uint32_t rho = a.erho ? a.erho[st + j] : static_cast<uint32_t>(a.ekey[st + j] & a.rho_mask);
      const double cv = a.ev[st + j] / s;
      a.crho[st + j] = rho;
      a.cval[st + j] = cv;
      h = mix64(h ^ rho);
      h = mix64(h ^ static_cast<uint64_t>(__double_as_longlong(cv)));
    }
  } else {
    // at most kMaxLocal entries (checked by the host): insertion sort by rho
    uint32_t rr[kMaxLocal];
    double vv[kMaxLocal];
    for (uint32_t j = 0; j < m; ++j) {
      const uint32_t r = a.erho[st + j];
      const double v = a.ev[st + j];
      uint32_t t = j;
      while (t > 0 && rr[t - 1] > r) {
        rr[t] = rr[t - 1];
        vv[t] = vv[t - 1];
        --t;
      }
      rr[t] = r;
      vv[t] = v;
    }
    s = vv[0];
    for (uint32_t j = 0; j < m; ++j) {
      const double cv = vv[j] / s;
      a.crho[st + j] = rr[j];
      a.cval[st + j] = cv;
      h = mix64(h ^ rr[j]);
      h = mix64(h ^ static_cast<uint64_t>(__double_as_longlong(cv)));
    }
  }
  a.colhash[c] = h;
  a.cols[c] = s;
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

__device__ __forceinline__ bool same_column(const uint32_t* __restrict__ crho, const double* __restrict__ cval,
                                            uint32_t sa, uint32_t sb, uint32_t m) {
  for (uint32_t j = 0; j < m; ++j) {
    if (crho[sa + j] != crho[sb + j]) return false;
    if (__double_as_longlong(cval[sa + j]) != __double_as_longlong(cval[sb + j])) return false;
  }
  return true;
}

__global__ __launch_bounds__(NT) void k_group(const uint64_t* __restrict__ colhash, const uint32_t* __restrict__ crho,
                                              const double* __restrict__ cval, const uint32_t* __restrict__ col_start,
                                              const uint64_t* __restrict__ rmkey, uint32_t ncols, uint64_t* table,
                                              uint64_t* slotmin, uint32_t tmask, uint32_t* __restrict__ slot,
                                              uint32_t* __restrict__ isrep) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c >= ncols) return;
  const uint64_t h = colhash[c];
  const uint32_t st = col_start[c];
  const uint32_t m = col_start[c + 1] - st;
  uint32_t p = static_cast<uint32_t>(h) & tmask;
  uint32_t rep = 0;
  // The table has more slots than columns, so an empty slot is always reached.
  for (uint32_t probe = 0; probe <= tmask; ++probe) {
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
  slot[c] = p;
  isrep[c] = rep;
  const uint64_t rk = rmkey[c];
  if (rk < __hip_atomic_load(&slotmin[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMin(reinterpret_cast<unsigned long long*>(&slotmin[p]), static_cast<unsigned long long>(rk));
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

__global__ __launch_bounds__(NT) void k_emit_n(const uint64_t* __restrict__ lslot, uint32_t beta,
                                               const uint64_t* __restrict__ table, const uint32_t* __restrict__ col_start,
                                               const uint32_t* __restrict__ npos, const uint32_t* __restrict__ crho,
                                               const double* __restrict__ cval, int64_t* __restrict__ colptr,
                                               int32_t* __restrict__ nrow, double* __restrict__ nval,
                                               const DevStatus* st) {
  const uint32_t j = blockIdx.x * NT + threadIdx.x;
  if (j == 0) colptr[beta] = st->nnz_n;
  if (j >= beta) return;
  const uint32_t p = static_cast<uint32_t>(lslot[j]);
  const uint32_t r = static_cast<uint32_t>(table[p] - 1);
  const uint32_t s0 = col_start[r], m = col_start[r + 1] - s0;
  const uint32_t o = npos[j];
  colptr[j] = o;
  for (uint32_t t = 0; t < m; ++t) {
    nrow[o + t] = static_cast<int32_t>(crho[s0 + t]);
    nval[o + t] = cval[s0 + t];
  }
}

__global__ __launch_bounds__(NT) void k_emit_next(EmitArgs a, ModeInfo mi) {
  const uint32_t c = blockIdx.x * NT + threadIdx.x;
  if (c >= a.ncols) return;
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

}  // namespace

void launch_ingest(const int32_t* idx, const double* val, uint32_t nnz, const ModeInfo& mi, uint64_t* keys,
                   uint64_t* vbits, DevStatus* st, hipStream_t s) {
  if (!nnz) return;
  k_ingest<<<grid_for(nnz, NT), NT, 0, s>>>(idx, val, nnz, mi, keys, vbits, st);
  TTS_LAUNCH_CHECK();
}

uint32_t norm_partials_count(uint32_t nE) { return grid_for(nE, NT); }

void launch_col_flags(const uint64_t* ekey, uint32_t nE, int sh, bool level1, bool check_long, const double* ev,
                      uint32_t* flag, double* norm_part, DevStatus* st, hipStream_t s) {
  k_col_flags<<<grid_for(nE, NT), NT, 0, s>>>(ekey, nE, sh, level1 ? 1 : 0, check_long ? 1 : 0, ev, flag,
                                              norm_part, st);
  TTS_LAUNCH_CHECK();
}

void launch_norm_final(const double* part, uint32_t np, DevStatus* st, hipStream_t s) {
  k_norm_final<<<1, NT, 0, s>>>(part, np, st);
  TTS_LAUNCH_CHECK();
}

void launch_col_starts(const uint32_t* flag, const uint32_t* pos, uint32_t nE, uint32_t* col_start,
                       const DevStatus* st, hipStream_t s) {
  k_col_starts<<<grid_for(nE, NT), NT, 0, s>>>(flag, pos, nE, col_start, st);
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

void launch_canon(const CanonArgs& a, const ModeInfo& mi, DevStatus*, hipStream_t s) {
  if (!a.ncols) return;
  // per column: read its entries' (key, rho, value) once, write (rho, c) and the
  // column record (hash, s, suffix, row-major key) once -- the caller passes the
  // entry count through the column starts; bytes are estimated from ncols here
  KTimer kt("level_canon", s, 56.0 * a.ncols, 0.0);
  k_canon<<<grid_for(a.ncols, NT), NT, 0, s>>>(a, mi);
  TTS_LAUNCH_CHECK();
}

void launch_group(const uint64_t* colhash, const uint32_t* crho, const double* cval, const uint32_t* col_start,
                  const uint64_t* rmkey, uint32_t ncols, uint64_t* table, uint64_t* slotmin, uint32_t tmask,
                  uint32_t* slot, uint32_t* isrep, hipStream_t s) {
  if (!ncols) return;
  // per column: read hash, start and row-major key, write slot and flag
  KTimer kt("level_group", s, 32.0 * ncols, 0.0);
  k_group<<<grid_for(ncols, NT), NT, 0, s>>>(colhash, crho, cval, col_start, rmkey, ncols, table, slotmin, tmask,
                                             slot, isrep);
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

void launch_emit_n(const uint64_t* lslot_sorted, uint32_t beta, const uint64_t* table, const uint32_t* col_start,
                   const uint32_t* npos, const uint32_t* crho, const double* cval, int64_t* colptr, int32_t* nrow,
                   double* nval, const DevStatus* st, hipStream_t s) {
  k_emit_n<<<grid_for(beta, NT), NT, 0, s>>>(lslot_sorted, beta, table, col_start, npos, crho, cval, colptr, nrow,
                                             nval, st);
  TTS_LAUNCH_CHECK();
}

void launch_emit_next(const EmitArgs& a, const ModeInfo& mi, hipStream_t s) {
  if (!a.ncols) return;
  k_emit_next<<<grid_for(a.ncols, NT), NT, 0, s>>>(a, mi);
  TTS_LAUNCH_CHECK();
}

}  // namespace tts
