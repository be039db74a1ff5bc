// C-ABI of libttsparse: argument checks, the host loop over levels and bonds, and
// result ownership.  Every step of the decomposition runs in the library's HIP
// kernels; the host only sequences launches and reads back small counts.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "dense.hpp"
#include "ftt.hpp"
#include "prim.hpp"
#include "slice.hpp"
#include "sparse.hpp"

namespace tts {

namespace {
thread_local std::string g_last_error;
thread_local DevStatus* g_host_status = nullptr;

void set_error(const std::string& m) { g_last_error = m; }
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

DevStatus* host_status() {
  if (!g_host_status) {
    void* p = nullptr;
    TTS_HIP(hipHostMalloc(&p, sizeof(DevStatus), hipHostMallocDefault));
    g_host_status = static_cast<DevStatus*>(p);
  }
  return g_host_status;
}

void configure_pool_once() {
  static bool done[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = std::numeric_limits<uint64_t>::max();
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

uint32_t bits_for(uint64_t n) {  // bits to hold values 0..n-1
  uint32_t b = 0;
  while (b < 64 && (n - 1) >> b) ++b;
  return b;
}

}  // namespace

void fail(tt_status s, const std::string& msg) { throw Error{s, msg}; }

bool log_on() {
  static const bool on = [] {
    const char* e = std::getenv("TTSPARSE_LOG");
    return e && e[0] == '1';
  }();
  return on;
}

void logf(const char* fmt, ...) {
  if (!log_on()) return;
  std::va_list ap;
  va_start(ap, fmt);
  std::fputs("[ttsparse] ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
}

double host_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Device block cache.  Blocks are kept per stream in size classes (four classes per
// power of two); a block released on a stream is handed out again only to work on
// the same stream, so stream order makes the reuse safe without synchronisation.
// Blocks stay cached until the process ends.
// ---------------------------------------------------------------------------
namespace {
struct BlockCache {
  std::mutex mu;
  std::map<std::pair<hipStream_t, size_t>, std::vector<void*>> free;
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();
  return *c;
}
size_t size_class(size_t bytes) {
  if (bytes <= 256) return 256;
  int lg = 63 - __builtin_clzll(static_cast<unsigned long long>(bytes - 1));
  const size_t step = (static_cast<size_t>(1) << lg) / 4;
  return ((bytes + step - 1) / step) * step;
}
}  // namespace

namespace {
// The staging buffer is pinned, mapped and coherent host memory: one small kernel
// writes every pending piece into it (a copy engine transfer per piece costs a blit
// launch each, about 4 us).
struct PinnedStage {
  char* p = nullptr;   // host address
  char* dp = nullptr;  // the same memory as the device sees it
  size_t cap = 0;
  ~PinnedStage() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local PinnedStage g_stage;
thread_local const Readback* g_stage_owner = nullptr;  // the Readback with pieces pending

constexpr int kGatherPieces = 8;
struct GatherList {
  const uint32_t* src[kGatherPieces];
  uint32_t off[kGatherPieces];    // in 4-byte words of the staging buffer
  uint32_t words[kGatherPieces];  // 4-byte words of the piece
  int n;
};
__global__ void k_gather_host(GatherList g, uint32_t* __restrict__ dst) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (int k = 0; k < g.n; ++k)
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < g.words[k]; w += stride)
      dst[g.off[k] + w] = g.src[k][w];
}
}  // namespace

Readback::~Readback() {
  if (g_stage_owner == this) g_stage_owner = nullptr;
}

void Readback::add(void* host, const void* dev, size_t bytes) {
  if (!bytes) return;
  if (g_stage_owner && g_stage_owner != this) fail(TT_ERR_DEVICE, "internal: overlapping read-backs on one thread");
  if ((bytes & 3) || (reinterpret_cast<uintptr_t>(dev) & 3)) fail(TT_ERR_DEVICE, "internal: unaligned read-back");
  const size_t off = (off_ + 255) & ~static_cast<size_t>(255);
  if (off + bytes > g_stage.cap) {
    // grow: the pieces already pending land first
    sync();
    const size_t cap = std::max<size_t>(size_t(1) << 20, 2 * bytes);
    if (g_stage.p) TTS_HIP(hipHostFree(g_stage.p));
    g_stage.p = g_stage.dp = nullptr;
    g_stage.cap = 0;
    void* q = nullptr;
    TTS_HIP(hipHostMalloc(&q, cap, hipHostMallocMapped | hipHostMallocCoherent));
    void* dq = nullptr;
    TTS_HIP(hipHostGetDevicePointer(&dq, q, 0));
    g_stage.p = static_cast<char*>(q);
    g_stage.dp = static_cast<char*>(dq);
    g_stage.cap = cap;
    add(host, dev, bytes);
    return;
  }
  g_stage_owner = this;
  pend_.push_back(Piece{host, dev, off, bytes});
  off_ = off + bytes;
}

void Readback::sync() {
  // one gather kernel per kGatherPieces pieces, then one wait
  for (size_t i = 0; i < pend_.size(); i += kGatherPieces) {
    GatherList g{};
    size_t total = 0;
    for (size_t k = i; k < std::min(pend_.size(), i + kGatherPieces); ++k) {
      g.src[g.n] = static_cast<const uint32_t*>(pend_[k].dev);
      g.off[g.n] = static_cast<uint32_t>(pend_[k].off / 4);
      g.words[g.n] = static_cast<uint32_t>(pend_[k].bytes / 4);
      total = std::max(total, pend_[k].bytes / 4);
      ++g.n;
    }
    const unsigned blocks = static_cast<unsigned>(std::min<size_t>((total + 255) / 256, 64));
    k_gather_host<<<std::max(1u, blocks), 256, 0, s_>>>(g, reinterpret_cast<uint32_t*>(g_stage.dp));
    TTS_LAUNCH_CHECK();
  }
  TTS_HIP(hipStreamSynchronize(s_));
  for (const Piece& x : pend_) std::memcpy(x.host, g_stage.p + x.off, x.bytes);
  pend_.clear();
  off_ = 0;
  if (g_stage_owner == this) g_stage_owner = nullptr;
}

void* cached_alloc(size_t bytes, hipStream_t s) {
  const size_t cls = size_class(bytes);
  {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.free.find({s, cls});
    if (it != c.free.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, cls, s);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void cached_free(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  c.free[{s, size_class(bytes)}].push_back(p);
}

// Releases every cached block (of every stream) after the device has finished all
// work; returns the bytes released.
uint64_t cache_trim() {
  BlockCache& c = block_cache();
  std::lock_guard<std::mutex> g(c.mu);
  TTS_HIP(hipDeviceSynchronize());
  uint64_t bytes = 0;
  for (auto& kv : c.free) {
    for (void* p : kv.second) {
      TTS_HIP(hipFree(p));
      bytes += kv.first.second;
    }
  }
  c.free.clear();
  return bytes;
}

void* Allocator::get(size_t bytes) {
  if (budget && in_use + bytes > budget)
    fail(TT_ERR_NOMEM, "device_mem_budget exceeded (" + std::to_string(in_use + bytes) + " bytes needed)");
  void* p = nullptr;
  if (hook_alloc) {
    p = hook_alloc(bytes, ctx);
    if (!p) fail(TT_ERR_NOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    p = cached_alloc(bytes, stream);
    if (!p) fail(TT_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  in_use += bytes;
  peak = std::max(peak, in_use);
  return p;
}

void Allocator::put(void* p, size_t bytes) {
  if (!p) return;
  if (hook_free)
    hook_free(p, ctx);
  else
    cached_free(p, bytes, stream);
  in_use -= bytes;
}

struct LevelData {
  uint32_t ncols = 0, beta = 0, nnz_n = 0;
  DBuf<int64_t> col;
  DBuf<int32_t> g;
  DBuf<double> s;
  DBuf<int64_t> colptr;
  DBuf<int32_t> row;
  DBuf<double> val;
};

}  // namespace tts

struct tt_result_s {
  tts::Allocator al;
  int32_t d = 0;
  std::vector<int64_t> dims;
  int64_t nnz = 0;
  double norm = 0.0, delta = 0.0;
  int32_t rounded = 0;
  std::vector<tts::LevelData> lev;
  tts::DBuf<double> last_exact;
  std::vector<int64_t> betas, qr_ranks, ranks;
  std::vector<tts::DBuf<char>> cores;
  int32_t dtype = TT_DTYPE_F64;
  std::vector<std::vector<double>> sigma;
  std::vector<double> tail;
  std::vector<double> bond_delta;
  double ms[TT_NUM_STAGES] = {};
  int32_t ftt_p = 0;        // fiber-trie FastTT result: the p used (0 otherwise)
  int64_t ftt_fibers = 0;   // and its number of nonzero p-fibers
  std::unique_ptr<tts::SliceOut> slice;  // bond-2 Gram slice result (tt_sparse_gram_slice)
};

namespace tts {
namespace {

struct Events {
  hipEvent_t e[TT_NUM_STAGES + 1] = {};
  Events() {
    for (auto& x : e) TTS_HIP(hipEventCreate(&x));
  }
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

void sync_status(DevStatus* d_st, hipStream_t s) {
  read_back(host_status(), d_st, 1, s);
}

// Exact sparse TT: ingest, sort, and parallel-vector rounding level by level.
//
// A level's host-side sizes are its column count, its group count beta and nnz(N_k).
// The careful pass reads them back as the level goes (up to two read-backs a level).
// The speculative pass reads every level's column count once, right after the sort
// (distinct suffixes of the sorted keys, k_level_counts), and sizes the rest by upper
// bounds (beta <= columns, nnz(N_k) <= entries), on the assumptions that no input
// value is an explicit zero, that no column is longer than kMaxLocal entries, and that
// beta fits the device-count leader sort (kSmallSortMax) where the column count does
// not already guarantee it (the grouping table then sized for that many).  Its kernels
// read the counts from the device and stay in bounds when an assumption fails; one
// read-back at the end checks them, and the stage is then redone carefully.  Returns
// false in that case.
bool sparse_stage_pass(tt_result_s* R, const int32_t* idx, const double* val, uint32_t nnz, const ModeInfo& mi,
                       int total_bits, bool keep, int key_bits, hipStream_t s, Events& ev, bool spec) {
  Allocator* al = &R->al;
  const int d = mi.d;
  DBuf<DevStatus> st(al, 1);
  TTS_HIP(hipMemsetAsync(st.get(), 0, sizeof(DevStatus), s));

  // a1: ingest
  DBuf<uint64_t> keys(al, nnz), vals(al, nnz);
  launch_ingest(idx, val, nnz, mi, keys.get(), vals.get(), st.get(), s);
  // the careful pass reads the status back here; the speculative one assumes no
  // explicit zeros and checks the status with its first read-back
  uint32_t kept = nnz;
  if (!spec) {
    sync_status(st.get(), s);
    kept = nnz - host_status()->dropped;
    const DevStatus* h = host_status();
    if (h->err & kErrIndex) fail(TT_ERR_INDEX, "a coordinate is outside its mode range");
    if (h->err & kErrNonfinite) fail(TT_ERR_NONFINITE, "a value is NaN or infinite");
    if (kept == 0) fail(TT_ERR_EMPTY, "no nonzero left after dropping explicit zeros");
  }
  R->nnz = kept;
  TTS_HIP(hipEventRecord(ev.e[1], s));

  // a2: one global stable sort by packed key; dropped entries (key ~0) go last
  {
    DBuf<uint64_t> kt(al, nnz), vt(al, nnz);
    const int sort_bits = total_bits + (kept < nnz ? 1 : 0);
    if (radix_sort_pairs_pp(al, keys.get(), vals.get(), kt.get(), vt.get(), nnz, sort_bits, s)) {
      keys.swap(kt);
      vals.swap(vt);
    }
  }
  TTS_HIP(hipEventRecord(ev.e[2], s));

  // every level's column count at once (speculative pass)
  std::vector<uint32_t> ncols_h(d + 1, 0);
  DBuf<uint32_t> lv(al, 4 * static_cast<size_t>(d));  // per level: columns, beta, nnz(N_k)
  if (spec) {
    const size_t nc = (static_cast<size_t>(d) + 1) * kLevelCountCopies;
    DBuf<uint32_t> cnt(al, nc);
    TTS_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(uint32_t) * nc, s));
    launch_level_counts(keys.get(), kept, mi, cnt.get(), st.get(), s);
    std::vector<uint32_t> cnt_h(nc, 0);
    Readback rb(s);
    rb.add(cnt_h.data(), cnt.get(), sizeof(uint32_t) * nc);
    rb.add(host_status(), st.get(), sizeof(DevStatus));
    rb.sync();
    for (int k = 0; k <= d; ++k)
      for (uint32_t c = 0; c < kLevelCountCopies; ++c) ncols_h[k] += cnt_h[k * kLevelCountCopies + c];
    const DevStatus* h = host_status();
    if (h->err & kErrIndex) fail(TT_ERR_INDEX, "a coordinate is outside its mode range");
    if (h->err & kErrNonfinite) fail(TT_ERR_NONFINITE, "a value is NaN or infinite");
    if (h->dropped) {
      logf("speculative sizes do not hold (%u explicit zeros among the nonzeros); redone carefully", h->dropped);
      return false;
    }
    if (h->err & kErrDuplicate) fail(TT_ERR_DUPLICATE, "a coordinate appears twice among the nonzeros");
  }

  // a3..a7: levels
  DBuf<uint64_t> ekey = std::move(keys);
  DBuf<uint32_t> erho;
  DBuf<double> evals;
  const double* evp = reinterpret_cast<const double*>(vals.get());
  uint32_t nE = kept;
  R->lev.clear();
  R->lev.resize(d - 1);
  R->betas.assign(d + 1, 1);
  std::vector<uint32_t> caps(d, 0);
  logf("sparse stage: %u nonzeros kept of %u, %d modes%s", kept, nnz, d, spec ? " (sizes read once)" : "");
  for (int k = 1; k <= d - 1; ++k) {
    const double t_level = host_ms();
    const int kidx = k;           // first suffix mode, 0-based
    const int sh = static_cast<int>(mi.bits[k - 1]);
    const bool level1 = (k == 1);
    uint32_t* d_ncols = spec ? lv.get() + 4 * k - 4 : &st.get()->ncols;
    uint32_t* d_beta = spec ? lv.get() + 4 * k - 3 : &st.get()->beta;
    uint32_t* d_nnz = spec ? lv.get() + 4 * k - 2 : &st.get()->nnz_n;
    DBuf<uint32_t> flag, pos, col_start(al, static_cast<size_t>(nE) + 1);
    if (spec && !level1 && nE <= kColsSmallMax) {
      // small level of a speculative pass (never the long-column path): one workgroup
      launch_columns_small(ekey.get(), nE, sh, k - 1, col_start.get(), d_ncols, st.get(), s);
    } else if (spec && starts_tiles(nE) <= kStartsMaxTiles) {
      // a speculative pass needs no flag arrays (the long-column path is the careful
      // pass's)
      const uint32_t nt = starts_tiles(nE);
      DBuf<uint32_t> part(al, nt);
      DBuf<double> norm_part;
      if (level1) norm_part.reset(al, nt);
      launch_starts(ekey.get(), nE, sh, level1, level1 ? -1 : k - 1, evp, part.get(), norm_part.get(),
                    col_start.get(), d_ncols, st.get(), s);
      if (level1) launch_norm_final(norm_part.get(), nt, st.get(), s);
    } else {
      flag.reset(al, nE);
      pos.reset(al, nE);
      DBuf<double> norm_part;
      if (level1) norm_part.reset(al, norm_partials_count(nE));
      launch_col_flags(ekey.get(), nE, sh, level1, level1 ? -1 : k - 1, evp, flag.get(), norm_part.get(),
                       st.get(), s);
      exclusive_scan_u32(al, flag.get(), pos.get(), nE, d_ncols, s);
      launch_col_starts(flag.get(), pos.get(), nE, col_start.get(), d_ncols, s);
      if (level1) launch_norm_final(norm_part.get(), norm_partials_count(nE), st.get(), s);
    }
    uint32_t ncols;
    bool longcol = false;
    if (!spec) {
      sync_status(st.get(), s);
      const DevStatus hs = *host_status();
      if (level1) {
        if (hs.err & kErrDuplicate) fail(TT_ERR_DUPLICATE, "a coordinate appears twice among the nonzeros");
        R->norm = std::sqrt(hs.norm2);
      }
      ncols = hs.ncols;
      longcol = !level1 && ((hs.longmask >> (k - 1)) & 1ull);
    } else {
      ncols = ncols_h[k];
    }
    bool sort_rows = !level1;
    if (longcol) {
      // long columns: order entries by (column, rho) with one composite sort
      const uint64_t maxrho = static_cast<uint64_t>(R->betas[k - 1]) * mi.n[k - 1];
      const int rbits = static_cast<int>(bits_for(maxrho));
      const int cbits = static_cast<int>(bits_for(ncols));
      if (rbits + cbits > 64) fail(TT_ERR_TOO_LARGE, "composite (column, row) key exceeds 64 bits");
      DBuf<uint64_t> ck(al, nE), cv(al, nE), ckt(al, nE), cvt(al, nE);
      launch_make_composite(flag.get(), pos.get(), erho.get(), nE, rbits, ck.get(), cv.get(), s);
      if (radix_sort_pairs_pp(al, ck.get(), cv.get(), ckt.get(), cvt.get(), nE, rbits + cbits, s)) {
        ck.swap(ckt);
        cv.swap(cvt);
      }
      DBuf<uint64_t> ek2(al, nE);
      DBuf<uint32_t> er2(al, nE);
      DBuf<double> ev2(al, nE);
      launch_permute_entries(cv.get(), nE, ekey.get(), erho.get(), evp, ek2.get(), er2.get(), ev2.get(), s);
      ekey = std::move(ek2);
      erho = std::move(er2);
      evals = std::move(ev2);
      evp = evals.get();
      sort_rows = false;
    }
    flag.release();
    // a4: canonicalise
    DBuf<uint32_t> crho(al, nE);
    DBuf<double> cval(al, nE), cols(al, ncols);
    DBuf<uint64_t> colhash(al, ncols), colsuf(al, ncols), rmkey(al, ncols);
    // a5's hash table and group ids, cleared by the canonicalisation kernel, with at
    // least twice as many slots as groups: twice the columns, or on a speculative pass
    // twice the most groups it allows (kSmallSortMax), probes then bounded by
    // kSpecMaxProbe (an overflow fails the speculation)
    const bool small_table = spec && ncols > kSmallSortMax;
    const uint32_t tcols = small_table ? kSmallSortMax : ncols;
    uint32_t tsize = 1;
    while (tsize < 2u * tcols + 2u) tsize <<= 1;
    DBuf<uint64_t> table(al, tsize), slotmin(al, tsize);
    DBuf<uint32_t> slot_gid(al, tsize);
    CanonArgs ca{};
    ca.ekey = ekey.get();
    ca.erho = level1 ? nullptr : erho.get();
    ca.ev = evp;
    ca.col_start = col_start.get();
    ca.ncols = ncols;
    ca.sh = sh;
    ca.rho_mask = (mi.bits[0] >= 64) ? ~0ull : ((1ull << mi.bits[0]) - 1ull);
    ca.kidx = kidx;
    ca.sort_rows = sort_rows;
    ca.snap = (key_bits >= 1 && key_bits <= 51) ? 52 - key_bits : 0;
    ca.crho = crho.get();
    ca.cval = cval.get();
    ca.colhash = colhash.get();
    ca.cols = cols.get();
    ca.colsuf = colsuf.get();
    ca.rmkey = rmkey.get();
    ca.table = table.get();
    ca.slotmin = slotmin.get();
    ca.tsize = tsize;
    ca.slot_gid = slot_gid.get();
    // levels with long columns and few columns: a workgroup per column
    launch_canon(ca, mi, st.get(), longcol && ncols <= 16384, s);
    // a5: group
    DBuf<uint32_t> slot(al, ncols), isrep(al, ncols);
    launch_group(colhash.get(), crho.get(), cval.get(), col_start.get(), rmkey.get(), ncols, table.get(),
                 slotmin.get(), tsize - 1, small_table ? kSpecMaxProbe : tsize,
                 small_table ? &st.get()->table_over : nullptr, slot.get(), isrep.get(), s);
    DBuf<uint32_t> reppos(al, ncols);
    int rm_bits = 0;
    for (int j = kidx; j < d; ++j) rm_bits += static_cast<int>(mi.bits[j]);
    // Up to kSmallSortMax groups (the common case) the leaders are ordered without
    // knowing beta on the host, in one workgroup that counts and lists the groups
    // itself (on a speculative pass from the grouping table, on a careful one from the
    // columns' flags up to kLeaderListMax columns) or reads the count from the device;
    // beta and nnz(N_k) come back in one read-back.
    // Beyond that the leaders are sorted again with the device-wide radix sort.
    const uint32_t cap = std::min<uint32_t>(ncols, kSmallSortMax);
    caps[k] = cap;
    DBuf<uint64_t> lkey, lslot, lss(al, cap);
    DBuf<uint32_t> nlen, npos(al, cap);
    LeaderArgs la{};
    if (spec && tsize <= kLeaderTableMax) {
      // every group owns one slot of the (small) table: the list comes from there
      la.tscan = 1;
      la.tsize = tsize;
      la.slotmin = slotmin.get();
    } else if (ncols <= kLeaderListMax) {
      la.isrep = isrep.get();
      la.reppos = reppos.get();
      la.slot = slot.get();
      la.slotmin = slotmin.get();
      la.ncols = ncols;
    } else {
      exclusive_scan_u32(al, isrep.get(), reppos.get(), ncols, d_beta, s);
      lkey.reset(al, cap);
      lslot.reset(al, cap);
      launch_rep_list(isrep.get(), reppos.get(), slot.get(), slotmin.get(), ncols, cap, lkey.get(), lslot.get(), s);
      la.lkey = lkey.get();
      la.lslot = lslot.get();
    }
    la.d_beta = d_beta;
    la.cap = cap;
    la.nbits = rm_bits;
    la.table = table.get();
    la.col_start = col_start.get();
    la.lss = lss.get();
    la.slot_gid = slot_gid.get();
    la.npos = npos.get();
    la.d_nnz = d_nnz;
    launch_leaders(la, s);
    // beta, nnz(N_k): exact (careful pass) or upper bounds (speculative pass: checked
    // at the end, beta <= cap assumed)
    uint32_t beta = cap, nnz_n = nE;
    if (!spec) {
      sync_status(st.get(), s);
      beta = host_status()->beta;
      if (static_cast<uint64_t>(beta) * (k < d ? mi.n[k] : 1) > static_cast<uint64_t>(INT32_MAX))
        fail(TT_ERR_TOO_LARGE, "rank times mode size exceeds 2^31");
      if (beta > cap) {
        lkey.reset(al, beta);
        lslot.reset(al, beta);
        launch_rep_list(isrep.get(), reppos.get(), slot.get(), slotmin.get(), ncols, beta, lkey.get(), lslot.get(),
                        s);
        {
          DBuf<uint64_t> kt(al, beta), vt(al, beta);
          if (radix_sort_pairs_pp(al, lkey.get(), lslot.get(), kt.get(), vt.get(), beta, rm_bits, s)) {
            lkey.swap(kt);
            lslot.swap(vt);
          }
        }
        lss = std::move(lslot);
        nlen.reset(al, beta);
        npos.reset(al, beta);
        launch_group_ids(lss.get(), beta, nullptr, beta, table.get(), col_start.get(), slot_gid.get(), nlen.get(),
                         s);
        exclusive_scan_u32(al, nlen.get(), npos.get(), beta, d_nnz, s);
        sync_status(st.get(), s);
      }
      nnz_n = host_status()->nnz_n;
    }
    LevelData& L = R->lev[k - 1];
    L.ncols = ncols;
    L.beta = beta;
    L.nnz_n = nnz_n;
    R->betas[k] = beta;
    // a6: N_k
    L.colptr.reset(al, static_cast<size_t>(beta) + 1);
    L.row.reset(al, nnz_n);
    L.val.reset(al, nnz_n);
    // a7: next level (or the last core), in the same launch
    EmitArgs ea{};
    ea.lss = lss.get();
    ea.bmax = beta;
    ea.d_beta = d_beta;
    ea.d_nnz = d_nnz;
    ea.table = table.get();
    ea.col_start = col_start.get();
    ea.npos = npos.get();
    ea.crho = crho.get();
    ea.cval = cval.get();
    ea.colptr = L.colptr.get();
    ea.nrow = L.row.get();
    ea.nval = L.val.get();
    ea.ncols = ncols;
    ea.slot = slot.get();
    ea.slot_gid = slot_gid.get();
    ea.colsuf = colsuf.get();
    ea.cols = cols.get();
    ea.kidx = kidx;
    ea.last = (k == d - 1);
    if (keep) {
      L.col.reset(al, ncols);
      L.g.reset(al, ncols);
      L.s.reset(al, ncols);
      ea.out_col = L.col.get();
      ea.out_g = L.g.get();
      ea.out_s = L.s.get();
    }
    DBuf<uint64_t> nk;
    DBuf<uint32_t> nr;
    DBuf<double> nv;
    if (!ea.last) {
      nk.reset(al, ncols);
      nr.reset(al, ncols);
      nv.reset(al, ncols);
      ea.next_ekey = nk.get();
      ea.next_rho = nr.get();
      ea.next_v = nv.get();
    } else {
      const size_t sz = static_cast<size_t>(beta) * mi.n[d - 1];
      R->last_exact.reset(al, sz);
      TTS_HIP(hipMemsetAsync(R->last_exact.get(), 0, sizeof(double) * sz, s));
      ea.last_core = R->last_exact.get();
    }
    launch_emit(ea, mi, s);
    if (!spec)
      logf("level %d: %u entries, %u columns, beta %u, nnz(N_k) %u, %.3f ms (host)", k, nE, ncols, beta, nnz_n,
           host_ms() - t_level);
    if (!ea.last) {
      ekey = std::move(nk);
      erho = std::move(nr);
      evals = std::move(nv);
      evp = evals.get();
      vals.release();
      nE = ncols;
    }
  }
  if (spec) {
    // one read-back for every level's counts; the assumptions are checked here
    std::vector<uint32_t> lh(4 * static_cast<size_t>(d), 0);
    Readback rb(s);
    rb.add(lh.data(), lv.get(), sizeof(uint32_t) * 4 * d);
    rb.add(host_status(), st.get(), sizeof(DevStatus));
    rb.sync();
    const DevStatus hs = *host_status();
    bool ok = true;
    if (hs.table_over) {
      logf("speculative sizes do not hold (a grouping table overflowed); redone carefully");
      return false;
    }
    uint32_t ne = kept;
    for (int k = 1; k <= d - 1; ++k) {
      const uint32_t nc = lh[4 * k - 4], beta = lh[4 * k - 3], nz = lh[4 * k - 2];
      const bool fits = nc == ncols_h[k] && beta >= 1 && beta <= caps[k] && nz <= ne &&
                        !(k >= 2 && ((hs.longmask >> (k - 1)) & 1ull)) &&
                        static_cast<uint64_t>(beta) * (k < d ? mi.n[k] : 1) <= static_cast<uint64_t>(INT32_MAX);
      if (!fits) {
        ok = false;
        logf("level %d: speculative sizes do not hold (columns %u / %u, beta %u, cap %u); redone carefully", k, nc,
             ncols_h[k], beta, caps[k]);
        break;
      }
      LevelData& L = R->lev[k - 1];
      L.beta = beta;
      L.nnz_n = nz;
      R->betas[k] = beta;
      logf("level %d: %u entries, %u columns, beta %u, nnz(N_k) %u", k, ne, nc, beta, nz);
      ne = nc;
    }
    if (!ok) return false;
    R->norm = std::sqrt(hs.norm2);
  }
  TTS_HIP(hipEventRecord(ev.e[3], s));
  return true;
}

void sparse_stage(tt_result_s* R, const int32_t* idx, const double* val, uint32_t nnz, const ModeInfo& mi,
                  int total_bits, bool keep, int key_bits, hipStream_t s, Events& ev) {
  // speculate only when the allocations are the library's own and unbudgeted (the
  // upper bounds hold more memory for the duration of the call)
  const bool spec = R->al.budget == 0 && !R->al.hook_alloc;
  if (!sparse_stage_pass(R, idx, val, nnz, mi, total_bits, keep, key_bits, s, ev, spec))
    sparse_stage_pass(R, idx, val, nnz, mi, total_bits, keep, key_bits, s, ev, false);
}

}  // namespace
}  // namespace tts

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
using namespace tts;

extern "C" {

void tt_options_default(tt_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = TT_FP64;
}

const char* tt_status_string(tt_status s) {
  switch (s) {
    case TT_OK: return "TT_OK";
    case TT_ERR_ARG: return "TT_ERR_ARG";
    case TT_ERR_INDEX: return "TT_ERR_INDEX";
    case TT_ERR_DUPLICATE: return "TT_ERR_DUPLICATE";
    case TT_ERR_NONFINITE: return "TT_ERR_NONFINITE";
    case TT_ERR_EMPTY: return "TT_ERR_EMPTY";
    case TT_ERR_TOO_LARGE: return "TT_ERR_TOO_LARGE";
    case TT_ERR_NOMEM: return "TT_ERR_NOMEM";
    case TT_ERR_DEVICE: return "TT_ERR_DEVICE";
  }
  return "TT_ERR_UNKNOWN";
}

const char* tt_last_error(void) { return g_last_error.c_str(); }

tt_status tt_sparse_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                              double eps, const tt_options* opt, void* stream, tt_result* out) {
  if (!out) {
    set_error("out is NULL");
    return TT_ERR_ARG;
  }
  *out = nullptr;
  tt_options o;
  tt_options_default(&o);
  if (opt) o = *opt;
  // host-side argument checks, before any launch
  std::string why;
  if (d < 2 || d > TT_MAX_D) why = "d must be in [2, 64]";
  else if (!dims) why = "dims is NULL";
  else if (nnz < 0 || nnz >= (int64_t(1) << 31)) why = "nnz must be in [0, 2^31)";
  else if (nnz > 0 && (!idx || !val)) why = "idx/val is NULL";
  else if (!(eps >= 0.0 && eps < 1.0)) why = "eps must satisfy 0 <= eps < 1";
  else if (o.precision < TT_FP64 || o.precision > TT_BF16_FP32ACC) why = "unknown precision";
  else if (o.max_rank < 0) why = "max_rank must be >= 0";
  else if (o.key_bits < 0 || o.key_bits > 52) why = "key_bits must be in [0, 52]";
  else if ((o.alloc == nullptr) != (o.free == nullptr)) why = "alloc and free hooks must be given together";
  if (why.empty())
    for (int k = 0; k < d; ++k)
      if (dims[k] < 1 || dims[k] > INT32_MAX) why = "every n_k must be in [1, 2^31-1]";
  if (!why.empty()) {
    set_error(why);
    return TT_ERR_ARG;
  }
  ModeInfo mi{};
  mi.d = d;
  int total_bits = 0;
  for (int k = 0; k < d; ++k) {
    mi.n[k] = static_cast<uint32_t>(dims[k]);
    mi.bits[k] = bits_for(static_cast<uint64_t>(dims[k]));
    mi.off[k] = static_cast<uint32_t>(total_bits);
    total_bits += static_cast<int>(mi.bits[k]);
  }
  if (total_bits > 63) {
    set_error("packed coordinate needs more than 63 bits");
    return TT_ERR_TOO_LARGE;
  }
  if (nnz == 0) {
    set_error("no nonzero given");
    return TT_ERR_EMPTY;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  tt_result_s* R = nullptr;
  try {
    configure_pool_once();
    R = new tt_result_s();
    R->al.stream = s;
    R->al.hook_alloc = o.alloc;
    R->al.hook_free = o.free;
    R->al.ctx = o.alloc_ctx;
    R->al.budget = o.device_mem_budget;
    R->d = d;
    R->dims.assign(dims, dims + d);
    Events ev;
    TTS_HIP(hipEventRecord(ev.e[0], s));
    sparse_stage(R, idx, val, static_cast<uint32_t>(nnz), mi, total_bits, o.keep_intermediates != 0, o.key_bits, s,
                 ev);
    R->delta = eps * R->norm / std::sqrt(static_cast<double>(d - 1));
    RoundInput in{};
    in.d = d;
    in.dims = R->dims;
    in.betas = R->betas;
    in.eps = eps;
    in.delta = R->delta;
    in.norm = R->norm;
    in.max_rank = o.max_rank;
    in.dynamic_delta = o.dynamic_delta != 0;
    if (o.key_bits >= 1 && o.key_bits <= 51) in.snap_rel = (d - 1) * std::ldexp(1.0, -(o.key_bits + 1));
    in.precision = o.precision;
    for (int k = 1; k <= d - 1; ++k) {
      const LevelData& L = R->lev[k - 1];
      in.n_colptr.push_back(L.colptr.get());
      in.n_row.push_back(L.row.get());
      in.n_val.push_back(L.val.get());
      in.n_nnz.push_back(L.nnz_n);
    }
    in.last_core = R->last_exact.get();
    if (o.sparse_only) {
      densify_exact_cores(R->al, in, R->cores, s);
      R->ranks = R->betas;
      R->dtype = TT_DTYPE_F64;
      TTS_HIP(hipEventRecord(ev.e[4], s));
      TTS_HIP(hipEventRecord(ev.e[5], s));
    } else {
      RoundOutput ro;
      round_tt(R->al, in, ro, s, ev.e[4]);
      R->qr_ranks = ro.qr_ranks;
      R->ranks = ro.ranks;
      R->cores = std::move(ro.cores);
      R->dtype = ro.dtype;
      R->sigma = std::move(ro.sigma);
      R->tail = std::move(ro.tail);
      R->bond_delta = std::move(ro.bond_delta);
      R->rounded = 1;
      TTS_HIP(hipEventRecord(ev.e[5], s));
    }
    TTS_HIP(hipEventRecord(ev.e[6], s));
    TTS_HIP(hipEventSynchronize(ev.e[6]));
    for (int i = 0; i < TT_NUM_STAGES - 1; ++i) {
      float ms = 0.f;
      TTS_HIP(hipEventElapsedTime(&ms, ev.e[i], ev.e[i + 1]));
      R->ms[i] = ms;
    }
    float tot = 0.f;
    TTS_HIP(hipEventElapsedTime(&tot, ev.e[0], ev.e[6]));
    R->ms[TT_NUM_STAGES - 1] = tot;
    if (!o.keep_intermediates) {
      for (auto& L : R->lev) {
        L.colptr.release();
        L.row.release();
        L.val.release();
      }
    }
    *out = R;
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return TT_ERR_NOMEM;
  }
}

tt_status tt_fasttt_decompose(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                              double eps, int32_t p, const tt_options* opt, void* stream, tt_result* out) {
  if (!out) {
    set_error("out is NULL");
    return TT_ERR_ARG;
  }
  *out = nullptr;
  tt_options o;
  tt_options_default(&o);
  if (opt) o = *opt;
  std::string why;
  if (d < 2 || d > TT_MAX_D) why = "d must be in [2, 64]";
  else if (!dims) why = "dims is NULL";
  else if (nnz < 0 || nnz >= (int64_t(1) << 31)) why = "nnz must be in [0, 2^31)";
  else if (nnz > 0 && (!idx || !val)) why = "idx/val is NULL";
  else if (!(eps >= 0.0 && eps < 1.0)) why = "eps must satisfy 0 <= eps < 1";
  else if (p < 0 || p > d) why = "p must be in [0, d] (0: chosen by Algorithm 9)";
  else if (o.precision < TT_FP64 || o.precision > TT_BF16_FP32ACC) why = "unknown precision";
  else if (o.max_rank < 0) why = "max_rank must be >= 0";
  else if (o.key_bits || o.keep_intermediates)
    why = "key_bits and keep_intermediates apply to tt_sparse_decompose only";
  else if ((o.alloc == nullptr) != (o.free == nullptr)) why = "alloc and free hooks must be given together";
  if (why.empty())
    for (int k = 0; k < d; ++k)
      if (dims[k] < 1 || dims[k] > INT32_MAX) why = "every n_k must be in [1, 2^31-1]";
  if (!why.empty()) {
    set_error(why);
    return TT_ERR_ARG;
  }
  if (nnz == 0) {
    set_error("no nonzero given");
    return TT_ERR_EMPTY;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  tt_result_s* R = nullptr;
  try {
    configure_pool_once();
    R = new tt_result_s();
    R->al.stream = s;
    R->al.hook_alloc = o.alloc;
    R->al.hook_free = o.free;
    R->al.ctx = o.alloc_ctx;
    R->al.budget = o.device_mem_budget;
    R->d = d;
    R->dims.assign(dims, dims + d);
    Events ev;
    TTS_HIP(hipEventRecord(ev.e[0], s));
    if (p == 0) p = ftt_select_p(&R->al, idx, val, static_cast<uint32_t>(nnz), R->dims, nullptr, s);
    TTS_HIP(hipEventRecord(ev.e[1], s));
    TTS_HIP(hipEventRecord(ev.e[2], s));
    FttExact ex;
    ftt_exact(&R->al, idx, val, static_cast<uint32_t>(nnz), R->dims, p, ex, s);
    TTS_HIP(hipEventRecord(ev.e[3], s));
    R->nnz = ex.nnz;
    R->norm = ex.norm;
    R->betas = ex.ranks;
    R->ftt_p = p;
    R->ftt_fibers = ex.fibers;
    R->delta = eps * ex.norm / (std::sqrt(static_cast<double>(p - 1)) + std::sqrt(static_cast<double>(d - p)));
    if (o.sparse_only) {
      R->cores = std::move(ex.cores);
      R->ranks = R->betas;
      R->dtype = TT_DTYPE_F64;
      TTS_HIP(hipEventRecord(ev.e[4], s));
      TTS_HIP(hipEventRecord(ev.e[5], s));
    } else {
      RoundOutput ro;
      std::vector<int64_t> r = ex.ranks;
      ftt_round(&R->al, R->dims, p, eps, ex.norm, o.max_rank, o.dynamic_delta != 0, o.precision, ex.cores, r, ro,
                ev.e[4], s);
      R->qr_ranks = ro.qr_ranks;
      R->ranks = ro.ranks;
      R->cores = std::move(ex.cores);
      R->sigma = std::move(ro.sigma);
      R->tail = std::move(ro.tail);
      R->bond_delta = std::move(ro.bond_delta);
      R->dtype = ro.dtype;
      R->rounded = 1;
      TTS_HIP(hipEventRecord(ev.e[5], s));
    }
    TTS_HIP(hipEventRecord(ev.e[6], s));
    TTS_HIP(hipEventSynchronize(ev.e[6]));
    for (int i = 0; i < TT_NUM_STAGES - 1; ++i) {
      float ms = 0.f;
      TTS_HIP(hipEventElapsedTime(&ms, ev.e[i], ev.e[i + 1]));
      R->ms[i] = ms;
    }
    float tot = 0.f;
    TTS_HIP(hipEventElapsedTime(&tot, ev.e[0], ev.e[6]));
    R->ms[TT_NUM_STAGES - 1] = tot;
    *out = R;
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return TT_ERR_NOMEM;
  }
}

tt_status tt_sparse_gram_slice(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                               const tt_options* opt, void* stream, tt_result* out) {
  if (!out) {
    set_error("out is NULL");
    return TT_ERR_ARG;
  }
  *out = nullptr;
  tt_options o;
  tt_options_default(&o);
  if (opt) o = *opt;
  std::string why;
  if (d < 3 || d > TT_MAX_D) why = "d must be in [3, 64]";
  else if (!dims) why = "dims is NULL";
  else if (nnz < 0 || nnz >= (int64_t(1) << 31)) why = "nnz must be in [0, 2^31)";
  else if (nnz > 0 && (!idx || !val)) why = "idx/val is NULL";
  else if (o.precision < TT_FP64 || o.precision > TT_BF16_FP32ACC) why = "unknown precision";
  else if (o.max_rank || o.dynamic_delta || o.sparse_only)
    why = "max_rank, dynamic_delta and sparse_only do not apply to the Gram slice";
  else if (o.key_bits < 0 || o.key_bits > 52) why = "key_bits must be in [0, 52]";
  else if ((o.alloc == nullptr) != (o.free == nullptr)) why = "alloc and free hooks must be given together";
  if (why.empty())
    for (int k = 0; k < d; ++k)
      if (dims[k] < 1 || dims[k] > INT32_MAX) why = "every n_k must be in [1, 2^31-1]";
  if (why.empty() && dims[0] > 208) why = "the Gram slice supports n_1 <= 208";
  if (!why.empty()) {
    set_error(why);
    return TT_ERR_ARG;
  }
  ModeInfo mi{};
  mi.d = d;
  int total_bits = 0;
  for (int k = 0; k < d; ++k) {
    mi.n[k] = static_cast<uint32_t>(dims[k]);
    mi.bits[k] = bits_for(static_cast<uint64_t>(dims[k]));
    mi.off[k] = static_cast<uint32_t>(total_bits);
    total_bits += static_cast<int>(mi.bits[k]);
  }
  if (total_bits > 63) {
    set_error("packed coordinate needs more than 63 bits");
    return TT_ERR_TOO_LARGE;
  }
  if (nnz == 0) {
    set_error("no nonzero given");
    return TT_ERR_EMPTY;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  tt_result_s* R = nullptr;
  try {
    configure_pool_once();
    R = new tt_result_s();
    R->al.stream = s;
    R->al.hook_alloc = o.alloc;
    R->al.hook_free = o.free;
    R->al.ctx = o.alloc_ctx;
    R->al.budget = o.device_mem_budget;
    R->d = d;
    R->dims.assign(dims, dims + d);
    Events ev;
    TTS_HIP(hipEventRecord(ev.e[0], s));
    sparse_stage(R, idx, val, static_cast<uint32_t>(nnz), mi, total_bits, o.keep_intermediates != 0, o.key_bits, s,
                 ev);
    SliceInput in{};
    in.d = d;
    in.dims = R->dims;
    in.betas = R->betas;
    in.precision = o.precision;
    for (int k = 1; k <= d - 1; ++k) {
      const LevelData& L = R->lev[k - 1];
      in.n_colptr.push_back(L.colptr.get());
      in.n_row.push_back(L.row.get());
      in.n_val.push_back(L.val.get());
      in.n_nnz.push_back(L.nnz_n);
    }
    in.last_core = R->last_exact.get();
    R->slice = std::make_unique<SliceOut>();
    gram_slice(R->al, in, *R->slice, s);
    TTS_HIP(hipEventRecord(ev.e[4], s));
    TTS_HIP(hipEventRecord(ev.e[5], s));
    TTS_HIP(hipEventRecord(ev.e[6], s));
    TTS_HIP(hipEventSynchronize(ev.e[6]));
    for (int i = 0; i < TT_NUM_STAGES - 1; ++i) {
      float ms = 0.f;
      TTS_HIP(hipEventElapsedTime(&ms, ev.e[i], ev.e[i + 1]));
      R->ms[i] = ms;
    }
    float tot = 0.f;
    TTS_HIP(hipEventElapsedTime(&tot, ev.e[0], ev.e[6]));
    R->ms[TT_NUM_STAGES - 1] = tot;
    R->ranks = R->betas;
    if (!o.keep_intermediates) {
      for (auto& L : R->lev) {
        L.colptr.release();
        L.row.release();
        L.val.release();
      }
      R->last_exact.release();
    }
    *out = R;
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    if (R) {
      (void)hipStreamSynchronize(s);
      delete R;
    }
    return TT_ERR_NOMEM;
  }
}

tt_status tt_get_slice_bond1(tt_result r, int64_t* m, const double** q1, const double** r1, const double** sigma) {
  if (!r || !r->slice) {
    set_error("not a Gram slice result");
    return TT_ERR_ARG;
  }
  const SliceOut& o = *r->slice;
  if (m) *m = o.m;
  if (q1) *q1 = o.q1.get();
  if (r1) *r1 = o.r1.get();
  if (sigma) *sigma = o.sigma1.data();
  return TT_OK;
}

tt_status tt_get_slice_x2(tt_result r, int64_t* nblocks, const int64_t** slot_ptr, const int32_t** blk_col,
                          const void** vals, int32_t* dtype) {
  if (!r || !r->slice) {
    set_error("not a Gram slice result");
    return TT_ERR_ARG;
  }
  const SliceOut& o = *r->slice;
  if (nblocks) *nblocks = o.nblocks;
  if (slot_ptr) *slot_ptr = o.slot_ptr.get();
  if (blk_col) *blk_col = o.blk_col.get();
  if (vals) *vals = o.x2.get();
  if (dtype) *dtype = o.x2_dtype;
  return TT_OK;
}

tt_status tt_get_slice_gram(tt_result r, const double** gram, double* wnorm2, int64_t* npairs, double* flops,
                            double* host_ms) {
  if (!r || !r->slice) {
    set_error("not a Gram slice result");
    return TT_ERR_ARG;
  }
  const SliceOut& o = *r->slice;
  if (gram) *gram = o.gram.get();
  if (wnorm2) *wnorm2 = o.wnorm2;
  if (npairs) *npairs = o.npairs;
  if (flops) *flops = o.gram_flops;
  if (host_ms)
    for (int i = 0; i < 5; ++i) host_ms[i] = o.ms[i];
  return TT_OK;
}

tt_status tt_get_fasttt_info(tt_result r, int32_t* p, int64_t* fibers) {
  if (!r) return TT_ERR_ARG;
  if (r->ftt_p == 0) {
    set_error("not a fiber-trie FastTT result");
    return TT_ERR_ARG;
  }
  if (p) *p = r->ftt_p;
  if (fibers) *fibers = r->ftt_fibers;
  return TT_OK;
}

tt_status tt_fasttt_select_p(int32_t d, const int64_t* dims, int64_t nnz, const int32_t* idx, const double* val,
                             double* costs, int32_t* p, void* stream) {
  std::string why;
  if (d < 2 || d > TT_MAX_D) why = "d must be in [2, 64]";
  else if (!dims || !p) why = "dims/p is NULL";
  else if (nnz <= 0 || nnz >= (int64_t(1) << 31)) why = "nnz must be in [1, 2^31)";
  else if (!idx || !val) why = "idx/val is NULL";
  if (why.empty())
    for (int k = 0; k < d; ++k)
      if (dims[k] < 1 || dims[k] > INT32_MAX) why = "every n_k must be in [1, 2^31-1]";
  if (!why.empty()) {
    set_error(why);
    return TT_ERR_ARG;
  }
  try {
    configure_pool_once();
    Allocator al;
    al.stream = static_cast<hipStream_t>(stream);
    std::vector<int64_t> dv(dims, dims + d);
    std::vector<double> c;
    *p = ftt_select_p(&al, idx, val, static_cast<uint32_t>(nnz), dv, &c, al.stream);
    if (costs) std::copy(c.begin(), c.end(), costs);
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

void tt_free(tt_result r) {
  if (!r) return;
  // The cores may still be read by the caller's work on any stream: wait for the
  // device, then return the blocks to the cache of the null stream.
  (void)hipDeviceSynchronize();
  r->al.stream = nullptr;
  delete r;
}

tt_status tt_get_ranks(tt_result r, int64_t* ranks) {
  if (!r || !ranks) return TT_ERR_ARG;
  std::copy(r->ranks.begin(), r->ranks.end(), ranks);
  return TT_OK;
}

tt_status tt_get_sparse_ranks(tt_result r, int64_t* betas, int64_t* qr_ranks) {
  if (!r) return TT_ERR_ARG;
  if (betas) std::copy(r->betas.begin(), r->betas.end(), betas);
  if (qr_ranks) {
    if (!r->rounded) return TT_ERR_ARG;
    std::copy(r->qr_ranks.begin(), r->qr_ranks.end(), qr_ranks);
  }
  return TT_OK;
}

tt_status tt_get_core(tt_result r, int32_t k, const void** dev_ptr, int32_t* dtype) {
  if (!r || !dev_ptr || k < 1 || k > r->d) return TT_ERR_ARG;
  if (r->cores.size() != static_cast<size_t>(r->d)) {
    set_error("cores not available (sparse_only result too large to densify)");
    return TT_ERR_TOO_LARGE;
  }
  *dev_ptr = r->cores[k - 1].get();
  if (dtype) *dtype = r->dtype;
  return TT_OK;
}

tt_status tt_get_info(tt_result r, int64_t* host_info, double* norm, double* delta) {
  if (!r) return TT_ERR_ARG;
  if (host_info) {
    host_info[0] = r->nnz;
    host_info[1] = r->rounded;
    host_info[2] = r->d;
  }
  if (norm) *norm = r->norm;
  if (delta) *delta = r->delta;
  return TT_OK;
}

tt_status tt_get_sigma(tt_result r, int32_t b, int64_t* count, const double** host_sigma, double* tail) {
  if (!r || b < 1 || b >= r->d) return TT_ERR_ARG;
  if (!r->rounded) {
    set_error("no singular values: sparse_only result");
    return TT_ERR_ARG;
  }
  if (count) *count = static_cast<int64_t>(r->sigma[b - 1].size());
  if (host_sigma) *host_sigma = r->sigma[b - 1].data();
  if (tail) *tail = r->tail[b - 1];
  return TT_OK;
}

tt_status tt_get_bond_delta(tt_result r, int32_t b, double* delta) {
  if (!r || b < 1 || b >= r->d || !delta) return TT_ERR_ARG;
  if (!r->rounded) {
    set_error("no truncation thresholds: sparse_only result");
    return TT_ERR_ARG;
  }
  *delta = r->bond_delta[b - 1];
  return TT_OK;
}

tt_status tt_get_times(tt_result r, double* host_ms) {
  if (!r || !host_ms) return TT_ERR_ARG;
  std::copy(r->ms, r->ms + TT_NUM_STAGES, host_ms);
  return TT_OK;
}

tt_status tt_get_level(tt_result r, int32_t k, int64_t* ncols, int64_t* beta, const int64_t** col, const int32_t** g,
                       const double** s, const int64_t** n_colptr, const int32_t** n_row, const double** n_val) {
  if (!r || k < 1 || k >= r->d) return TT_ERR_ARG;
  if (r->lev.size() < static_cast<size_t>(k)) {
    set_error("no sparse-stage levels in this result (fiber-trie FastTT)");
    return TT_ERR_ARG;
  }
  const LevelData& L = r->lev[k - 1];
  if (ncols) *ncols = L.ncols;
  if (beta) *beta = L.beta;
  const bool have = L.g.get() != nullptr || L.ncols == 0;
  if ((col || g || s || n_colptr || n_row || n_val) && !have) {
    set_error("level data not kept (set keep_intermediates)");
    return TT_ERR_ARG;
  }
  if (col) *col = L.col.get();
  if (g) *g = L.g.get();
  if (s) *s = L.s.get();
  if (n_colptr) *n_colptr = L.colptr.get();
  if (n_row) *n_row = L.row.get();
  if (n_val) *n_val = L.val.get();
  return TT_OK;
}

tt_status tt_cache_trim(uint64_t* bytes_released) {
  try {
    const uint64_t b = cache_trim();
    if (bytes_released) *bytes_released = b;
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

tt_status tt_get_level_sizes(tt_result r, int32_t k, int64_t* sizes) {
  if (!r || !sizes || k < 1 || k >= r->d) {
    set_error("result, sizes or k invalid");
    return TT_ERR_ARG;
  }
  if (r->lev.size() < static_cast<size_t>(k)) {
    set_error("no sparse-stage levels in this result (fiber-trie FastTT)");
    return TT_ERR_ARG;
  }
  const LevelData& L = r->lev[k - 1];
  sizes[0] = L.ncols;
  sizes[1] = L.beta;
  sizes[2] = L.nnz_n;
  return TT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Kernel-family timer.
// ---------------------------------------------------------------------------
#include <mutex>

namespace tts {
namespace {
struct TimerState {
  std::mutex mu;
  std::string family;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<hipEvent_t> pool;
  double bytes = 0.0, flops = 0.0;
  int64_t launches = 0;
  // launches whose flops scale with a device count: (flops per unit, slot in dcount)
  std::vector<std::pair<double, int>> per_count;
  int32_t* dcount = nullptr;  // device copies of the counts (timer-owned)
  int dcount_cap = 0;
};
TimerState& timer_state() {
  static TimerState* t = new TimerState();
  return *t;
}
hipEvent_t pool_event(TimerState& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  TTS_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

KTimer::KTimer(const char* family, hipStream_t s, double bytes, double flops) {
  TimerState& t = timer_state();
  std::lock_guard<std::mutex> g(t.mu);
  if (t.family.empty() || t.family != family) return;
  s_ = s;
  hipEvent_t a = pool_event(t), b = pool_event(t);
  TTS_HIP(hipEventRecord(a, s));
  t.ev.emplace_back(a, b);
  slot_ = static_cast<int>(t.ev.size()) - 1;
  t.bytes += bytes;
  t.flops += flops;
  t.launches += 1;
  flops_ = flops;
}

void KTimer::flops_per_count(const int32_t* dev_count) {
  if (slot_ < 0 || !dev_count) return;
  count_ = dev_count;
}

KTimer::~KTimer() {
  if (slot_ < 0) return;
  TimerState& t = timer_state();
  std::lock_guard<std::mutex> g(t.mu);
  if (slot_ < static_cast<int>(t.ev.size())) (void)hipEventRecord(t.ev[slot_].second, s_);
  if (count_) {
    // keep a copy of the count, stream-ordered after the launch, for the read
    if (!t.dcount) {
      void* p = nullptr;
      if (hipMalloc(&p, sizeof(int32_t) * 65536) == hipSuccess) {
        t.dcount = static_cast<int32_t*>(p);
        t.dcount_cap = 65536;
      }
    }
    const int k = static_cast<int>(t.per_count.size());
    if (t.dcount && k < t.dcount_cap &&
        hipMemcpyAsync(t.dcount + k, count_, sizeof(int32_t), hipMemcpyDeviceToDevice, s_) == hipSuccess) {
      t.flops -= flops_;
      t.per_count.emplace_back(flops_, k);
    }
  }
}

}  // namespace tts

extern "C" tt_status tt_kernel_timer_start(const char* family) {
  tts::TimerState& t = tts::timer_state();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& p : t.ev) {
    t.pool.push_back(p.first);
    t.pool.push_back(p.second);
  }
  t.ev.clear();
  t.bytes = t.flops = 0.0;
  t.launches = 0;
  t.per_count.clear();
  t.family = family ? family : "";
  return TT_OK;
}

extern "C" tt_status tt_kernel_timer_read(double* total_ms, int64_t* launches, double* algo_bytes,
                                          double* algo_flops) {
  tts::TimerState& t = tts::timer_state();
  std::lock_guard<std::mutex> g(t.mu);
  double ms = 0.0;
  for (auto& p : t.ev) {
    if (hipEventSynchronize(p.second) != hipSuccess) return TT_ERR_DEVICE;
    float x = 0.f;
    if (hipEventElapsedTime(&x, p.first, p.second) != hipSuccess) return TT_ERR_DEVICE;
    ms += x;
  }
  double flops = t.flops;
  if (!t.per_count.empty()) {
    std::vector<int32_t> cnt(t.per_count.size());
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(cnt.data(), t.dcount, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return TT_ERR_DEVICE;
    for (size_t i = 0; i < cnt.size(); ++i) flops += t.per_count[i].first * cnt[t.per_count[i].second];
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = t.launches;
  if (algo_bytes) *algo_bytes = t.bytes;
  if (algo_flops) *algo_flops = flops;
  return TT_OK;
}
