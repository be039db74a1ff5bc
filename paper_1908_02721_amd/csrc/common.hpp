// Shared host/device helpers of libttsparse (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ttsparse.h"

namespace tts {

// ---------------------------------------------------------------------------
// Host-side error handling: internal code throws tts::Error, the C-ABI entry
// points catch it and turn it into a tt_status (nothing crosses the ABI).
// ---------------------------------------------------------------------------
struct Error {
  tt_status code;
  std::string msg;
};

[[noreturn]] void fail(tt_status s, const std::string& msg);
// Message returned by tt_last_error() on the calling thread.
void set_last_error(const std::string& msg);

#define TTS_HIP(x)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      ::tts::fail(TT_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define TTS_LAUNCH_CHECK() TTS_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Device memory: stream-ordered allocations from the caller's hooks or from the
// device's default pool, with an optional budget.
// ---------------------------------------------------------------------------
struct Allocator {
  hipStream_t stream = nullptr;
  void* (*hook_alloc)(size_t, void*) = nullptr;
  void (*hook_free)(void*, void*) = nullptr;
  void* ctx = nullptr;
  uint64_t budget = 0;
  uint64_t in_use = 0;
  uint64_t peak = 0;

  void* get(size_t bytes);
  void put(void* p, size_t bytes);
};

// Stream-ordered block cache shared by every allocation of the library.
void* cached_alloc(size_t bytes, hipStream_t s);
void cached_free(void* p, size_t bytes, hipStream_t s);
uint64_t cache_trim();  // frees every cached block after a device synchronisation

// Read-backs to the host go through a per-thread pinned buffer: a device-to-host copy
// into pageable memory is staged by the runtime and costs about 8 us more per round
// trip (measured: kernel + copy + synchronisation 22.8 us pageable, 14.7 us pinned).
// add() records a piece (device address 4-byte aligned, a multiple of 4 bytes);
// sync() launches one small kernel on the stream that writes the pending pieces into
// the buffer, waits for the stream and moves every piece to its destination.  The
// values read are those the device holds after all work enqueued before sync().
// One Readback at a time per thread.
class Readback {
 public:
  explicit Readback(hipStream_t s) : s_(s) {}
  ~Readback();
  Readback(const Readback&) = delete;
  Readback& operator=(const Readback&) = delete;
  void add(void* host, const void* dev, size_t bytes);
  void sync();

 private:
  struct Piece {
    void* host;
    const void* dev;
    size_t off, bytes;
  };
  hipStream_t s_;
  size_t off_ = 0;
  std::vector<Piece> pend_;
};
// One read-back of n values, waited for.
template <class T>
void read_back(T* host, const T* dev, size_t n, hipStream_t s) {
  Readback rb(s);
  rb.add(host, dev, sizeof(T) * n);
  rb.sync();
}

template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(Allocator* a, size_t n) { reset(a, n); }
  ~DBuf() { release(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { swap(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      swap(o);
    }
    return *this;
  }
  void reset(Allocator* a, size_t n) {
    release();
    al_ = a;
    n_ = n;
    p_ = n ? static_cast<T*>(a->get(n * sizeof(T))) : nullptr;
  }
  void release() {
    if (p_ && al_) al_->put(p_, n_ * sizeof(T));
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  void swap(DBuf& o) noexcept {
    std::swap(al_, o.al_);
    std::swap(p_, o.p_);
    std::swap(n_, o.n_);
  }

 private:
  Allocator* al_ = nullptr;
  T* p_ = nullptr;
  size_t n_ = 0;
};

// Live timing of one kernel family (see tt_kernel_timer_start).  Construct a
// KTimer around a launch: when the family is being timed, events are recorded on
// the launch's stream before and after it.
class KTimer {
 public:
  KTimer(const char* family, hipStream_t s, double bytes, double flops);
  ~KTimer();
  KTimer(const KTimer&) = delete;
  KTimer& operator=(const KTimer&) = delete;
  // The launch's flops are `flops` times the int32 the launch leaves at dev_count
  // (e.g. the sweeps an iteration ran), read when the timer is read.  Null: fixed.
  void flops_per_count(const int32_t* dev_count);

 private:
  int slot_ = -1;
  hipStream_t s_ = nullptr;
  double flops_ = 0.0;
  const int32_t* count_ = nullptr;
};

// Progress log on stderr, on when the environment has TTSPARSE_LOG=1 (read once):
// per level of the sparse stage and per bond of the sweeps, sizes, ranks and host
// milliseconds (each line is written after the step's own read-back).
bool log_on();
void logf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
double host_ms();  // monotonic host clock in milliseconds

inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  return static_cast<unsigned>(g == 0 ? 1 : g);
}

// ---------------------------------------------------------------------------
// Device helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned l = __lane_id();
  return (l == 0) ? 0ull : ((~0ull) >> (64 - l));
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
  const unsigned lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= static_cast<unsigned>(o)) x += y;
  }
  return x;
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Exclusive scan of one value per thread over a block of NT threads.
// `lds` must hold NT/64 words.  Returns the exclusive prefix; *total = block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x, uint32_t* lds, uint32_t* total) {
  constexpr int NW = NT / 64;
  const unsigned lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan_u32(x);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    uint32_t v = (lane < NW) ? lds[lane] : 0u;
    v = wave_incl_scan_u32(v);
    if (lane < NW) lds[lane] = v;
  }
  __syncthreads();
  const uint32_t wbase = (w > 0) ? lds[w - 1] : 0u;
  *total = lds[NW - 1];
  __syncthreads();
  return wbase + inc - x;
}

// 64-bit mixing step (SplitMix64 finaliser).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace tts
