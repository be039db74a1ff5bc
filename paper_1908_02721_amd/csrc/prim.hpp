// Device-wide primitives: exclusive scan and stable LSD radix sort (gfx950).
#pragma once

#include "common.hpp"

namespace tts {

// out[i] = sum_{j<i} in[i] (u32).  The total is written to d_total (device).
// `in` and `out` may alias.  Temporary storage from `al`.
void exclusive_scan_u32(Allocator* al, const uint32_t* in, uint32_t* out, uint32_t n,
                        uint32_t* d_total, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key bits [0, nbits), 8-bit digits.
// Sorts in place on (keys, vals), using (ktmp, vtmp) as the ping-pong buffers.
// Keys with bits above nbits must be equal (or zero) for a full order.
void radix_sort_pairs(Allocator* al, uint64_t* keys, uint64_t* vals, uint64_t* ktmp,
                      uint64_t* vtmp, uint32_t n, int nbits, hipStream_t s);
// The same sort without the final copy: returns true when the sorted pairs are in
// (ktmp, vtmp) (an odd number of passes), false when they are in (keys, vals).
bool radix_sort_pairs_pp(Allocator* al, uint64_t* keys, uint64_t* vals, uint64_t* ktmp,
                         uint64_t* vtmp, uint32_t n, int nbits, hipStream_t s);
// Most pairs a one-workgroup rank sort takes (the sort itself for small counts, and
// the sparse stage's leader phase).
constexpr uint32_t kSmallSortMax = 2048;

}  // namespace tts
