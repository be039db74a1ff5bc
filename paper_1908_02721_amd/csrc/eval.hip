// Sampled-entry evaluation of a TT and its gradient (placeholder).
#include "common.hpp"

extern "C" tt_status tt_eval_entries(int32_t, const int64_t*, const int64_t*, const void* const*, int32_t, int64_t,
                                     const int32_t*, void*, void*) {
  return TT_ERR_ARG;
}

extern "C" tt_status tt_eval_entries_backward(int32_t, const int64_t*, const int64_t*, const void* const*, int32_t,
                                              int64_t, const int32_t*, const void*, void* const*, void*) {
  return TT_ERR_ARG;
}
