// TT-rounding of the exact sparse TT (placeholder until the dense sweeps land).
#include "dense.hpp"

namespace tts {

void round_tt(Allocator&, const RoundInput&, RoundOutput&, hipStream_t, hipEvent_t) {
  fail(TT_ERR_ARG, "rounding not available in this build (use sparse_only)");
}

}  // namespace tts
