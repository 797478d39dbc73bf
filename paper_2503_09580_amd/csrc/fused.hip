// Fused persistent kernel: one workgroup per cell.  (Filled in below.)
#include "internal.h"

namespace lincoll {

bool fused_supported(int, int) { return false; }

hipError_t fused_apply(const ApplyCtx&) { return hipErrorInvalidValue; }

}  // namespace lincoll
