// Fused frame-resident kernel, FP32, codes of row degree <= 8.
#include <algorithm>

#include "fused_kernels.h"

namespace ldpc {
LDPC_DEFINE_FUSED_BUCKET(ArithF32, 8)
}  // namespace ldpc
