// Fused frame-resident kernel, FP64, codes of row degree <= 32.
#include <algorithm>

#include "fused_kernels.h"

namespace ldpc {
LDPC_DEFINE_FUSED_BUCKET(ArithF64, 32)
}  // namespace ldpc
