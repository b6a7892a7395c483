// Fused frame-resident kernel, FP64, codes of row degree <= 16.
#include <algorithm>

#include "fused_kernels.h"

namespace ldpc {
LDPC_DEFINE_FUSED_BUCKET(ArithF64, 16)
}  // namespace ldpc
