// Check-node kernels, FP32, rows of degree <= 16 (exact-degree bodies).
#include "flood_kernels.h"

namespace ldpc {
LDPC_DEFINE_CHECK_BUCKET(ArithF32, 16, true)
}  // namespace ldpc
