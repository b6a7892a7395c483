// Check-node kernels, FP32, rows of degree <= 24 (exact-degree bodies).
#include "flood_kernels.h"

namespace ldpc {
LDPC_DEFINE_CHECK_BUCKET(ArithF32, 24, true)
}  // namespace ldpc
