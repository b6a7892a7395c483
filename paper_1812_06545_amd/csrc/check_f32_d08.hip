// Check-node kernels, FP32, rows of degree <= 8 (exact-degree bodies).
#include "flood_kernels.h"

namespace ldpc {
LDPC_DEFINE_CHECK_BUCKET(ArithF32, 8, true)
}  // namespace ldpc
