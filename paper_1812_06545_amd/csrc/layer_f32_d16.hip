// Layer kernels, FP32, rows of degree <= 16 (exact-degree bodies).
#include "layered_kernels.h"

namespace ldpc {
LDPC_DEFINE_LAYER_BUCKET(ArithF32, 16, true)
}  // namespace ldpc
