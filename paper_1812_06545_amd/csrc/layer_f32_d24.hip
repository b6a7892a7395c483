// Layer kernels, FP32, rows of degree <= 24 (exact-degree bodies).
#include "layered_kernels.h"

namespace ldpc {
LDPC_DEFINE_LAYER_BUCKET(ArithF32, 24, true)
}  // namespace ldpc
