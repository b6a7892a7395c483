// Layer kernels, FP32, rows of degree <= 32 (exact-degree bodies).
#include "layered_kernels.h"

namespace ldpc {
LDPC_DEFINE_LAYER_BUCKET(ArithF32, 32, true)
}  // namespace ldpc
