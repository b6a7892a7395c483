// Layer kernels with run-time degree loops: FP32 rows of degree 33..64 and
// every FP64 bucket.
#include "layered_kernels.h"

namespace ldpc {
LDPC_DEFINE_LAYER_BUCKET(ArithF32, 64, false)
LDPC_DEFINE_LAYER_BUCKET(ArithF64, 8, false)
LDPC_DEFINE_LAYER_BUCKET(ArithF64, 16, false)
LDPC_DEFINE_LAYER_BUCKET(ArithF64, 32, false)
LDPC_DEFINE_LAYER_BUCKET(ArithF64, 64, false)
}  // namespace ldpc
