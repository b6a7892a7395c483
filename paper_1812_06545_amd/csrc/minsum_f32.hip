// Min-sum check and layer kernels, FP32, rows of degree <= 8 / 16 / 32 / 64.
#include "minsum_kernels.h"

namespace ldpc {
LDPC_DEFINE_MS_BUCKET(ArithF32, 8)
LDPC_DEFINE_MS_BUCKET(ArithF32, 16)
LDPC_DEFINE_MS_BUCKET(ArithF32, 32)
LDPC_DEFINE_MS_BUCKET(ArithF32, 64)
}  // namespace ldpc
