// Min-sum check and layer kernels, FP64, rows of degree <= 8 / 16 / 32 / 64.
#include "minsum_kernels.h"

namespace ldpc {
LDPC_DEFINE_MS_BUCKET(ArithF64, 8)
LDPC_DEFINE_MS_BUCKET(ArithF64, 16)
LDPC_DEFINE_MS_BUCKET(ArithF64, 32)
LDPC_DEFINE_MS_BUCKET(ArithF64, 64)
}  // namespace ldpc
