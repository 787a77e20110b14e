// 2D kernels instantiated for orders 11 (n = 12 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(12)
