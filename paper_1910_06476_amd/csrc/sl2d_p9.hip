// 2D kernels instantiated for order 15 (n = 16 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(16)
