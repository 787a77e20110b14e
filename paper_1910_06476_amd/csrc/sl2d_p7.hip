// 2D kernels instantiated for order 13 (n = 14 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(14)
