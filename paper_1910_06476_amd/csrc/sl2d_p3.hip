// 2D kernels instantiated for orders 7, 8 (n = 8, 9 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(8)
SL2D_DEFINE_OPS(9)
