// 2D kernels instantiated for orders 5, 6 (n = 6, 7 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(6)
SL2D_DEFINE_OPS(7)
