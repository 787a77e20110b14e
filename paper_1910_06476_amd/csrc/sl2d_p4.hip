// 2D kernels instantiated for orders 9, 10 (n = 10, 11 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(10)
SL2D_DEFINE_OPS(11)
