// 2D kernels instantiated for orders 1, 2, 3, 4 (n = 2, 3, 4, 5 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(2)
SL2D_DEFINE_OPS(3)
SL2D_DEFINE_OPS(4)
SL2D_DEFINE_OPS(5)
