// 2D kernels instantiated for order 16 (n = 17 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(17)
