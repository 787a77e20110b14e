// 2D kernels instantiated for order 14 (n = 15 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(15)
