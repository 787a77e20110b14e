// 2D kernels instantiated for orders 12 (n = 13 nodes per direction).
#include "sl2d_kernels.h"

SL2D_DEFINE_OPS(13)
