// Per-order launch table of the 2D kernels: the orders are compiled in
// separate units (sl2d_p*.hip) and reached through these tables.
#pragma once

#include "sl_internal.h"

namespace sl {

struct Ops2D {
    int (*prep)(int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM,
                const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s);
    int (*facevel)(int kx, int ky, int periodic, const double* aN, const double* tab, double vzero, double* vface,
                   hipStream_t s);
    int (*facevel_mixed)(int K_b, int bucket, int kx, int ky, const int32_t* elems, const int32_t* mix,
                         const double* aN_all, const double* tab_all, const double* interp, double vzero,
                         double* vface, hipStream_t s);
    int (*con_mixed)(const Step2DArgs& A, hipStream_t s);
    int (*adv)(const Step2DArgs& A, hipStream_t s);
    int (*con)(const Step2DArgs& A, hipStream_t s);
    int (*bt)(const Step2DArgs& A, hipStream_t s);
    int (*tgt)(const Step2DArgs& A, hipStream_t s);
    int (*adv_batch)(const Step2DArgs& A0, const Step2DArgs* As, const int* start, int nreq, int nblocks,
                     hipStream_t s);
    int (*con_batch)(const Step2DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s);
};

// the table of order n - 1 (host functions, one per unit that instantiates n)
const Ops2D* ops2d_2();
const Ops2D* ops2d_3();
const Ops2D* ops2d_4();
const Ops2D* ops2d_5();
const Ops2D* ops2d_6();
const Ops2D* ops2d_7();
const Ops2D* ops2d_8();
const Ops2D* ops2d_9();
const Ops2D* ops2d_10();
const Ops2D* ops2d_11();
const Ops2D* ops2d_12();
const Ops2D* ops2d_13();
const Ops2D* ops2d_14();
const Ops2D* ops2d_15();
const Ops2D* ops2d_16();
const Ops2D* ops2d_17();

}  // namespace sl
