// 2D explicit semi-Lagrangian step on gfx950 (FP64), the paper's two
// dimensional scheme (eq. 5.1, eq. 5.4, eq. 2dx_bnd_interpolate and
// eq. 2dy_bnd_interpolate).
//
// Mapping: one lane per particle (n^2 lanes per element), floor(256/n^2)
// elements per 256-lane block.
//
// advect (per element):
//   - RK move of the n^2 particles with the tensor Chebyshev interpolant of
//     the velocity (coefficients in LDS);
//   - the moved-point generalized Vandermonde system of eq. 5.4,
//     V_{p,(l,m)} = l_l(xi*_p) l_m(eta*_p), solved matrix-free by defect
//     correction x <- x + M^{-1} (phi* - V x) with the separable
//     preconditioner M = B0 (x) A0 built from the mean column / row
//     displacements (M^{-1} is two 1D remaps from the shifted nodes);
//   - the 4n edge traces of the remapped polynomial.
// constrain (per element): upwind face values (eq. 4.12a) and the boundary
// rows through C_B^+ (HARD) or (I + C_B^T C_B)^{-1} (SOFT); with mass or
// energy rows, their targets (eq. 4.14 and eq. remap_mass / remap_energy
// generalised to the RK quadrature) and the rows imposed after the boundary
// block, energy by Picard iteration.
// The kernels live in sl2d_kernels.h and are instantiated per order in the
// sl2d_p*.hip units; this unit holds the order dispatch and the launch
// geometry.
#include "sl2d_ops.h"

namespace sl {

constexpr int kBlock2 = 256;  // as in sl2d_kernels.h

int advect2d_shapes(int n) { return n >= 2 && n <= kMax2D ? 3 : 0; }

int advect2d_elems(int n, int bs)
{
    const int nd = n * n;
    const int BS = bs == 0 ? kBlock2 : bs == 1 ? ((nd + 63) / 64) * 64 : 2 * kBlock2;
    return BS / nd;
}

int blocks2d(int n, int K)
{
    if (n < 2 || n > kMax2D) return 0;
    // elements per block of the 256-lane shape, or one above 16 nodes per
    // direction (both kernels take no fewer)
    const int E = kBlock2 / (n * n) > 0 ? kBlock2 / (n * n) : 1;
    return (K + E - 1) / E;
}

namespace {

const Ops2D* ops2d(int n)
{
    switch (n) {
    case 2: return ops2d_2(); case 3: return ops2d_3(); case 4: return ops2d_4(); case 5: return ops2d_5();
    case 6: return ops2d_6(); case 7: return ops2d_7(); case 8: return ops2d_8(); case 9: return ops2d_9();
    case 10: return ops2d_10(); case 11: return ops2d_11(); case 12: return ops2d_12(); case 13: return ops2d_13();
    case 14: return ops2d_14(); case 15: return ops2d_15(); case 16: return ops2d_16(); case 17: return ops2d_17();
    default: return nullptr;
    }
}

}  // namespace

int advect2d_blocks(int n, int bs, int K)
{
    const int E = advect2d_elems(n, bs);
    return E > 0 ? (K + E - 1) / E : 0;
}

// elements per chunk of the boundary-row solve (ConShape in the kernels)
int constrain2d_chunks(int n, int K)
{
    const int a = 2 * kBlock2 / (n * n), b = kBlock2 / (4 * n);
    const int E = a < b ? a : b;
    return E > 0 ? (K + E - 1) / E : 0;
}

int launch_advect2d_batch(int n, const Step2DArgs& A0, const Step2DArgs* As, const int* start, int nreq,
                          int nblocks, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->adv_batch(A0, As, start, nreq, nblocks, s) : 1;
}

int launch_constrain2d_batch(int n, const Step2DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->con_batch(As, start, nreq, nblocks, s) : 1;
}

int launch_prep2d(int n, int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM,
                  const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->prep(K, has_div, cons, aN, aM, divN, divM, tab, dx, dy, vscale, vdeg, s) : 1;
}

int launch_facevel2d(int n, int kx, int ky, int periodic, const double* aN, const double* tab, double vzero,
                     double* vface, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->facevel(kx, ky, periodic, aN, tab, vzero, vface, s) : 1;
}

int launch_facevel2d_mixed(int n, int K_b, int bucket, int kx, int ky, const int32_t* elems, const int32_t* mix,
                           const double* aN_all, const double* tab_all, const double* interp, double vzero,
                           double* vface, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->facevel_mixed(K_b, bucket, kx, ky, elems, mix, aN_all, tab_all, interp, vzero, vface, s) : 1;
}

int launch_constrain2d_mixed(int n, const Step2DArgs& A, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->con_mixed(A, s) : 1;
}

int launch_advect2d(int n, const Step2DArgs& A, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->adv(A, s) : 1;
}

int launch_constrain2d(int n, const Step2DArgs& A, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->con(A, s) : 1;
}

int launch_targets2d(int n, const Step2DArgs& A, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->tgt(A, s) : 1;
}

int launch_backtrace2d(int n, const Step2DArgs& A, hipStream_t s)
{
    const Ops2D* o = ops2d(n);
    return o ? o->bt(A, s) : 1;
}

}  // namespace sl
