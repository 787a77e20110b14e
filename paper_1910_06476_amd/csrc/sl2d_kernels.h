// Kernels and per-order launchers of the 2D step, included by the
// sl2d_p*.hip units; each unit instantiates them for a few orders, so the
// orders compile in parallel.  See sl2d.hip for the method's outline.
#pragma once
#include <atomic>
#include <type_traits>
#include <utility>

#include "sl2d_ops.h"
#include "sl_batch.h"

namespace sl {
namespace {

constexpr int kBlock2 = 256;

__device__ __forceinline__ bool outside2(double s) { return s < -1e-10 || s > 1.0 + 1e-10; }

// table layout of a 2D mesh
template <int N> struct Off2 {
    static constexpr int ND = N * N;
    static constexpr int XI = 0, W = N, L0 = 2 * N, L1 = 3 * N, TINV = 4 * N, DM = 4 * N + ND, LAM = 4 * N + 2 * ND,
                         QH = 5 * N + 2 * ND, QS = QH + 16 * ND, ZMH = QS + 16 * ND, ZMS = ZMH + ND;
};

__device__ __forceinline__ double upwind2(double vn, double lo, double hi)
{
    if (vn > 0.0) return lo;
    if (vn < 0.0) return hi;
    return 0.5 * (lo + hi);
}

// sum_{k,l <= d} C[k + N l] T_k(x) T_l(y): Clenshaw in x inside Clenshaw in y
template <int N>
__device__ __forceinline__ double cheb2(const double* __restrict__ C, double x, double y, int d)
{
    const double x2 = 2.0 * x, y2 = 2.0 * y;
    double c1 = 0.0, c2 = 0.0;
    for (int l = d; l >= 0; --l) {
        const double* row = C + N * l;
        double b1 = 0.0, b2 = 0.0;
        for (int k = d; k >= 1; --k) {
            const double b0 = fma(x2, b1, row[k] - b2);
            b2 = b1;
            b1 = b0;
        }
        const double inner = fma(x, b1, row[0] - b2);
        if (l >= 1) {
            const double c0 = fma(y2, c1, inner - c2);
            c2 = c1;
            c1 = c0;
        } else {
            return fma(y, c1, inner - c2);
        }
    }
    return 0.0;
}

// NC tensor Chebyshev series C[c][N*l + k] (k: degree in x, l: degree in y,
// both <= D) at (x, y), summed directly over T_k(x) T_l(y).  The three-term
// recurrence gives T_k(x), T_l(y) (bounded by 1 on [-1, 1], as the sums are
// for particles inside their element); then (D+1)^2 FMAs per series against
// Clenshaw's 2(D+1)^2, and the D+1 row sums of every series are independent
// of each other.
template <int N, int D, int NC, int LR = 0>
__device__ __forceinline__ void cheb2_direct(const double* const (&C)[NC], double x, double y, double (&out)[NC])
{
    static_assert(D < N, "degree");
    double tx[D + 1], ty[D + 1];
    tx[0] = ty[0] = 1.0;
    if constexpr (D >= 1) {
        tx[1] = x;
        ty[1] = y;
    }
    const double x2 = 2.0 * x, y2 = 2.0 * y;
#pragma unroll
    for (int k = 2; k <= D; ++k) {
        tx[k] = fma(x2, tx[k - 1], -tx[k - 2]);
        ty[k] = fma(y2, ty[k - 1], -ty[k - 2]);
    }
    if constexpr (LR > 0) {
        // LR rows at a time: at most LR (D + 1) coefficients of each series
        // in flight (the unrolled sums load all of them at once, which in
        // the backtraces held the kernels' registers, and for coefficients
        // read through the scalar cache took more scalar registers than
        // there are); the same sums.  T_l(y) is carried by its recurrence
        // from T_0 = 1 and T_{-1} = y (then T_1 = 2y - y = y exactly), the
        // same values as ty[].
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        double tyl = 1.0, tym = y;
#pragma unroll 1
        for (int l0 = 0; l0 <= D; l0 += LR) {
#pragma unroll
            for (int r = 0; r < LR; ++r) {
                const int l = l0 + r;
                if (l <= D) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        double row = 0.0;
#pragma unroll
                        for (int k = 0; k <= D; ++k) row = fma(C[c][N * l + k], tx[k], row);
                        acc[c] = fma(tyl, row, acc[c]);
                    }
                    const double tyn = fma(y2, tyl, -tym);
                    tym = tyl;
                    tyl = tyn;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c] = acc[c];
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l <= D; ++l) {
                double row = 0.0;
#pragma unroll
                for (int k = 0; k <= D; ++k) row = fma(C[c][N * l + k], tx[k], row);
                acc = fma(ty[l], row, acc);
            }
            out[c] = acc;
        }
    }
}

// the same at a run-time degree d: compile-time degrees up to 7 (the
// effective degree of a resolved velocity), Clenshaw beyond
template <int N, int NC, int LR = 0>
__device__ __forceinline__ void cheb2_eval(const double* const (&C)[NC], double x, double y, int d, double (&out)[NC])
{
#define SL_CHEB2_CASE(DD)                                         \
    if constexpr (N > DD)                                        \
        if (d == DD) {                                           \
            cheb2_direct<N, DD, NC, LR>(C, x, y, out);           \
            return;                                              \
        }
    SL_CHEB2_CASE(0) SL_CHEB2_CASE(1) SL_CHEB2_CASE(2) SL_CHEB2_CASE(3)
    SL_CHEB2_CASE(4) SL_CHEB2_CASE(5) SL_CHEB2_CASE(6) SL_CHEB2_CASE(7)
#undef SL_CHEB2_CASE
#pragma unroll
    for (int c = 0; c < NC; ++c) out[c] = cheb2<N>(C[c], x, y, d);
}

// ---------------------------------------------------------------------------
// velocity preparation: tensor Chebyshev coefficients, divergence, own edge
// normal speeds, effective degree
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_prep2d(int K, int has_div, int cons, const double* __restrict__ aN, double* __restrict__ aM,
                         double* __restrict__ divN, double* __restrict__ divM, const double* __restrict__ tab, double invdx, double invdy, double vscale,
                         int* __restrict__ vdeg)
{
    using O = Off2<N>;
    constexpr int ND = N * N;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const double* U = aN + (size_t)e * ND;
    const double* V = aN + (size_t)K * ND + (size_t)e * ND;
    double* CU = aM + (size_t)e * ND;
    double* CV = aM + (size_t)K * ND + (size_t)e * ND;
    // C[l][k] = sum_j sum_i Tinv[l][j] Tinv[k][i] F[j][i]  (F[j][i] = node i + N j)
    auto modal = [&](const double* F, double* C) {
        double tmp[ND];  // tmp[j][k] = sum_i Tinv[k][i] F[j][i]
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s = fma(tab[O::TINV + k * N + i], F[i + N * j], s);
                tmp[k + N * j] = s;
            }
        for (int l = 0; l < N; ++l)
            for (int k = 0; k < N; ++k) {
                double s = 0.0;
                for (int j = 0; j < N; ++j) s = fma(tab[O::TINV + l * N + j], tmp[k + N * j], s);
                C[k + N * l] = s;
            }
    };
    modal(U, CU);
    modal(V, CV);
    double* dvn = divN + (size_t)e * ND;
    if (!has_div) {
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double sx = 0.0, sy = 0.0;
                for (int l = 0; l < N; ++l) sx = fma(tab[O::DM + i * N + l], U[l + N * j], sx);
                for (int m = 0; m < N; ++m) sy = fma(tab[O::DM + j * N + m], V[i + N * m], sy);
                dvn[i + N * j] = sx * invdx + sy * invdy;
            }
    }
    modal(dvn, divM + (size_t)e * ND);
    // effective degree: the 1D rule applied to the row and column sums of
    // |C|, with the noise threshold taken against max(sum |C|, scale)
    auto degree = [&](const double* C, double scale) {
        double tot = 0.0;
        for (int q = 0; q < ND; ++q) tot += fabs(C[q]);
        const double thr = fmax(tot, scale) * 0x1p-46;
        int d = 0;
        double tx = 0.0, ty = 0.0;
        for (int k = N - 1; k >= 1; --k) {
            for (int l = 0; l < N; ++l) {
                tx += fabs(C[k + N * l]);
                ty += fabs(C[l + N * k]);
            }
            if (d == 0 && (tx > thr || ty > thr)) d = k;
        }
        return d;
    };
    int d = max(degree(CU, vscale), degree(CV, vscale));
    if (cons) d = max(d, degree(divM + (size_t)e * ND, 0.0));
    atomicMax(vdeg, d);
}

// ---------------------------------------------------------------------------
// For edge point tt of element e (layout: left j, right j, bottom i, top i):
// the neighbour across that face (-1 outside the domain), the matching edge
// point in the neighbour, the ghost index, and whether e is the high side of
// the face (its left or bottom face).  periodic: bit 0 the left and right
// sides of the domain wrap onto each other, bit 1 the bottom and top sides.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void face_partner2(int e, int tt, int kx, int ky, int periodic, int& nbe, int& nbt,
                                              int& gidx, bool& high)
{
    const int side = tt / N, k = tt % N;
    const int ex = e % kx, ey = e / kx;
    const int KL = ky * N, KB = kx * N;
    switch (side) {
    case 0:
        nbe = ex > 0 ? e - 1 : ((periodic & 1) ? ey * kx + kx - 1 : -1);
        nbt = N + k; gidx = ey * N + k; high = true;
        break;
    case 1:
        nbe = ex < kx - 1 ? e + 1 : ((periodic & 1) ? ey * kx : -1);
        nbt = k; gidx = KL + ey * N + k; high = false;
        break;
    case 2:
        nbe = ey > 0 ? e - kx : ((periodic & 2) ? (ky - 1) * kx + ex : -1);
        nbt = 3 * N + k; gidx = 2 * KL + ex * N + k; high = true;
        break;
    default:
        nbe = ey < ky - 1 ? e + kx : ((periodic & 2) ? ex : -1);
        nbt = 2 * N + k; gidx = 2 * KL + KB + ex * N + k; high = false;
        break;
    }
}

// ---------------------------------------------------------------------------
// face normal velocity at every element's own edge points: the mean of the
// two sides' interpolated normal components (the interior side alone at a
// ghost boundary); a speed at or below vzero has no upwind side and is
// stored as zero.  Built once per velocity.
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_facevel2d(int kx, int ky, int periodic, const double* __restrict__ aN,
                            const double* __restrict__ tab, double vzero, double* __restrict__ vface)
{
    using O = Off2<N>;
    constexpr int ND = N * N, NB = 4 * N;
    const int K = kx * ky;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long)K * NB) return;
    const int e = (int)(gid / NB), tt = (int)(gid % NB);
    auto normal = [&](int el, int t2) {
        const int side = t2 / N, k = t2 % N;
        const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
        double s = 0.0;
        if (side < 2) {
            const double* U = aN + (size_t)el * ND;
            for (int c = 0; c < N; ++c) s = fma(lv[c], U[c + N * k], s);
        } else {
            const double* V = aN + (size_t)K * ND + (size_t)el * ND;
            for (int c = 0; c < N; ++c) s = fma(lv[c], V[k + N * c], s);
        }
        return s;
    };
    int nbe, nbt, gidx;
    bool high;
    face_partner2<N>(e, tt, kx, ky, periodic, nbe, nbt, gidx, high);
    double vn = normal(e, tt);
    if (nbe >= 0) vn = 0.5 * (vn + normal(nbe, nbt));
    if (fabs(vn) <= vzero) vn = 0.0;
    vface[gid] = vn;
}

// ---------------------------------------------------------------------------
// Lagrange basis row l_k(x), k < N, in product form:
// l_k(x) = lambda_k prod_{j != k} (x - xi_j), from prefix and suffix products
// (no division, exact at the nodes)
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void lag_row(const double* __restrict__ xi, const double* __restrict__ lam, double x,
                                        double (&l)[N])
{
    double pre[N];
    double acc = 1.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        pre[k] = acc;
        acc *= (x - xi[k]);
    }
    acc = 1.0;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        l[k] = lam[k] * pre[k] * acc;
        acc *= (x - xi[k]);
    }
}

template <int N>
__device__ __forceinline__ void lag_row(const double* __restrict__ tab, double x, double (&l)[N])
{
    using O = Off2<N>;
    lag_row<N>(tab + O::XI, tab + O::LAM, x, l);
}

// phi^n (nodal values f of one element, in LDS) carried back along the
// characteristic through reference point (s, r) over time h: the value of
// phi^n at the foot, times the source factor of the conservative form.  The
// trace uses the same explicit RK tableau as the particles (eq. 4.11 in 2D);
// `out` is set when a stage position leaves the element.
// xi, lam: the nodes and barycentric weights (the table's, or a copy in LDS)
template <int N>
__device__ double backtrace2(const Step2DArgs& A, const double* cu, const double* cv, const double* cd,
                             const double* f, double h, double s, double r, bool& out, const double* xi,
                             const double* lam)
{
    const RKTab& T = A.rk;
    double qf = 1.0;
    if (h > 0.0) {
        double ks[4], kr[4], kq[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            ks[st] = kr[st] = kq[st] = 0.0;
            if (st < T.s) {
                double ss = s, rr = r, qq = qf;
                for (int m = 0; m < st; ++m) {
                    ss += h * T.a[st][m] * ks[m];
                    rr += h * T.a[st][m] * kr[m];
                    qq += h * T.a[st][m] * kq[m];
                }
                out |= outside2(ss) || outside2(rr);
                const double x = 2.0 * ss - 1.0, y = 2.0 * rr - 1.0;
                if (A.cons) {
                    const double* C3[3] = {cu, cv, cd};
                    double o[3];
                    cheb2_eval<N, 3, 1>(C3, x, y, A.vdeg, o);
                    ks[st] = -o[0] * A.invdx;
                    kr[st] = -o[1] * A.invdy;
                    kq[st] = -o[2] * qq;
                } else {
                    const double* C2[2] = {cu, cv};
                    double o[2];
                    cheb2_eval<N, 2, 1>(C2, x, y, A.vdeg, o);
                    ks[st] = -o[0] * A.invdx;
                    kr[st] = -o[1] * A.invdy;
                    kq[st] = 0.0;
                }
            }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st)
            if (st < T.s) {
                s += h * T.b[st] * ks[st];
                r += h * T.b[st] * kr[st];
                qf += h * T.b[st] * kq[st];
            }
        out |= outside2(s) || outside2(r);
    }
    double ls[N], lr[N];
    lag_row<N>(xi, lam, s, ls);
    lag_row<N>(xi, lam, r, lr);
    double acc = 0.0;
    // row by row: unrolled, the n^2 loads of f are invariant in a caller's
    // loop over traces and were hoisted out of it, all held in registers
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
        double in = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) in = fma(ls[i], f[i + N * j], in);
        acc = fma(lr[j], in, acc);
    }
    return qf * acc;
}

// ---------------------------------------------------------------------------
// advect + remap (eq. 5.4 by defect correction) + edge traces
//
// One lane per particle (n^2 lanes per element, floor(256/n^2) elements per
// block).  With PR = 1 the separable preconditioner is stored and applied in
// FP32, with PR = 2 its entries and operands are BF16 with FP32
// accumulation; the residual and the iterate stay FP64 (iterative
// refinement).  PR = 0 is FP64 throughout.
//
// Record of element e (stride A.rstride): its 4n edge traces of phi-hat;
// with mass or energy rows the 8n + 3 target terms of k_targets2d; with
// backtracking interface values, last, the 4n face values it offers.
// ---------------------------------------------------------------------------
// block shapes of the advect kernel: 0 = 256 lanes, 1 = the fewest whole
// waves that hold one element, 2 = 512 lanes.  With one element per block
// the residual takes the iterate by row broadcasts (resid_bcast).
template <int N, int BSEL> struct Shape2 {
    static constexpr int ND = N * N;
    static constexpr int BS = BSEL == 0 ? kBlock2 : BSEL == 1 ? ((ND + 63) / 64) * 64 : 2 * kBlock2;
    static constexpr int E = BS / ND;
};

// Preconditioner storage and arithmetic of precision PR: FP64, FP32, or BF16
// (the upper half of an FP32, rounded to nearest even) with FP32 products
// and sums.  The BF16 operands multiply exactly in FP32.
template <int PR> struct Prec;
template <> struct Prec<0> {
    using S = double;  // storage
    using A = double;  // arithmetic
    __device__ static S put(double v) { return v; }
    __device__ static A get(S v) { return v; }
};
template <> struct Prec<1> {
    using S = float;
    using A = float;
    __device__ static S put(double v) { return (float)v; }
    __device__ static A get(S v) { return v; }
};
template <> struct Prec<2> {
    using S = unsigned short;
    using A = float;
    __device__ static S put(double v)
    {
        const unsigned int b = __float_as_uint((float)v);
        if ((b & 0x7f800000u) == 0x7f800000u) return (S)(b >> 16);  // inf / nan: truncate
        return (S)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);          // round to nearest even
    }
    __device__ static A get(S v) { return __uint_as_float((unsigned int)v << 16); }
};

// v = max(v, the v of the lane that DPP control CTRL selects), one VALU
// instruction (the compiler does not fold a separate DPP move into the
// max); lanes in rows outside the row mask keep their v.  The s_nop gives
// the two wait states a DPP read needs after a VALU write of its source.
#define SL_DPP_MAX_U32(v, CTRL) asm volatile("s_nop 1\n\tv_max_u32_dpp %0, %0, %0 " CTRL : "+v"(v))

// Maximum over the 64 lanes of a wave, left in lane 63: butterflies within
// quads (quad_perm [1,0,3,2], [2,3,0,1]), then half-rows and rows (mirror),
// then across rows (broadcast of lane 15 into rows 1 and 3, of lane 31 into
// rows 2 and 3).  VALU data movement only, none through the LDS unit.
// Every lane of the wave runs it.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    SL_DPP_MAX_U32(v, "quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf");
    SL_DPP_MAX_U32(v, "quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf");
    SL_DPP_MAX_U32(v, "row_half_mirror row_mask:0xf bank_mask:0xf");
    SL_DPP_MAX_U32(v, "row_mirror row_mask:0xf bank_mask:0xf");
    SL_DPP_MAX_U32(v, "row_bcast:15 row_mask:0xa bank_mask:0xf");
    SL_DPP_MAX_U32(v, "row_bcast:31 row_mask:0xc bank_mask:0xf");
    return v;
}

// The same for 64-bit values, exactly: the upper words first, then the
// lower words of the lanes whose upper word is the maximum (32-bit maxima
// only, no 64-bit compares).
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    const unsigned hi = (unsigned)(v >> 32);
    const unsigned top = (unsigned)__builtin_amdgcn_readlane((int)wave_max_u32(hi), 63);
    const unsigned lo = wave_max_u32(hi == top ? (unsigned)v : 0u);
    return ((unsigned long long)top << 32) | lo;
}

// Maximum of the bit patterns `bits` (non-negative doubles, and NaN above
// them, order as their bits) over the lanes of each element slot present in
// one 64-lane wave, published to dst[slot] with one LDS atomic per slot
// instead of one per lane: same-address LDS atomics serialise.  Valid when a
// wave spans at most two slots (n^2 >= 64), or with every lane in slot 0
// (the constrain kernels' block-wide residual).  Every lane of the wave calls
// it; lanes without a value pass 0.
// (the slots sit S words apart in dst).
template <int E, int S = 1>
__device__ __forceinline__ void slot_max(unsigned long long* dst, int slot, unsigned long long bits)
{
    if constexpr (E == 1) {
        // one slot: lanes outside it pass 0
        const unsigned long long a = wave_max_u64(bits);
        if ((threadIdx.x & 63) == 63 && a) atomicMax(&dst[0], a);
    } else {
        const int first = __builtin_amdgcn_readfirstlane(slot);  // every lane is active here: lane 0's slot
        const unsigned long long a = wave_max_u64(slot == first ? bits : 0ull);
        const unsigned long long b = wave_max_u64(slot == first + 1 ? bits : 0ull);
        if ((threadIdx.x & 63) == 63) {
            if (first < E && a) atomicMax(&dst[first * S], a);
            if (first + 1 < E && b) atomicMax(&dst[(first + 1) * S], b);
        }
    }
}

__device__ __forceinline__ unsigned long long abs_bits(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}

// acc += x' * a, where x' is lane K of this lane's row of 16 lanes (DPP
// row_newbcast on the 64-bit source of one v_fmac_f64: the broadcast costs
// no instruction of its own; the compiler does not fold a separate
// broadcast move into the FMA).  The s_nop gives the two wait states a DPP
// read needs after a VALU write of its source, whatever the compiler placed
// before.  Register operands only.  Volatile: kept where every lane runs it.
template <int K>
__device__ __forceinline__ void fmac_bcast(double& acc, double x, double a)
{
    asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(x), "v"(a), "n"(K));
}

// Residual product (V x)_p = sum_m b_m sum_l a_l x[m][l] of one particle,
// for blocks that hold one element: every row of 16 lanes then belongs to
// it, and each lane keeps iterate value 16 c + (lane % 16) of the chunks c
// a row of x touches, so each product takes its x from a row broadcast
// instead of an LDS read (2 reads per row of x instead of n).  Same
// products and sums in the same order as the LDS form.
// Up to four of them in one asm block, with one s_nop for the block: inside
// it only the accumulator is written, never a broadcast source.
template <int K0, int K1, int K2, int K3>
__device__ __forceinline__ void fmac_bcast4(double& acc, double x0, double a0, double x1, double a1, double x2,
                                            double a2, double x3, double a3)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %1, %2 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %3, %4 row_newbcast:%10 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %5, %6 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %7, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(x0), "v"(a0), "v"(x1), "v"(a1), "v"(x2), "v"(a2), "v"(x3), "v"(a3), "n"(K0), "n"(K1),
                   "n"(K2), "n"(K3));
}
template <int K0, int K1, int K2>
__device__ __forceinline__ void fmac_bcast3(double& acc, double x0, double a0, double x1, double a1, double x2,
                                            double a2)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %1, %2 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %3, %4 row_newbcast:%8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %5, %6 row_newbcast:%9 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(x0), "v"(a0), "v"(x1), "v"(a1), "v"(x2), "v"(a2), "n"(K0), "n"(K1), "n"(K2));
}
template <int K0, int K1>
__device__ __forceinline__ void fmac_bcast2(double& acc, double x0, double a0, double x1, double a1)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %1, %2 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %3, %4 row_newbcast:%6 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(x0), "v"(a0), "v"(x1), "v"(a1), "n"(K0), "n"(K1));
}

// products L0.. of row M of the residual, four to an asm block
template <int N, int M, int L0>
__device__ __forceinline__ void resid_row_from(double& inner, const double (&a)[N], double xa, double xb)
{
    constexpr int C0 = (N * M) >> 4;
    auto X = [&](int l) { return ((N * M + l) >> 4) == C0 ? xa : xb; };
    constexpr int R = N - L0;
    if constexpr (R >= 4) {
        fmac_bcast4<(N * M + L0) & 15, (N * M + L0 + 1) & 15, (N * M + L0 + 2) & 15, (N * M + L0 + 3) & 15>(
            inner, X(L0), a[L0], X(L0 + 1), a[L0 + 1], X(L0 + 2), a[L0 + 2], X(L0 + 3), a[L0 + 3]);
        resid_row_from<N, M, L0 + 4>(inner, a, xa, xb);
    } else if constexpr (R == 3) {
        fmac_bcast3<(N * M + L0) & 15, (N * M + L0 + 1) & 15, (N * M + L0 + 2) & 15>(
            inner, X(L0), a[L0], X(L0 + 1), a[L0 + 1], X(L0 + 2), a[L0 + 2]);
    } else if constexpr (R == 2) {
        fmac_bcast2<(N * M + L0) & 15, (N * M + L0 + 1) & 15>(inner, X(L0), a[L0], X(L0 + 1), a[L0 + 1]);
    } else if constexpr (R == 1) {
        fmac_bcast<(N * M + L0) & 15>(inner, X(L0), a[L0]);
    }
}

template <int N, int M, int... L>
__device__ __forceinline__ double resid_row(const double (&a)[N], double xa, double xb,
                                            std::integer_sequence<int, L...>)
{
    double inner = 0.0;
    resid_row_from<N, M, 0>(inner, a, xa, xb);
    return inner;
}

template <int N, int... M>
__device__ __forceinline__ double resid_bcast(const double (&a)[N], const double (&b)[N], const double* x, int k16,
                                              std::integer_sequence<int, M...>)
{
    constexpr int ND = N * N;
    double vx = 0.0;
    // the chunk values past the iterate's end are clamped to its last entry
    // (in bounds; no product takes them)
    ((vx = fma(b[M],
               resid_row<N, M>(a, x[min(16 * ((N * M) >> 4) + k16, ND - 1)],
                               x[min(16 * ((N * M + N - 1) >> 4) + k16, ND - 1)], std::make_integer_sequence<int, N>{}),
               vx)),
     ...);
    return vx;
}

// rows of the velocity series per batch in one-element advect blocks (0:
// all at once).  Measured on the C4 recipe (degree-5 series, per launch):
// one row at a time n = 9 174 -> 168 us, n = 7 84 -> 82 us (no spilled
// scalar registers); at n = 13 the unrolled sums stay faster (330 us against
// 334 one row and 337 two rows at a time).
template <int N> constexpr int kSeriesRows = N >= 13 ? 0 : 1;

template <int N, int PR, int BSEL>
__device__ __forceinline__ void advect2d_body(const Step2DArgs& A, const int bid)
{
    using O = Off2<N>;
    using PP = Prec<PR>;
    using PT = typename PP::S;
    using AT = typename PP::A;
    constexpr bool P32 = PR != 0;  // reduced-precision preconditioner, operands scaled
    constexpr int ND = N * N, E = Shape2<N, BSEL>::E, NB = 4 * N;
    __shared__ double s_cu[E][ND], s_cv[E][ND], s_cd[E][ND];
    __shared__ double s_x[E][ND], s_r[E][ND], s_f[E][ND];
    __shared__ PT s_z[E][ND];
    __shared__ PT s_ai[E][ND], s_bi[E][ND];
    __shared__ double s_mx[E][N], s_my[E][N];
    __shared__ unsigned long long s_nrm[2][E];  // max |y| per element, double-buffered by sweep parity
    __shared__ int s_flag, s_sw_sum, s_sw_max;
    __shared__ unsigned long long s_res;
    __shared__ unsigned long long s_ref[E];  // max |phi*| per element

    const int t = threadIdx.x;
    const int slot = t / ND, q = t - slot * ND;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const int e = bid * E + slot;
    const bool live = inblk && e < A.K;
    const double* __restrict__ tab = A.tab;
    const int K = A.K;
    const int ii = q % N, jj = q / N;
    if (t == 0) {
        s_flag = 0;
        s_sw_sum = 0;
        s_sw_max = 0;
        s_res = 0ull;
    }
    if (t < E * 2) s_nrm[t / E][t % E] = 0ull;
    if (t < E) s_ref[t] = 0ull;

    double phi_p = 0.0, u_p = 0.0, v_p = 0.0, dv_p = 0.0;
    {
        const size_t g = (size_t)(live ? e : 0) * ND + (inblk ? q : 0);
        if (live) {
            phi_p = A.phi[g];
            u_p = A.aN[g];
            v_p = A.aN[(size_t)K * ND + g];
            if (A.cons) dv_p = A.divN[g];
        }
        if (inblk) {
            // only the coefficients within the effective degree are read
            const bool used = live && ii <= A.vdeg && jj <= A.vdeg;
            s_cu[slot][q] = used ? A.aM[g] : 0.0;
            s_cv[slot][q] = used ? A.aM[(size_t)K * ND + g] : 0.0;
            if (A.cons) s_cd[slot][q] = used ? A.divM[g] : 0.0;
        }
    }
    __syncthreads();

    const RKTab& T = A.rk;
    bool out = false;

    // forward motion of the particle (eq. 5.1 tensor interpolant of the velocity)
    const int d = A.vdeg;
    const double h = A.dt;
    double sx, sy, sq;
    // A series of degree <= 1 (constant, shear, rotation) is evaluated from
    // registers: the same operations as the Clenshaw sum at that degree.
    const bool low = d <= 1;
    double lu[4] = {0.0, 0.0, 0.0, 0.0}, lv[4] = {0.0, 0.0, 0.0, 0.0}, ld[4] = {0.0, 0.0, 0.0, 0.0};
    if (low) {
        const int at[4] = {0, 1, N, N + 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lu[k] = s_cu[sl][at[k]];
            lv[k] = s_cv[sl][at[k]];
            if (A.cons) ld[k] = s_cd[sl][at[k]];
        }
    }
    auto vel = [&](const double (&c)[4], double x, double y) {
        return d == 0 ? c[0] : fma(y, fma(x, c[3], c[2]), fma(x, c[1], c[0]));
    };
    {
        const double s = tab[O::XI + ii], rr0 = tab[O::XI + jj], qv = phi_p;
        double ks[4], kr[4], kq[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            ks[st] = kr[st] = kq[st] = 0.0;
            if (st < T.s) {
                double ss = s, rr = rr0, qq = qv;
                for (int m = 0; m < st; ++m) {
                    ss += h * T.a[st][m] * ks[m];
                    rr += h * T.a[st][m] * kr[m];
                    qq += h * T.a[st][m] * kq[m];
                }
                double uu, vv, dd = 0.0;
                if (st == 0) {
                    uu = u_p;
                    vv = v_p;
                    dd = dv_p;
                } else {
                    const double x = 2.0 * ss - 1.0, y = 2.0 * rr - 1.0;
                    if (low) {
                        uu = vel(lu, x, y);
                        vv = vel(lv, x, y);
                        if (A.cons) dd = vel(ld, x, y);
                    } else if (A.cons) {
                        double o[3];
                        if constexpr (Shape2<N, BSEL>::E == 1) {
                            // one element per block: its coefficients have a block-uniform
                            // address and are read through the scalar cache, not LDS
                            const double* gu = A.aM + (size_t)bid * ND;
                            const double* C3[3] = {gu, gu + (size_t)K * ND, A.divM + (size_t)bid * ND};
                            cheb2_eval<N, 3, kSeriesRows<N>>(C3, x, y, d, o);
                        } else {
                            const double* C3[3] = {s_cu[sl], s_cv[sl], s_cd[sl]};
                            cheb2_eval<N, 3>(C3, x, y, d, o);
                        }
                        uu = o[0];
                        vv = o[1];
                        dd = o[2];
                    } else {
                        double o[2];
                        if constexpr (Shape2<N, BSEL>::E == 1) {
                            const double* gu = A.aM + (size_t)bid * ND;
                            const double* C2[2] = {gu, gu + (size_t)K * ND};
                            cheb2_eval<N, 2, kSeriesRows<N>>(C2, x, y, d, o);
                        } else {
                            const double* C2[2] = {s_cu[sl], s_cv[sl]};
                            cheb2_eval<N, 2>(C2, x, y, d, o);
                        }
                        uu = o[0];
                        vv = o[1];
                    }
                    out |= inblk && (outside2(ss) || outside2(rr));
                }
                ks[st] = uu * A.invdx;
                kr[st] = vv * A.invdy;
                kq[st] = A.cons ? -dd * qq : 0.0;
            }
        }
        double ds = 0.0, dr = 0.0, dq = 0.0;
#pragma unroll
        for (int st = 0; st < 4; ++st)
            if (st < T.s) {
                ds += T.b[st] * ks[st];
                dr += T.b[st] * kr[st];
                dq += T.b[st] * kq[st];
            }
        sx = s + h * ds;
        sy = rr0 + h * dr;
        sq = qv + h * dq;
        out |= inblk && (outside2(sx) || outside2(sy));
    }

    // row of V for this particle: a_l = l_l(xi*), b_m = l_m(eta*) (eq. 5.4)
    double a[N], b[N];
    lag_row<N>(tab, sx, a);
    lag_row<N>(tab, sy, b);

    // separable preconditioner: mean displacement of each x-column i and of
    // each y-row j of particles
    if (inblk) {
        s_r[slot][q] = sx - tab[O::XI + ii];
        s_x[slot][q] = sy - tab[O::XI + jj];
        s_f[slot][q] = sq;  // phi*
    }
    if constexpr (ND >= 64) slot_max<E>(s_ref, slot, inblk ? abs_bits(sq) : 0ull);
    else if (inblk) atomicMax(&s_ref[slot], abs_bits(sq));
    __syncthreads();
    for (int c = q; inblk && c < 2 * N; c += ND) {
        double m = 0.0;
        if (c < N) {
            for (int j = 0; j < N; ++j) m += s_r[slot][c + N * j];
            s_mx[slot][c] = m / N;
        } else {
            for (int i = 0; i < N; ++i) m += s_x[slot][i + N * (c - N)];
            s_my[slot][c - N] = m / N;
        }
    }
    __syncthreads();
    // A0^{-1}[l][c]: interpolation from the shifted nodes xi_k + mx_k back to
    // node xi_l, prod_{k != c} (xi_l - s_k) / prod_{k != c} (s_c - s_k)
    if (inblk) {
        const int l = ii, c = jj;
        const double xl = tab[O::XI + l];
        const double sc = tab[O::XI + c] + s_mx[slot][c], tc = tab[O::XI + c] + s_my[slot][c];
        // The denominators by the product rule (the factor at k = c is
        // exactly zero; see the 1D remap weights), the numerators with a
        // select: no branch on k == c, so every read is unconditional.
        double na = 1.0, nb = 1.0, pa = 1.0, da = 0.0, pb = 1.0, db = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double sk = tab[O::XI + k] + s_mx[slot][k];
            const double tk = tab[O::XI + k] + s_my[slot][k];
            const double fa = sc - sk, fb = tc - tk;
            da = fma(da, fa, pa);
            pa *= fa;
            db = fma(db, fb, pb);
            pb *= fb;
            na *= (k == c) ? 1.0 : xl - sk;
            nb *= (k == c) ? 1.0 : xl - tk;
        }
        s_ai[slot][q] = PP::put(na / da);
        s_bi[slot][q] = PP::put(nb / db);
    }
    __syncthreads();

    // y = M^{-1} f (f in s_f or s_r, node c + N jj):
    //   stage 1: z[jj][l] = sum_c Ai[l][c] f[jj][c]
    //   stage 2: y[m][l] = sum_jj Bi[m][jj] z[jj][l]
    // In FP32 or BF16 the operand is first scaled by 2^-e, e = exponent of a
    // reference magnitude of it (max |phi*| of the element, then the last
    // correction), so that it sits near 1 and never in the subnormal range;
    // M^{-1} is linear, so the result is scaled back exactly.  In BF16 the
    // operand and the stage-1 result are rounded to BF16 before each product.
    auto precond = [&](double (*src)[ND], int e2) -> double {
        const double sc = P32 ? ldexp(1.0, -e2) : 1.0;
        if (inblk) {
            AT zz = 0;
            for (int c = 0; c < N; ++c) {
                const double v = src[slot][c + N * jj];
                zz = fma(PP::get(s_ai[slot][ii + N * c]), PP::get(PP::put(P32 ? v * sc : v)), zz);
            }
            s_z[slot][q] = PP::put(zz);
        }
        __syncthreads();
        AT acc = 0;
        if (inblk)
            for (int j = 0; j < N; ++j) acc = fma(PP::get(s_bi[slot][jj + N * j]), PP::get(s_z[slot][ii + N * j]), acc);
        return P32 ? ldexp((double)acc, e2) : (double)acc;
    };
    // exponent of a reference magnitude, clamped so 2^-e stays finite
    auto ref_exp = [](double ref) { return ref > 0.0 ? max(ilogb(ref), -1000) : 0; };

    const double ref = __longlong_as_double((long long)s_ref[sl]);  // max |phi*| of the element
    int e2 = P32 ? ref_exp(ref) : 0;
    double x = precond(s_f, e2);
    if (inblk) s_x[slot][q] = x;
    __syncthreads();
    bool conv = !live;
    int sweeps = A.refine;   // sweeps this element needed
    double prev = 0.0;       // max |y| of the previous sweep
    // |y| of the last sweep taken and of the one before it (the estimated
    // error left is formed from them once, after the loop)
    double eny_last = 0.0, prev_last = 0.0;
    bool had_prev = false;
    for (int it = 0; it < A.refine; ++it) {
        // residual r_p = phi*_p - (V x)_p, (V x)_p = sum_m b_m sum_l a_l x[m][l]
        double vx = 0.0;
        if constexpr (E == 1) {
            // every lane of the block takes part (the row broadcasts read
            // from idle lanes too)
            vx = resid_bcast<N>(a, b, s_x[0], t & 15, std::make_integer_sequence<int, N>{});
            // an empty use in every lane: the products stay where the
            // broadcasts are, instead of sinking into the store's branch
            // with every broadcast value live until then
            asm volatile("" : : "v"(vx));
        } else {
#pragma unroll
            for (int m = 0; m < N; ++m) {
                double inner = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) inner = fma(a[l], s_x[sl][l + N * m], inner);
                vx = fma(b[m], inner, vx);
            }
        }
        if (inblk) s_r[slot][q] = sq - vx;
        __syncthreads();  // s_x is no longer read in this sweep
        // clear the other parity's slot, last read before this sweep's first barrier
        if (t < E) s_nrm[(it + 1) & 1][t] = 0ull;
        const double y = precond(s_r, e2);
        if (inblk) {
            if (!conv) x += y;
            s_x[slot][q] = x;
        }
        if constexpr (ND >= 64) slot_max<E>(s_nrm[it & 1], slot, inblk ? abs_bits(y) : 0ull);
        else if (inblk) atomicMax(&s_nrm[it & 1][slot], abs_bits(y));
        __syncthreads();
        if (inblk) {
            const double eny = __longlong_as_double((long long)s_nrm[it & 1][slot]);
            if (P32 && eny > 0.0) e2 = ref_exp(eny);
            if (!conv) {
                eny_last = eny;
                prev_last = prev;
                had_prev = it > 0;
                // Stop when the correction is below 2^-44 of max |phi*|, or
                // when the observed contraction q = |y_k| / |y_{k-1}| <= 1/2
                // puts the remaining error (about q |y_k|) below 2^-50 of it.
                // Both sit above the rounding floor of the residual (about
                // n^2 eps) and far below the FP64 parity bar.
                const bool small = eny <= 0x1p-44 * ref;
                const bool contracted = it > 0 && eny <= 0.5 * prev && eny * eny <= 0x1p-50 * ref * prev;
                if (small || contracted) {
                    conv = true;
                    sweeps = it + 1;
                }
            }
            prev = eny;
        }
        if constexpr (E == 1) {
            // conv is the element's, the same in all its lanes, and lane 0
            // of every wave is one of them: each wave breaks alike with no
            // barrier (the barriers above order every LDS access of the
            // next sweep)
            if (__builtin_amdgcn_readfirstlane(conv)) break;
        } else {
            if (__syncthreads_and(conv)) break;
        }
    }
    // estimated error left after the last sweep taken: its correction times
    // the observed contraction, relative to max |phi*|
    double lastrel = 0.0;
    if (inblk && ref > 0.0) {
        const double left = (had_prev && prev_last > 0.0) ? fmin(eny_last, eny_last * eny_last / prev_last) : eny_last;
        lastrel = left / ref;
    }

    // edge traces of the remapped polynomial (eq. 2dx/2dy_bnd_interpolate):
    // t < N left (xi=0, eta_t), < 2N right, < 3N bottom (xi_k, eta=0), top
    int fl = 0;
    if (live) {
        if (out) fl |= FLAG_CONTAIN;
        if (!conv || !isfinite(x)) fl |= FLAG_SINGULAR;
        if (q == 0) {
            atomicAdd(&s_sw_sum, sweeps);
            atomicMax(&s_sw_max, sweeps);
            atomicMax(&s_res, (unsigned long long)__double_as_longlong(lastrel));
        }
        A.phihat[(size_t)e * ND + q] = x;
        for (int tt = q; tt < NB; tt += ND) {
            const int side = tt / N, k = tt % N;
            const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
            double tr = 0.0;
            if (side < 2)
                for (int c = 0; c < N; ++c) tr = fma(lv[c], s_x[slot][c + N * k], tr);
            else
                for (int c = 0; c < N; ++c) tr = fma(lv[c], s_x[slot][k + N * c], tr);
            A.rec[(size_t)e * A.rstride + tt] = tr;
        }
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[bid] |= s_flag;
        // one block owns each slot row; launches on the stream are ordered
        double* sp = A.stat_part + (size_t)bid * kStatSlots;
        sp[4] += (double)s_sw_sum;
        sp[5] = fmax(sp[5], (double)s_sw_max);
        sp[6] = fmax(sp[6], __longlong_as_double((long long)s_res));
    }
}

template <int N, int PR, int BSEL = 0>
__global__ __launch_bounds__((Shape2<N, BSEL>::BS)) void k_advect2d(Step2DArgs A)
{
    advect2d_body<N, PR, BSEL>(A, blockIdx.x);
}

// One step of several meshes in one launch: the blocks of request r are
// start[r] .. start[r + 1] - 1, each running the kernel above on the
// request's own arguments As[r] (boundary rows only)
template <int N, int PR, int BSEL>
__global__ __launch_bounds__((Shape2<N, BSEL>::BS)) void k_advect2d_batch(const Step2DArgs* __restrict__ As,
                                                                          const int* __restrict__ start, int nreq)
{
    const int r = batch_request(start, nreq, blockIdx.x);
    advect2d_body<N, PR, BSEL>(As[r], blockIdx.x - start[r]);
}

// ---------------------------------------------------------------------------
// boundary-constrained least squares (2D)
// ---------------------------------------------------------------------------
// persistent blocks: each loads the 4n x 4n table Q into LDS once and loops
// over chunks of E elements
constexpr int kConGrid = 2048;

// Blocks of a persistent launch: no more than are resident at once (the
// 4n x 4n table limits them by LDS at large n: 24 KB per block at n = 13),
// so that no block waits for a whole element loop of another, and at most
// kConGrid.  Computed once per kernel and device, in cache[device] (atomic:
// meshes may be stepped from several host threads).
constexpr int kMaxDevices = 64;
template <typename Kern>
int resident_blocks(Kern kernel, std::atomic<int>* cache)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return kConGrid;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock2, 0) != hipSuccess || per < 1 || cus < 1)
            return kConGrid;  // not cached: asked again next time
        c = per * cus < kConGrid ? per * cus : kConGrid;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// Elements per chunk of the persistent boundary-row solves: as many as two
// nodes per lane hold, with every edge point of the chunk on a lane of its
// own (at n = 13: three elements, against one per block with a lane per
// node; more elements in flight per compute unit, and a third of the
// barriers per element).  Node work runs on "virtual lanes" v = t + 256 k,
// k < PASS.
template <int N> struct ConShape {
    static constexpr int ND = N * N, NB = 4 * N;
    static constexpr int E = (2 * kBlock2) / ND < kBlock2 / NB ? (2 * kBlock2) / ND : kBlock2 / NB;
    static constexpr int PASS = (E * ND + kBlock2 - 1) / kBlock2;
    static_assert(E >= 1 && PASS <= 2 && E * NB <= kBlock2, "constrain chunk shape");
};

// The rows' solution for the chunk's elements once the face values are in
// s_fv and d_B - C_B phihat in s_rb (edge lane te, tt):
//   phi = phihat + C_B^T z, z = Q (d_B - C_B phihat), Q = (C_B C_B^T)^+
// (HARD) or (I + C_B C_B^T)^{-1} (SOFT); then phi is stored and the edge
// lanes take the largest boundary-row residual of the result.
template <int N>
__device__ __forceinline__ void con_chunk_solve(const Step2DArgs& A, const double* s_q, double (*s_rb)[4 * N],
                                                double (*s_d)[4 * N], const double (*s_fv)[4 * N],
                                                double (*s_y)[N * N], const double (&ph)[ConShape<N>::PASS],
                                                const int (&vslot)[ConShape<N>::PASS],
                                                const int (&vp)[ConShape<N>::PASS],
                                                const double (&lc)[ConShape<N>::PASS][4], int base, int nel,
                                                bool bnd, int te, int tt, bool edge, int& fl,
                                                unsigned long long& rmax)
{
    using O = Off2<N>;
    using S = ConShape<N>;
    constexpr int ND = S::ND, NB = S::NB, E = S::E, PASS = S::PASS;
    if (bnd) {
        if (edge) {
            double z = 0.0;
            // a partial unroll: the loads of a full one hold too many VGPRs
#pragma unroll 8
            for (int q = 0; q < NB; ++q) z = fma(s_q[tt * NB + q], s_rb[te][q], z);
            s_d[te][tt] = z;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PASS; ++k) {
        const int slot = vslot[k];
        if (slot < E) {
            const int p = vp[k], i = p % N, j = p / N;
            double phi = ph[k];
            if (bnd)
                phi = ph[k] + lc[k][0] * s_d[slot][j] + lc[k][1] * s_d[slot][N + j] + lc[k][2] * s_d[slot][2 * N + i] +
                      lc[k][3] * s_d[slot][3 * N + i];
            s_y[slot][p] = phi;
            if (base + slot < nel) {
                if (!isfinite(phi)) fl |= FLAG_NONFINITE;
                A.phi_out[(size_t)(base + slot) * ND + p] = phi;
            }
        }
    }
    __syncthreads();
    if (bnd && edge && base + te < nel) {
        const double* tab = A.tab;
        const int side = tt / N, k = tt % N;
        const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
        double tr = 0.0;
        if (side < 2)
            for (int c = 0; c < N; ++c) tr = fma(lv[c], s_y[te][c + N * k], tr);
        else
            for (int c = 0; c < N; ++c) tr = fma(lv[c], s_y[te][k + N * c], tr);
        rmax = abs_bits(tr - s_fv[te][tt]);
    }
}

// The chunk's node lanes: element slot, node, the C_B^T coefficients
// l0(xi_i), l1(xi_i), l0(xi_j), l1(xi_j), and phi-hat
template <int N>
__device__ __forceinline__ void con_chunk_nodes(const Step2DArgs& A, int t, int (&vslot)[ConShape<N>::PASS],
                                                int (&vp)[ConShape<N>::PASS], double (&lc)[ConShape<N>::PASS][4])
{
    using O = Off2<N>;
    using S = ConShape<N>;
#pragma unroll
    for (int k = 0; k < S::PASS; ++k) {
        const int v = t + kBlock2 * k;
        vslot[k] = v / S::ND;
        vp[k] = v - vslot[k] * S::ND;
        const int i = vp[k] % N, j = vp[k] / N;
        lc[k][0] = A.tab[O::L0 + i];
        lc[k][1] = A.tab[O::L1 + i];
        lc[k][2] = A.tab[O::L0 + j];
        lc[k][3] = A.tab[O::L1 + j];
    }
}

template <int N>
__device__ __forceinline__ void con_chunk_load(const Step2DArgs& A, int base, int nel,
                                               const int (&vslot)[ConShape<N>::PASS],
                                               const int (&vp)[ConShape<N>::PASS], double (&ph)[ConShape<N>::PASS])
{
    using S = ConShape<N>;
#pragma unroll
    for (int k = 0; k < S::PASS; ++k) {
        const int li = base + vslot[k];
        ph[k] = (vslot[k] < S::E && li < nel) ? A.phihat[(size_t)li * S::ND + vp[k]] : 0.0;
    }
}

// chunks c0, c0 + stride, ... of the launch; the block's statistics go to
// row sidx of the per-block partials
template <int N, bool BT>
__device__ __forceinline__ void constrain2d_body(const Step2DArgs& A, const int c0, const int stride, const int sidx)
{
    using O = Off2<N>;
    using S = ConShape<N>;
    constexpr int ND = S::ND, NB = S::NB, E = S::E, PASS = S::PASS, NQ = 16 * ND;
    __shared__ double s_q[NQ];
    // per element: z, d_B - C_B phihat, d_B, phi
    __shared__ double s_d[E][NB], s_rb[E][NB], s_fv[E][NB], s_y[E][ND];
    __shared__ int s_flag;
    __shared__ unsigned long long s_stat;

    const int t = threadIdx.x;
    const int kx = A.kx, ky = A.ky, K = A.K;
    const bool bnd = (A.cmask & SL_C_BOUNDARY) != 0;
    const double* Qg = A.tab + (A.mode == SL_MODE_HARD ? O::QH : O::QS);
    for (int k = t; k < NQ; k += kBlock2) s_q[k] = Qg[k];
    if (t == 0) {
        s_flag = 0;
        s_stat = 0ull;
    }
    int vslot[PASS], vp[PASS];
    double lc[PASS][4];
    con_chunk_nodes<N>(A, t, vslot, vp, lc);
    const int te = t / NB, tt = t - te * NB;  // edge lane: element slot, edge point
    const bool edge = te < E;
    const int nchunk = (K + E - 1) / E;
    int fl = 0;
    unsigned long long rmax = 0ull;  // this lane's largest boundary-row residual

    for (int chunk = c0; chunk < nchunk; chunk += stride) {
        const int base = chunk * E;
        double ph[PASS];
        con_chunk_load<N>(A, base, K, vslot, vp, ph);

        // face value at the element's edge point tt: upwind of its own trace
        // and the neighbour's matching trace (eq. 4.12a); ghost values at the
        // domain boundary
        if (edge) {
            const int ee = base + te < K ? base + te : 0;
            int nbe, nbt, gidx;
            bool high;
            face_partner2<N>(ee, tt, kx, ky, A.periodic, nbe, nbt, gidx, high);
            // offered face values: the traces, or with backtracking (BT) the
            // record's last 4n slots; the residual takes the own trace
            const int fo = BT ? A.rstride - NB : 0;
            const double trace = A.rec[(size_t)ee * A.rstride + tt];
            const double mine = BT ? A.rec[(size_t)ee * A.rstride + fo + tt] : trace;
            const double other = nbe >= 0 ? A.rec[(size_t)nbe * A.rstride + fo + nbt] : A.gnext[gidx];
            const double vn = A.vface[(size_t)ee * NB + tt];
            const double lo = high ? other : mine, hi = high ? mine : other;
            const double dv = upwind2(vn, lo, hi);
            s_fv[te][tt] = dv;
            s_rb[te][tt] = dv - trace;
        }
        __syncthreads();
        unsigned long long r = 0ull;
        con_chunk_solve<N>(A, s_q, s_rb, s_d, s_fv, s_y, ph, vslot, vp, lc, base, K, bnd, te, tt, edge, fl, r);
        rmax = r > rmax ? r : rmax;
        __syncthreads();  // s_fv, s_rb, s_d, s_y are rewritten by the next chunk
    }
    slot_max<1>(&s_stat, 0, rmax);  // one block-wide slot: one atomic per wave
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[A.nblk + sidx] |= s_flag;
        double* sp = A.stat_part + (size_t)sidx * kStatSlots;
        sp[0] = fmax(sp[0], __longlong_as_double((long long)s_stat));
    }
}

template <int N, bool BT>
__global__ __launch_bounds__(kBlock2) void k_constrain2d(Step2DArgs A)
{
    constrain2d_body<N, BT>(A, blockIdx.x, gridDim.x, blockIdx.x);
}

// batched: one chunk per block, block start[r] + c doing chunk c of request
// r, whose statistics row c is then its own (a request has no more chunks
// than partial rows from four nodes per direction on)
template <int N>
__global__ __launch_bounds__(kBlock2) void k_constrain2d_batch(const Step2DArgs* __restrict__ As,
                                                               const int* __restrict__ start, int nreq)
{
    const int r = batch_request(start, nreq, blockIdx.x);
    const int c = blockIdx.x - start[r];
    constrain2d_body<N, false>(As[r], c, 1 << 30, c);
}

// ---------------------------------------------------------------------------
// boundary-constrained least squares with mass and energy rows (2D)
//
// With the boundary rows' solution `base` (as in k_constrain2d) and the
// extra rows G (mass W, energy W o phi linearised at the previous iterate),
// both modes take the form
//   phi = base + Z S^{-1} (d_G - G base),  Z = P G^T,  S = G Z (+ I in SOFT),
// with P = I - C_B^T Q C_B: the projector onto null(C_B) for HARD (Q =
// (C_B C_B^T)^+, the prioritised reading), and (I + C_B^T C_B)^{-1} by
// Woodbury for SOFT (Q = (I + C_B C_B^T)^{-1}), i.e. the paper's stacked
// least squares.  Without boundary rows P = I and base = phi-hat.  P W is a
// per-mesh table.
// Persistent: each block takes chunks of floor(256/n^2) elements (one lane
// per node), blockIdx.x, blockIdx.x + gridDim.x, ..., with Q staged once.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kBlock2) void k_constrain2d_me(Step2DArgs A)
{
    using O = Off2<N>;
    constexpr int ND = N * N, E = kBlock2 / ND, NB = 4 * N, NQ = 16 * ND, NDOT = 5;
    __shared__ double s_q[NQ];
    __shared__ double s_fv[E][NB], s_tr[E][NB], s_w[E][NB];
    __shared__ double s_v[E][ND];
    __shared__ double s_red[E][NDOT][ND];
    __shared__ double s_dot[E][NDOT];
    __shared__ double s_tgt[E][3];
    __shared__ unsigned long long s_mx[E][2];
    __shared__ int s_flag, s_pic;
    __shared__ unsigned long long s_stat[3];

    const int t = threadIdx.x;
    const int slot = t / ND, p = t - slot * ND;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const double* __restrict__ tab = A.tab;
    const bool bnd = (A.cmask & SL_C_BOUNDARY) != 0;
    const bool mass = (A.cmask & SL_C_MASS) != 0;
    const bool energy = (A.cmask & SL_C_ENERGY) != 0;
    const bool soft = A.mode == SL_MODE_SOFT;
    const double* Qg = tab + (soft ? O::QS : O::QH);
    for (int k = t; k < NQ; k += kBlock2) s_q[k] = Qg[k];
    if (t == 0) {
        s_flag = 0;
        s_pic = 0;
        s_stat[0] = s_stat[1] = s_stat[2] = 0ull;
    }
    if (t < 2 * E) s_mx[t / 2][t % 2] = 0ull;
    const int i = p % N, j = p / N;
    const double l0i = tab[O::L0 + i], l1i = tab[O::L1 + i], l0j = tab[O::L0 + j], l1j = tab[O::L1 + j];
    const double Wp = A.dx * A.dy * tab[O::W + i] * tab[O::W + j];
    // mass row: Z_M = P W from the table (P W is W without boundary rows)
    const double zm = bnd ? A.dx * A.dy * tab[(soft ? O::ZMS : O::ZMH) + p] : Wp;
    const int nchunk = (A.K + E - 1) / E;
    int fl = 0;

    // persistent: chunks of E elements, blockIdx.x + c gridDim.x for c = 0, 1, ...
    for (int chunk = blockIdx.x; chunk < nchunk; chunk += gridDim.x) {
        const int e = chunk * E + slot;
        const bool live = inblk && e < A.K;
        const int ee = live ? e : 0;
        const double* rec = A.rec + (size_t)ee * A.rstride;
        const double ph = live ? A.phihat[(size_t)ee * ND + p] : 0.0;
        const double cme = rec[3 * NB + 2];  // the element's mean at t^n

        // the element's local mass and deviation energy terms, loaded with the
        // face data below: every load of the chunk is issued before the first
        // wait (one memory latency per chunk)
        const double Mloc = rec[3 * NB], Eloc = rec[3 * NB + 1];

        // face values (eq. 4.12a) and the face terms of the targets: inflow
        // positive, the upwind side's stage sums (own, neighbour's or ghost)
        const RKTab& T = A.rk;
        for (int tt = p; inblk && tt < NB; tt += ND) {
            int nbe, nbt, gidx;
            bool high;
            face_partner2<N>(ee, tt, A.kx, A.ky, A.periodic, nbe, nbt, gidx, high);
            const double vn = A.vface[(size_t)ee * NB + tt];
            // offered face values: the traces, or with backtracking the record's
            // last NB slots
            const int fo = A.iface == SL_IFACE_BACKTRACK ? A.rstride - NB : 0;
            const double mine = rec[fo + tt];
            const double other = nbe >= 0 ? A.rec[(size_t)nbe * A.rstride + fo + nbt] : A.gnext[gidx];
            // both sides' stage sums, whichever is upwind: the choice waits
            // for vn, the loads do not
            const double* rn = A.rec + (size_t)(nbe >= 0 ? nbe : ee) * A.rstride;
            const double s1o = rec[NB + tt], s2o = rec[2 * NB + tt];
            const double s1n = rn[NB + nbt], s2n = rn[2 * NB + nbt], cn = rn[3 * NB + 2];
            const double g0 = nbe >= 0 ? 0.0 : A.gnow[gidx];
            const double fwt = tab[O::W + tt % N];
            s_fv[slot][tt] = upwind2(vn, high ? other : mine, high ? mine : other);
            double fm = 0.0, fe = 0.0;
            if (vn != 0.0) {
                const bool up = high ? vn < 0.0 : vn > 0.0;
                // sum_q b_q v_q and sum_q b_q (v_q - c)^2 about this element's
                // mean c; a neighbour's sums are about its own mean c', so with
                // delta = c' - c: S2 + delta (2 S1 + delta) and S1 + c'
                double sm, se;
                if (up) {
                    sm = s1o + cme;
                    se = s2o;
                } else if (nbe >= 0) {
                    const double dl = cn - cme;
                    sm = s1n + cn;
                    se = fma(dl, fma(2.0, s1n, dl), s2n);
                } else {
                    // inflow from outside: ghost values, linear in time
                    sm = se = 0.0;
                    for (int c = 0; c < T.nq; ++c) {
                        const double g = (1.0 - T.cu[c]) * g0 + T.cu[c] * other;
                        sm = fma(T.bu[c], g, sm);
                        se = fma(T.bu[c], (g - cme) * (g - cme), se);
                    }
                }
                const int side = tt / N;
                const double fw = (side < 2 ? A.dy : A.dx) * fwt;
                const double sg = high ? vn : -vn;
                fm = sg * fw * sm;
                fe = sg * fw * se;
            }
            s_tr[slot][tt] = fm;
            s_w[slot][tt] = fe;
        }
        __syncthreads();
        if (live && p == 0) {
            double fm = 0.0, fe = 0.0;
            for (int tt = 0; tt < NB; ++tt) {
                fm += s_tr[slot][tt];
                fe += s_w[slot][tt];
            }
            const double Mn = Mloc + A.dt * fm, Ed = Eloc + A.dt * fe;
            s_tgt[slot][0] = Mn;
            s_tgt[slot][1] = Ed;
            s_tgt[slot][2] = Ed + cme * (2.0 * Mn - cme * A.sumW);
        }
        __syncthreads();
        // M^{n+1}, the deviation energy Ed^{n+1} = sum W (phi - c)^2 and the
        // energy E^{n+1} = Ed + 2 c M - c^2 sum W of phi^2
        const double Mt = s_tgt[sl][0], Edt = s_tgt[sl][1], Et = s_tgt[sl][2];

        // element-wise sums of up to NDOT per-node values, in a fixed order
        auto dots = [&](int k, const double* vals) {
            if (inblk)
                for (int c = 0; c < k; ++c) s_red[slot][c][p] = vals[c];
            __syncthreads();
            for (int c = p; inblk && c < k; c += ND) {
                double s = 0.0;
                for (int r = 0; r < ND; ++r) s += s_red[slot][c][r];
                s_dot[slot][c] = s;
            }
            __syncthreads();
        };
        // C_B^T Q (h - C_B v) at this node, v in s_v; h = d_B (face values) or 0
        auto cbt_q = [&](bool with_data) -> double {
            for (int tt = p; inblk && tt < NB; tt += ND) {
                const int side = tt / N, k = tt % N;
                const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
                double tr = 0.0;
                if (side < 2)
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_v[slot][c + N * k], tr);
                else
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_v[slot][k + N * c], tr);
                s_tr[slot][tt] = (with_data ? s_fv[slot][tt] : 0.0) - tr;
            }
            __syncthreads();
            for (int tt = p; inblk && tt < NB; tt += ND) {
                double z = 0.0;
    #pragma unroll 8
                for (int c = 0; c < NB; ++c) z = fma(s_q[tt * NB + c], s_tr[slot][c], z);
                s_w[slot][tt] = z;
            }
            __syncthreads();
            const double r = l0i * s_w[sl][j] + l1i * s_w[sl][N + j] + l0j * s_w[sl][2 * N + i] +
                             l1j * s_w[sl][3 * N + i];
            __syncthreads();  // s_v, s_tr, s_w are rewritten by the next call
            return r;
        };

        // boundary rows: base = phihat + C_B^T Q (d_B - C_B phihat)
        double base = ph;
        if (bnd) {
            if (inblk) s_v[slot][p] = ph;
            __syncthreads();
            base = ph + cbt_q(true);
        }
        const double shift = soft ? 1.0 : 0.0;
        double gb = 0.0, gz = 0.0;
        double cur = base;
        if (mass) {
            const double v[2] = {Wp * base, Wp * zm};
            dots(2, v);
            gb = s_dot[sl][0];
            gz = s_dot[sl][1];
            const double S = gz + shift;
            if (!(S != 0.0) || !isfinite(S)) fl |= FLAG_SINGULAR;
            cur = base + zm * ((Mt - gb) / S);
        }
        double prev = cur;
        int picard = 0;
        // the energy row (section "Local energy conservation").  SOFT: the
        // paper's linearisation sum W phi^(k-1) phi = E^{n+1}, stacked.  HARD:
        // its fixed point, reached by Newton's linearisation of the same row,
        // written for y = phi - sh with the target Tt:
        //   sum W y^(k-1) y = (Tt + sum W (y^(k-1))^2) / 2,
        // with a mass row as the deviation from the element's mean (sh = c,
        // Tt = Ed^{n+1}: the same constraint on the mass row's level set),
        // otherwise sh = 0, Tt = E^{n+1}.  Stop when max |phi^(k) - phi^(k-1)|
        // < tol (strict, as printed).  Where the linearised row lies in the span
        // of the others the sweep makes no change (singular if the row is not
        // met).
        const bool devf = !soft && mass;
        const double sh = devf ? cme : 0.0;
        if (energy) {
            const double Tt = devf ? Edt : Et;
            bool done = !live, conv = false;
            for (int k = 1; k <= A.emaxit; ++k) {
                const double yv = prev - sh;
                const double gE = Wp * yv;
                if (inblk) s_v[slot][p] = gE;
                __syncthreads();
                const double zE = bnd ? gE + cbt_q(false) : gE;
                double sig_m = 0.0, sig_e = 0.0, numer;
                bool ok;
                if (mass) {
                    const double v[5] = {Wp * zE, gE * zm, gE * zE, gE * (base - sh), gE * yv};
                    dots(5, v);
                    const double a11 = gz + shift, a12 = s_dot[sl][0], a21 = s_dot[sl][1], a22 = s_dot[sl][2] + shift;
                    const double r1 = Mt - gb;
                    const double r2 = (soft ? Et : 0.5 * (Tt + s_dot[sl][4])) - s_dot[sl][3];
                    const double det = a11 * a22 - a12 * a21;
                    numer = a11 * r2 - a21 * r1;
                    ok = det != 0.0 && isfinite(det);
                    sig_m = ok ? (r1 * a22 - a12 * r2) / det : 0.0;
                    sig_e = ok ? numer / det : 0.0;
                } else {
                    const double v[3] = {gE * zE, gE * (base - sh), gE * yv};
                    dots(3, v);
                    const double S = s_dot[sl][0] + shift;
                    numer = (soft ? Et : 0.5 * (Tt + s_dot[sl][2])) - s_dot[sl][1];
                    ok = S != 0.0 && isfinite(S);
                    sig_e = ok ? numer / S : 0.0;
                }
                const double nxt = ok ? base + zm * sig_m + zE * sig_e : prev;
                const bool act = inblk && !done;
                if (act && !ok && numer != 0.0) fl |= FLAG_SINGULAR;
                if constexpr (ND >= 64) {
                    slot_max<E, 2>(&s_mx[0][0], slot, act ? abs_bits(nxt - prev) : 0ull);
                } else if (act) {
                    atomicMax(&s_mx[slot][0], abs_bits(nxt - prev));
                }
                __syncthreads();
                if (inblk && !done) {
                    const double diff = __longlong_as_double((long long)s_mx[slot][0]);
                    prev = nxt;
                    picard = k;
                    if (diff < A.etol) {
                        conv = true;
                        done = true;
                    }
                }
                const bool all = __syncthreads_and(done);
                if (t < 2 * E) s_mx[t / 2][t % 2] = 0ull;
                __syncthreads();
                if (all) break;
            }
            if (live && !conv && A.etol > 0.0) fl |= FLAG_NOCONV;
        }

        // store, residuals: boundary (traces of phi vs the face values), mass,
        // energy
        const double phi = prev;
        if (live) {
            if (!isfinite(phi)) fl |= FLAG_NONFINITE;
            A.phi_out[(size_t)e * ND + p] = phi;
        }
        if (inblk) s_v[slot][p] = phi;
        {
            // energy residual of the row as imposed: HARD with a mass row in the
            // deviation form, otherwise sum W phi^2 against E^{n+1}
            const double v[2] = {Wp * phi, Wp * (phi - sh) * (phi - sh)};
            dots(2, v);  // its first barrier also publishes s_v
        }
        unsigned long long rmax = 0ull;  // this lane's largest boundary-row residual
        if (live) {
            for (int tt = p; bnd && tt < NB; tt += ND) {
                const int side = tt / N, k = tt % N;
                const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
                double tr = 0.0;
                if (side < 2)
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_v[slot][c + N * k], tr);
                else
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_v[slot][k + N * c], tr);
                const unsigned long long r = abs_bits(tr - s_fv[slot][tt]);
                rmax = r > rmax ? r : rmax;
            }
        }
        slot_max<1>(&s_stat[0], 0, rmax);  // one block-wide slot: one atomic per wave
        if (live) {
            if (p == 0) {
                if (mass) atomicMax(&s_stat[1], (unsigned long long)__double_as_longlong(fabs(s_dot[slot][0] - Mt)));
                if (energy)
                    atomicMax(&s_stat[2],
                              (unsigned long long)__double_as_longlong(fabs(s_dot[slot][1] - (devf ? Edt : Et))));
                atomicMax(&s_pic, picard);
            }
        }
        __syncthreads();  // the chunk's shared rows are rewritten by the next
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[A.nblk + blockIdx.x] |= s_flag;
        double* sp = A.stat_part + (size_t)blockIdx.x * kStatSlots;
        sp[0] = fmax(sp[0], __longlong_as_double((long long)s_stat[0]));
        sp[1] = fmax(sp[1], __longlong_as_double((long long)s_stat[1]));
        sp[2] = fmax(sp[2], __longlong_as_double((long long)s_stat[2]));
        sp[3] = fmax(sp[3], (double)s_pic);
    }
}

// ---------------------------------------------------------------------------
// mixed-order meshes (periodic, boundary rows): elements are grouped in
// buckets of one order; each launch covers one bucket.  The face value at an
// element's own edge point comes from the upwind side; when the neighbour
// has another order its edge polynomial (its n' traces along the shared
// edge) is interpolated to this element's edge nodes by a precomputed
// n x n' Lagrange matrix, which is exact for that polynomial.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void periodic_partner(int e, int side, int kx, int ky, int& nbe, bool& high)
{
    const int ex = e % kx, ey = e / kx;
    switch (side) {
    case 0: nbe = ey * kx + (ex + kx - 1) % kx; high = true; break;
    case 1: nbe = ey * kx + (ex + 1) % kx; high = false; break;
    case 2: nbe = ((ey + ky - 1) % ky) * kx + ex; high = true; break;
    default: nbe = ((ey + 1) % ky) * kx + ex; high = false; break;
    }
}

// normal velocity of element j of bucket b (order n) at its own edge point
// q of side sd: the u (x-faces) or v (y-faces) interpolant on that edge
__device__ double edge_speed_mixed(const int* meta, const double* __restrict__ aN_all,
                                   const double* __restrict__ tab_all, int b, int j, int sd, int q)
{
    const int n = meta[MixMeta::kN + b], nd = n * n;
    const double* lv = tab_all + meta[MixMeta::kTab + b] + ((sd & 1) ? 3 * n : 2 * n);  // l(1) or l(0)
    const double* base = aN_all + meta[MixMeta::kVel + b];
    double s = 0.0;
    if (sd < 2) {
        const double* U = base + (size_t)j * nd;
        for (int c = 0; c < n; ++c) s = fma(lv[c], U[c + n * q], s);
    } else {
        const double* V = base + ((size_t)meta[MixMeta::kK + b] + j) * nd;
        for (int c = 0; c < n; ++c) s = fma(lv[c], V[q + n * c], s);
    }
    return s;
}

// face normal velocity at the own edge points of one bucket's elements: the
// mean of this element's normal velocity interpolant and the neighbour's,
// both at this element's edge node (the neighbour's edge values
// interpolated when its order differs); at or below vzero it is zero
template <int N>
__global__ void k_facevel2d_mixed(int K_b, int bucket, int kx, int ky, const int32_t* __restrict__ elems,
                                  const int32_t* __restrict__ mix, const double* __restrict__ aN_all,
                                  const double* __restrict__ tab_all, const double* __restrict__ interp,
                                  double vzero, double* __restrict__ vface)
{
    constexpr int NB = 4 * N;
    const int K = kx * ky;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long)K_b * NB) return;
    const int i = (int)(gid / NB), tt = (int)(gid % NB);
    const int side = tt / N, k = tt % N;
    const int e = elems[i];
    const int* meta = mix + 2 * K;
    double vn = edge_speed_mixed(meta, aN_all, tab_all, bucket, i, side, k);
    int nbe;
    bool high;
    periodic_partner(e, side, kx, ky, nbe, high);
    const int b2 = mix[nbe], j2 = mix[K + nbe];
    const int n2 = meta[MixMeta::kN + b2];
    const int s2 = side ^ 1;  // the neighbour's side on the shared face
    double other = 0.0;
    if (n2 == N) {
        other = edge_speed_mixed(meta, aN_all, tab_all, b2, j2, s2, k);
    } else {
        const double* M = interp + meta[MixMeta::kInterp + kMaxBuckets * bucket + b2];
        for (int q = 0; q < n2; ++q) other = fma(M[k * n2 + q], edge_speed_mixed(meta, aN_all, tab_all, b2, j2, s2, q), other);
    }
    vn = 0.5 * (vn + other);
    if (fabs(vn) <= vzero) vn = 0.0;
    vface[(size_t)i * NB + tt] = vn;
}

// boundary least squares of one bucket's elements (as k_constrain2d), with
// the neighbour's trace taken from its bucket and interpolated to this
// element's edge nodes when the orders differ
template <int N>
__global__ __launch_bounds__(kBlock2) void k_constrain2d_mixed(Step2DArgs A)
{
    using O = Off2<N>;
    using S = ConShape<N>;
    constexpr int ND = S::ND, NB = S::NB, E = S::E, PASS = S::PASS, NQ = 16 * ND;
    __shared__ double s_q[NQ];
    __shared__ double s_d[E][NB], s_rb[E][NB], s_fv[E][NB], s_y[E][ND];
    __shared__ int s_flag;
    __shared__ unsigned long long s_stat;

    const int t = threadIdx.x;
    const int K_b = A.K;
    const double* Qg = A.tab + (A.mode == SL_MODE_HARD ? O::QH : O::QS);
    for (int k = t; k < NQ; k += kBlock2) s_q[k] = Qg[k];
    if (t == 0) {
        s_flag = 0;
        s_stat = 0ull;
    }
    int vslot[PASS], vp[PASS];
    double lc[PASS][4];
    con_chunk_nodes<N>(A, t, vslot, vp, lc);
    const int te = t / NB, tt = t - te * NB;  // edge lane: element slot, edge point
    const bool edge = te < E;
    const int side = tt / N, k = tt % N;
    const bool high = side == 0 || side == 2;  // e is the high side of its left and bottom faces
    const int nchunk = (K_b + E - 1) / E;
    int fl = 0;
    unsigned long long rmax = 0ull;  // this lane's largest boundary-row residual

    for (int chunk = blockIdx.x; chunk < nchunk; chunk += gridDim.x) {
        const int base = chunk * E;
        double ph[PASS];
        con_chunk_load<N>(A, base, K_b, vslot, vp, ph);

        if (edge) {
            const int ll = base + te < K_b ? base + te : 0;  // index within the bucket
            // the neighbour's trace row from the face partner table (one load
            // where the topology lookup took a chain of four)
            const int32_t* f = A.nbr + (size_t)ll * MixFace::kPer + side * MixFace::kField;
            const int n2 = f[MixFace::kOrder];
            const double* tr2 = A.rec_all + f[MixFace::kRecOff];
            double other = 0.0;
            if (n2 == N) {
                other = tr2[k];
            } else {
                // the interpolation in groups of 4 whose loads are independent (one
                // latency per group): indices clamped to the row, terms past its
                // end multiplied by zero (the same sum)
                const double* M = A.interp + f[MixFace::kInterpOff] + k * n2;
                for (int q0 = 0; q0 < n2; q0 += 4) {
                    double mv[4], tv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int q = q0 + u, qq = q < n2 ? q : n2 - 1;
                        mv[u] = M[qq];
                        tv[u] = tr2[qq];
                        if (q >= n2) tv[u] = 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) other = fma(mv[u], tv[u], other);
                }
            }
            const double mine = A.rec[(size_t)ll * NB + tt];
            const double vn = A.vface[(size_t)ll * NB + tt];
            const double dv = upwind2(vn, high ? other : mine, high ? mine : other);
            s_fv[te][tt] = dv;
            s_rb[te][tt] = dv - mine;
        }
        __syncthreads();
        unsigned long long r = 0ull;
        con_chunk_solve<N>(A, s_q, s_rb, s_d, s_fv, s_y, ph, vslot, vp, lc, base, K_b, true, te, tt, edge, fl, r);
        rmax = r > rmax ? r : rmax;
        __syncthreads();  // s_fv, s_rb, s_d, s_y are rewritten by the next chunk
    }
    slot_max<1>(&s_stat, 0, rmax);  // one block-wide slot: one atomic per wave
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[A.nblk + blockIdx.x] |= s_flag;
        double* sp = A.stat_part + (size_t)blockIdx.x * kStatSlots;
        sp[0] = fmax(sp[0], __longlong_as_double((long long)s_stat));
    }
}

template <int N>
int prep_n(int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM,
           const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s)
{
    const int bs = 64;
    hipLaunchKernelGGL(k_prep2d<N>, dim3((K + bs - 1) / bs), dim3(bs), 0, s, K, has_div, cons, aN, aM, divN, divM,
                       tab, 1.0 / dx, 1.0 / dy, vscale, vdeg);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int facevel_n(int kx, int ky, int periodic, const double* aN, const double* tab, double vzero, double* vface,
              hipStream_t s)
{
    const int bs = 256;
    const long tot = (long)kx * ky * 4 * N;
    hipLaunchKernelGGL(k_facevel2d<N>, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s, kx, ky, periodic, aN,
                       tab, vzero, vface);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N, int PR>
void adv_launch(const Step2DArgs& A, dim3 grid, hipStream_t s)
{
    launch_timed((k_advect2d<N, PR>), grid, dim3(kBlock2), 0, s, A);
}

// Every block of an advect or constrain launch owns a row of the per-block
// statistics and flags, which hold A.nblk rows: a launch with more blocks is
// refused on the host (it would write past them).
template <int N, int BSEL>
int adv_shape(const Step2DArgs& A, hipStream_t s)
{
    using S = Shape2<N, BSEL>;
    const int grid = (A.K + S::E - 1) / S::E;
    if (grid > A.nblk) return 1;
    launch_timed((k_advect2d<N, 0, BSEL>), dim3(grid), dim3(S::BS), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int adv_n(const Step2DArgs& A, hipStream_t s)
{
    // the alternative block shapes exist for the FP64 kernel
    if (A.bs != 0 && A.precision == SL_PREC_FP64)
        return A.bs == 1 ? adv_shape<N, 1>(A, s) : adv_shape<N, 2>(A, s);
    // the 256-lane shape (and the reduced-precision variants, which exist
    // for it only) holds no element above 16 nodes per direction
    if constexpr (N * N > kBlock2) {
        return 1;
    } else {
    constexpr int E = kBlock2 / (N * N);
    const dim3 grid((A.K + E - 1) / E);
    if ((int)grid.x > A.nblk) return 1;
    if (A.precision == SL_PREC_FP32_REFINED) adv_launch<N, 1>(A, grid, s);
    else if (A.precision == SL_PREC_BF16_REFINED) adv_launch<N, 2>(A, grid, s);
    else adv_launch<N, 0>(A, grid, s);
    return hipGetLastError() == hipSuccess ? 0 : 1;
    }
}

// grid of a persistent constrain launch over nchunk chunks: no more blocks
// than are resident at once (r), nor than the per-block partials hold
inline int con_grid(int nchunk, int r, int nblk)
{
    int g = nchunk < r ? nchunk : r;
    return g < nblk ? g : nblk;
}

template <int N>
int con_n(const Step2DArgs& A, hipStream_t s)
{
    static std::atomic<int> cap_bt[kMaxDevices], cap[kMaxDevices];
    if (A.nblk < 1) return 1;
    if (A.cmask & (SL_C_MASS | SL_C_ENERGY)) {
        if constexpr (N * N > kBlock2) {
            return 1;  // one lane per node: up to 16 nodes per direction
        } else {
            constexpr int E = kBlock2 / (N * N);
            const int nchunk = (A.K + E - 1) / E;
            if (nchunk > A.nblk) return 1;
            static std::atomic<int> cap_me[kMaxDevices];
            const int r = resident_blocks(k_constrain2d_me<N>, cap_me);
            launch_timed(k_constrain2d_me<N>, dim3(con_grid(nchunk, r, A.nblk)), dim3(kBlock2), 0, s, A);
            return hipGetLastError() == hipSuccess ? 0 : 1;
        }
    }
    const int nchunk = (A.K + ConShape<N>::E - 1) / ConShape<N>::E;
    if (A.iface == SL_IFACE_BACKTRACK) {
        const int r = resident_blocks(k_constrain2d<N, true>, cap_bt);
        launch_timed((k_constrain2d<N, true>), dim3(con_grid(nchunk, r, A.nblk)), dim3(kBlock2), 0, s, A);
    } else {
        const int r = resident_blocks(k_constrain2d<N, false>, cap);
        launch_timed((k_constrain2d<N, false>), dim3(con_grid(nchunk, r, A.nblk)), dim3(kBlock2), 0, s, A);
    }
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

// batched launches (boundary rows, interpolated face values): the advect's
// variant (precision, block shape) is A0's, which every member shares
template <int N>
int adv_batch_n(const Step2DArgs& A0, const Step2DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s)
{
    const dim3 grid(nblocks);
    if (A0.targets) return 1;
    if (A0.bs == 1 && A0.precision == SL_PREC_FP64) {
        hipLaunchKernelGGL((k_advect2d_batch<N, 0, 1>), grid, dim3(Shape2<N, 1>::BS), 0, s, As, start, nreq);
    } else if constexpr (N * N > kBlock2) {
        return 1;
    } else {
        if (A0.bs != 0) return 1;
        if (A0.precision == SL_PREC_FP32_REFINED)
            hipLaunchKernelGGL((k_advect2d_batch<N, 1, 0>), grid, dim3(kBlock2), 0, s, As, start, nreq);
        else if (A0.precision == SL_PREC_BF16_REFINED)
            hipLaunchKernelGGL((k_advect2d_batch<N, 2, 0>), grid, dim3(kBlock2), 0, s, As, start, nreq);
        else
            hipLaunchKernelGGL((k_advect2d_batch<N, 0, 0>), grid, dim3(kBlock2), 0, s, As, start, nreq);
    }
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int con_batch_n(const Step2DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_constrain2d_batch<N>, dim3(nblocks), dim3(kBlock2), 0, s, As, start, nreq);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

// backtracking interface values (eq. 4.11), a launch of their own before
// the advect kernel: one lane per edge point (4n per element, floor(256/4n)
// elements per block).  phi^n and the velocity (and divergence) series of
// each element are staged in LDS; a lane whose point lies on a face where
// the flow leaves the element (or the face speed vanishes) traces the
// characteristic back over dt and stores phi^n at the foot, times the
// source factor in the conservative form, in the record's last 4n slots.
// The other points store zero: the upwind rule never selects them.
template <int N>
__global__ __launch_bounds__(kBlock2) void k_backtrace2d(Step2DArgs A)
{
    using O = Off2<N>;
    constexpr int ND = N * N, NB = 4 * N, EB = kBlock2 / NB;
    __shared__ double s_f[EB][ND], s_cu[EB][ND], s_cv[EB][ND], s_cd[EB][ND];
    __shared__ int s_flag;
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * EB;
    if (t == 0) s_flag = 0;
    const size_t KND = (size_t)A.K * ND;
    for (int k = t; k < EB * ND; k += kBlock2) {
        const int le = k / ND, q = k - le * ND, e = e0 + le;
        const bool live = e < A.K;
        const size_t g = (size_t)(live ? e : 0) * ND + q;
        const int ii = q % N, jj = q / N;
        const bool used = live && ii <= A.vdeg && jj <= A.vdeg;
        s_f[le][q] = live ? A.phi[g] : 0.0;
        s_cu[le][q] = used ? A.aM[g] : 0.0;
        s_cv[le][q] = used ? A.aM[KND + g] : 0.0;
        s_cd[le][q] = (used && A.cons) ? A.divM[g] : 0.0;
    }
    __syncthreads();
    const int le = t / NB, tt = t - le * NB, e = e0 + le;
    bool out = false;
    if (le < EB && e < A.K) {
        const int side = tt / N, k = tt % N;
        const double vn = A.vface[(size_t)e * NB + tt];
        const bool up = (side == 0 || side == 2) ? vn <= 0.0 : vn >= 0.0;
        double v = 0.0;
        if (up) {
            const double s = side == 0 ? 0.0 : side == 1 ? 1.0 : A.tab[O::XI + k];
            const double r = side == 2 ? 0.0 : side == 3 ? 1.0 : A.tab[O::XI + k];
            v = backtrace2<N>(A, s_cu[le], s_cv[le], s_cd[le], s_f[le], A.dt, s, r, out, A.tab + O::XI,
                              A.tab + O::LAM);
        }
        A.rec[(size_t)e * A.rstride + (A.rstride - NB) + tt] = v;
    }
    if (out) atomicOr(&s_flag, FLAG_CONTAIN);
    __syncthreads();
    // the advect kernel's flag slots; several blocks may share one
    if (t == 0 && s_flag) atomicOr(&A.flag_part[blockIdx.x % A.nblk], s_flag);
}

template <int N>
int bt_n(const Step2DArgs& A, hipStream_t s)
{
    constexpr int EB = kBlock2 / (4 * N);
    launch_timed(k_backtrace2d<N>, dim3((A.K + EB - 1) / EB), dim3(kBlock2), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

// The local parts of the mass and energy targets (eq. 4.14 with the energy
// taken for the deviation from the element's mean, generalised to the RK
// quadrature), a launch of their own before the advect with mass or energy
// rows; EB = floor(256 / 4n) elements per block, one lane per edge point.
// Into record slots of element e, after its 4n edge traces:
//   [4n, 8n)   per edge point where e is upwind, sum_q bu_q (v_q - c), and
//   [8n, 12n)  sum_q bu_q (v_q - c)^2, of phi^n at the foot v_q of the
//              characteristic through the point for each of the tableau's
//              distinct abscissae, about the element's mean c at t^n (zero
//              at the other points);
//   12n        M^n + dt sum_q bu_q V_q,
//   12n + 1    sum W (phi^n - c)^2 + dt sum_q bu_q V'_q, with the volume
//              terms V, V' of the mass and deviation energy balance laws
//              (mass: +div phi in advective form; deviation energy: +div psi^2
//              advective, -div (psi^2 + 2 c psi) conservative), each node's
//              share summed in node order;
//   12n + 2    c.
// In the advect these backtraces held the kernel's registers (two waves per
// SIMD in place of four) for every step with targets, whether the flow has
// volume terms or not.
// Three waves per SIMD (at most 168 VGPRs, a few spilled slots at n = 9):
// C3 with mass rows 300 -> 266 us against two waves at 235 VGPRs; at four
// waves the spills cost more than the occupancy gains (376 us).
template <int N>
__global__ __launch_bounds__(kBlock2, 3) void k_targets2d(Step2DArgs A)
{
    using O = Off2<N>;
    constexpr int ND = N * N, NB = 4 * N, EB = kBlock2 / NB;
    __shared__ double s_f[EB][ND], s_cu[EB][ND], s_cv[EB][ND], s_cd[EB][ND];
    __shared__ double s_m[EB][ND], s_e[EB][ND], s_dv[EB][ND];
    __shared__ double s_mean[EB], s_tw[N], s_txi[N], s_lam[N];  // + weights, nodes, barycentric weights
    __shared__ int s_flag;
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * EB;
    if (t == 0) s_flag = 0;
    if (t < N) {
        s_tw[t] = A.tab[O::W + t];
        s_txi[t] = A.tab[O::XI + t];
        s_lam[t] = A.tab[O::LAM + t];
    }
    const size_t KND = (size_t)A.K * ND;
    for (int k = t; k < EB * ND; k += kBlock2) {
        const int le = k / ND, q = k - le * ND, e = e0 + le;
        const bool live = e < A.K;
        const size_t g = (size_t)(live ? e : 0) * ND + q;
        const int ii = q % N, jj = q / N;
        const bool used = live && ii <= A.vdeg && jj <= A.vdeg;
        s_f[le][q] = live ? A.phi[g] : 0.0;
        s_cu[le][q] = used ? A.aM[g] : 0.0;
        s_cv[le][q] = used ? A.aM[KND + g] : 0.0;
        s_cd[le][q] = (used && A.cons) ? A.divM[g] : 0.0;
        s_dv[le][q] = (live && A.vol) ? A.divN[g] : 0.0;
    }
    __syncthreads();
    // the element's mean at t^n, c = M^n / sum W: the energy balance is
    // taken for the deviation phi - c, computed from differences of like size
    if (t < EB) {
        double cmean = 0.0, sw = 0.0;
        for (int pp = 0; pp < ND; ++pp) {
            const double wq = s_tw[pp % N] * s_tw[pp / N];
            cmean = fma(wq, s_f[t][pp], cmean);
            sw += wq;
        }
        s_mean[t] = cmean / sw;
    }
    __syncthreads();
    const RKTab& T = A.rk;
    const int le = t / NB, tt = t - le * NB, e = e0 + le;
    const bool live = le < EB && e < A.K;
    bool out = false;
    if (live) {
        const double cmean = s_mean[le];
        double* rec = A.rec + (size_t)e * A.rstride;
        // work items of lane tt: its edge point, then the nodes tt, tt + 4n, ...
        // (one backtrace call site for both: two would hold the registers of both)
#pragma unroll 1
        for (int it = tt; it < NB + ND; it += NB) {
            const bool edge = it < NB;
            const int q = edge ? 0 : it - NB;
            const int ii = q % N, jj = q / N;
            double s, r, dv_p = 0.0;
            bool act;
            if (edge) {
                const int side = tt / N, k = tt % N;
                const double vn = A.vface[(size_t)e * NB + tt];
                // e is upwind where the flow leaves it: left/bottom faces
                // for vn < 0, right/top faces for vn > 0
                act = (side == 0 || side == 2) ? vn < 0.0 : vn > 0.0;
                s = side == 0 ? 0.0 : side == 1 ? 1.0 : s_txi[k];
                r = side == 2 ? 0.0 : side == 3 ? 1.0 : s_txi[k];
            } else {
                // volume terms where the velocity has a divergence at the node
                dv_p = s_dv[le][q];
                act = dv_p != 0.0;
                s = s_txi[ii];
                r = s_txi[jj];
            }
            double vm = 0.0, vd = 0.0, ve = 0.0;
            if (act) {
                // one trace at a time: interleaved, they would hold the registers of all
#pragma unroll 1
                for (int c = 0; c < T.nq; ++c) {
                    // no LDS value is kept in registers from one trace to
                    // the next (they would be held through all of them)
                    __asm__ __volatile__("" ::: "memory");
                    const double v = backtrace2<N>(A, s_cu[le], s_cv[le], s_cd[le], s_f[le], T.cu[c] * A.dt, s, r,
                                                   out, s_txi, s_lam);
                    const double dv = v - cmean;
                    vm = fma(T.bu[c], v, vm);
                    vd = fma(T.bu[c], dv, vd);
                    ve = fma(T.bu[c], dv * dv, ve);
                }
            }
            if (edge) {
                rec[NB + tt] = vd;
                rec[2 * NB + tt] = ve;
            } else {
                // the node's share of the local mass and deviation energy
                const double phi_p = s_f[le][q];
                const double Wp = A.dx * A.dy * s_tw[ii] * s_tw[jj];
                const double dn = phi_p - cmean;
                double cm = Wp * phi_p, ce = Wp * dn * dn;
                if (act) {
                    if (!A.cons) cm += A.dt * Wp * dv_p * vm;
                    ce += A.dt * Wp * dv_p * (A.cons ? -fma(2.0 * cmean, vd, ve) : ve);
                }
                s_m[le][q] = cm;
                s_e[le][q] = ce;
            }
        }
    }
    if (out) atomicOr(&s_flag, FLAG_CONTAIN);
    __syncthreads();
    if (t < EB && e0 + t < A.K) {
        double M = 0.0, En = 0.0;
        for (int p = 0; p < ND; ++p) {
            M += s_m[t][p];
            En += s_e[t][p];
        }
        double* rec = A.rec + (size_t)(e0 + t) * A.rstride;
        rec[3 * NB] = M;
        rec[3 * NB + 1] = En;
        rec[3 * NB + 2] = s_mean[t];
    }
    // the advect kernel's flag slots; several blocks may share one
    if (t == 0 && s_flag) atomicOr(&A.flag_part[blockIdx.x % A.nblk], s_flag);
}

template <int N>
int tgt_n(const Step2DArgs& A, hipStream_t s)
{
    // mass and energy rows are taken up to 16 nodes per direction (the
    // constrain kernel's one lane per node)
    if constexpr (N * N > kBlock2) {
        return 1;
    } else {
        constexpr int EB = kBlock2 / (4 * N);
        launch_timed(k_targets2d<N>, dim3((A.K + EB - 1) / EB), dim3(kBlock2), 0, s, A);
        return hipGetLastError() == hipSuccess ? 0 : 1;
    }
}

template <int N>
int facevel_mixed_n(int K_b, int bucket, int kx, int ky, const int32_t* elems, const int32_t* mix,
                    const double* aN_all, const double* tab_all, const double* interp, double vzero, double* vface,
                    hipStream_t s)
{
    const int bs = 256;
    const long tot = (long)K_b * 4 * N;
    hipLaunchKernelGGL(k_facevel2d_mixed<N>, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s, K_b, bucket, kx, ky,
                       elems, mix, aN_all, tab_all, interp, vzero, vface);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int con_mixed_n(const Step2DArgs& A, hipStream_t s)
{
    if (A.nblk < 1) return 1;
    const int nchunk = (A.K + ConShape<N>::E - 1) / ConShape<N>::E;
    static std::atomic<int> cap[kMaxDevices];
    const int r = resident_blocks(k_constrain2d_mixed<N>, cap);
    launch_timed(k_constrain2d_mixed<N>, dim3(con_grid(nchunk, r, A.nblk)), dim3(kBlock2), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace
}  // namespace sl

// the per-order launch table of one order N (defined in one sl2d_p*.hip)
#define SL2D_DEFINE_OPS(N)                                                                                  \
    namespace sl {                                                                                          \
    const Ops2D* ops2d_##N()                                                                                \
    {                                                                                                       \
        static const Ops2D t = {prep_n<N>, facevel_n<N>, facevel_mixed_n<N>, con_mixed_n<N>, adv_n<N>,      \
                                con_n<N>,  bt_n<N>,      tgt_n<N>,           adv_batch_n<N>, con_batch_n<N>}; \
        return &t;                                                                                          \
    }                                                                                                       \
    }
