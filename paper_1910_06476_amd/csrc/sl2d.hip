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
// rows through C_B^+ (HARD) or (I + C_B^T C_B)^{-1} (SOFT).
#include <type_traits>

#include "sl_internal.h"

namespace sl {
namespace {

constexpr int kBlock2 = 256;

__device__ __forceinline__ bool outside2(double s) { return s < -1e-10 || s > 1.0 + 1e-10; }

// table layout of a 2D mesh
template <int N> struct Off2 {
    static constexpr int ND = N * N;
    static constexpr int XI = 0, W = N, L0 = 2 * N, L1 = 3 * N, TINV = 4 * N, DM = 4 * N + ND, LAM = 4 * N + 2 * ND,
                         QH = 5 * N + 2 * ND, QS = QH + 16 * ND;
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

// ---------------------------------------------------------------------------
// velocity preparation: tensor Chebyshev coefficients, divergence, own edge
// normal speeds, effective degree
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_prep2d(int K, int has_div, int cons, const double* __restrict__ aN, double* __restrict__ aM,
                         double* __restrict__ divN, double* __restrict__ divM, double* __restrict__ vedge,
                         const double* __restrict__ tab, double invdx, double invdy, double vscale,
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
    // own edge normal speeds: left (xi=0, eta_j), right, bottom (xi_i, eta=0), top
    double* ve = vedge + (size_t)e * 4 * N;
    for (int k = 0; k < N; ++k) {
        double l0 = 0.0, r0 = 0.0, b0 = 0.0, t0 = 0.0;
        for (int q = 0; q < N; ++q) {
            l0 = fma(tab[O::L0 + q], U[q + N * k], l0);
            r0 = fma(tab[O::L1 + q], U[q + N * k], r0);
            b0 = fma(tab[O::L0 + q], V[k + N * q], b0);
            t0 = fma(tab[O::L1 + q], V[k + N * q], t0);
        }
        ve[k] = l0;
        ve[N + k] = r0;
        ve[2 * N + k] = b0;
        ve[3 * N + k] = t0;
    }
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
// advect + remap (eq. 5.4 by defect correction) + edge traces
//
// PPL particles per lane for n >= 5 (one by default: more cut the LDS reads
// of the iterate in V x but the register growth costs more occupancy than
// the reads save, measured at n = 9).  With P32 the separable
// preconditioner is stored and applied in FP32 while the residual and the
// iterate stay FP64 (iterative refinement).
// ---------------------------------------------------------------------------
#ifndef SL2D_PPL
#define SL2D_PPL 1  // particles per lane of the 2D advect kernel for n >= 5
#endif
template <int N> struct Lanes2 {
    static constexpr int ND = N * N;
    static constexpr int PPL = N >= 5 ? SL2D_PPL : 1;
    static constexpr int L = (ND + PPL - 1) / PPL;  // lanes per element
    static constexpr int E = kBlock2 / L;           // elements per block
};

template <int N, bool P32>
__global__ __launch_bounds__(kBlock2) void k_advect2d(Step2DArgs A)
{
    using O = Off2<N>;
    using G = Lanes2<N>;
    using PT = typename std::conditional<P32, float, double>::type;
    constexpr int ND = G::ND, PPL = G::PPL, L = G::L, E = G::E;
    __shared__ double s_cu[E][ND], s_cv[E][ND], s_cd[E][ND];
    __shared__ double s_x[E][ND], s_r[E][ND], s_f[E][ND];
    __shared__ PT s_z[E][ND];
    __shared__ PT s_ai[E][ND], s_bi[E][ND];
    __shared__ double s_mx[E][N], s_my[E][N];
    __shared__ unsigned long long s_nrm[2][E];  // max |y| per element, double-buffered by sweep parity
    __shared__ int s_flag, s_sw_sum, s_sw_max;
    __shared__ unsigned long long s_res;
    __shared__ unsigned long long s_ref[E];  // max |phi*| per element (FP32 scaling)

    const int t = threadIdx.x;
    const int slot = t / L, q = t - slot * L;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const int e = blockIdx.x * E + slot;
    const bool live = inblk && e < A.K;
    const double* __restrict__ tab = A.tab;
    const int K = A.K;
    if (t == 0) {
        s_flag = 0;
        s_sw_sum = 0;
        s_sw_max = 0;
        s_res = 0ull;
    }
    if (t < E * 2) s_nrm[t / E][t % E] = 0ull;
    if (t < E) s_ref[t] = 0ull;

    // items of this lane: particle / node indices q, q + L, q + 2L (< n^2)
    int idx[PPL];
    bool has[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        idx[r] = q + r * L;
        has[r] = inblk && idx[r] < ND;
    }
    double phi_p[PPL], u_p[PPL], v_p[PPL], dv_p[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        phi_p[r] = u_p[r] = v_p[r] = dv_p[r] = 0.0;
        const size_t g = (size_t)(live ? e : 0) * ND + (has[r] ? idx[r] : 0);
        if (live && has[r]) {
            phi_p[r] = A.phi[g];
            u_p[r] = A.aN[g];
            v_p[r] = A.aN[(size_t)K * ND + g];
            if (A.cons) dv_p[r] = A.divN[g];
        }
        if (has[r]) {
            s_cu[slot][idx[r]] = live ? A.aM[g] : 0.0;
            s_cv[slot][idx[r]] = live ? A.aM[(size_t)K * ND + g] : 0.0;
            if (A.cons) s_cd[slot][idx[r]] = live ? A.divM[g] : 0.0;
        }
    }
    __syncthreads();

    // forward motion of each particle (eq. 5.1 tensor interpolant of the velocity)
    const RKTab& T = A.rk;
    const int d = A.vdeg;
    const double h = A.dt;
    bool out = false;
    double sx[PPL], sy[PPL], sq[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const int ii = idx[r] % N, jj = idx[r] / N;
        double s = tab[O::XI + (has[r] ? ii : 0)], rr0 = tab[O::XI + (has[r] ? jj : 0)], qv = phi_p[r];
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
                    uu = u_p[r];
                    vv = v_p[r];
                    dd = dv_p[r];
                } else {
                    const double x = 2.0 * ss - 1.0, y = 2.0 * rr - 1.0;
                    uu = cheb2<N>(s_cu[sl], x, y, d);
                    vv = cheb2<N>(s_cv[sl], x, y, d);
                    if (A.cons) dd = cheb2<N>(s_cd[sl], x, y, d);
                    out |= has[r] && (outside2(ss) || outside2(rr));
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
        sx[r] = s + h * ds;
        sy[r] = rr0 + h * dr;
        sq[r] = qv + h * dq;
        out |= has[r] && (outside2(sx[r]) || outside2(sy[r]));
    }

    // rows of V: a_l = l_l(xi*_p), b_m = l_m(eta*_p) (eq. 5.4), product form
    double a[PPL][N], b[PPL][N];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        double pa[N], pb[N];
        double acc_a = 1.0, acc_b = 1.0;
#pragma unroll
        for (int l = 0; l < N; ++l) {
            pa[l] = acc_a;
            pb[l] = acc_b;
            acc_a *= (sx[r] - tab[O::XI + l]);
            acc_b *= (sy[r] - tab[O::XI + l]);
        }
        acc_a = 1.0;
        acc_b = 1.0;
#pragma unroll
        for (int l = N - 1; l >= 0; --l) {
            a[r][l] = tab[O::LAM + l] * pa[l] * acc_a;
            b[r][l] = tab[O::LAM + l] * pb[l] * acc_b;
            acc_a *= (sx[r] - tab[O::XI + l]);
            acc_b *= (sy[r] - tab[O::XI + l]);
        }
    }

    // separable preconditioner: mean displacement of each x-column i and of
    // each y-row j of particles
#pragma unroll
    for (int r = 0; r < PPL; ++r)
        if (has[r]) {
            const int ii = idx[r] % N, jj = idx[r] / N;
            s_r[slot][idx[r]] = sx[r] - tab[O::XI + ii];
            s_x[slot][idx[r]] = sy[r] - tab[O::XI + jj];
            s_f[slot][idx[r]] = sq[r];  // phi*
            atomicMax(&s_ref[slot], (unsigned long long)__double_as_longlong(fabs(sq[r])));
        }
    __syncthreads();
    for (int c = q; inblk && c < 2 * N; c += L) {
        double m = 0.0;
        if (c < N) {
            for (int jj = 0; jj < N; ++jj) m += s_r[slot][c + N * jj];
            s_mx[slot][c] = m / N;
        } else {
            for (int ii = 0; ii < N; ++ii) m += s_x[slot][ii + N * (c - N)];
            s_my[slot][c - N] = m / N;
        }
    }
    __syncthreads();
    // A0^{-1}[l][c]: interpolation from the shifted nodes xi_k + mx_k back to
    // node xi_l, prod_{k != c} (xi_l - s_k) / prod_{k != c} (s_c - s_k)
#pragma unroll
    for (int r = 0; r < PPL; ++r)
        if (has[r]) {
            const int l = idx[r] % N, c = idx[r] / N;
            const double xl = tab[O::XI + l];
            const double sc = tab[O::XI + c] + s_mx[slot][c], tc = tab[O::XI + c] + s_my[slot][c];
            double na = 1.0, da = 1.0, nb = 1.0, db = 1.0;
            for (int k = 0; k < N; ++k) {
                if (k == c) continue;
                const double sk = tab[O::XI + k] + s_mx[slot][k];
                const double tk = tab[O::XI + k] + s_my[slot][k];
                na *= (xl - sk);
                da *= (sc - sk);
                nb *= (xl - tk);
                db *= (tc - tk);
            }
            s_ai[slot][idx[r]] = (PT)(na / da);
            s_bi[slot][idx[r]] = (PT)(nb / db);
        }
    __syncthreads();

    // y = M^{-1} f (f in s_f or s_r, node c + N jj), per item:
    //   stage 1: z[jj][l] = sum_c Ai[l][c] f[jj][c]
    //   stage 2: y[m][l] = sum_jj Bi[m][jj] z[jj][l]
    // In FP32 the operand is first scaled by 2^-e, e = exponent of a
    // reference magnitude of it (max |phi*| of the element, then the last
    // correction), so that it sits near 1 and never in the FP32 subnormal
    // range; M^{-1} is linear, so the result is scaled back exactly.
    auto precond = [&](double (*src)[ND], double (&yy)[PPL], int e2) {
        const double sc = P32 ? ldexp(1.0, -e2) : 1.0;
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (has[r]) {
                const int l = idx[r] % N, jj = idx[r] / N;
                PT zz = 0;
                for (int c = 0; c < N; ++c) {
                    const double v = src[slot][c + N * jj];
                    zz = fma(s_ai[slot][l + N * c], (PT)(P32 ? v * sc : v), zz);
                }
                s_z[slot][idx[r]] = zz;
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            PT acc = 0;
            if (has[r]) {
                const int l = idx[r] % N, m = idx[r] / N;
                for (int jj = 0; jj < N; ++jj) acc = fma(s_bi[slot][m + N * jj], s_z[slot][l + N * jj], acc);
            }
            yy[r] = P32 ? ldexp((double)acc, e2) : (double)acc;
        }
    };
    // exponent of a reference magnitude, clamped so 2^-e stays finite
    auto ref_exp = [](double ref) { return ref > 0.0 ? max(ilogb(ref), -1000) : 0; };

    double x[PPL], y[PPL];
    const double ref = __longlong_as_double((long long)s_ref[sl]);  // max |phi*| of the element
    int e2 = 0;
    if (P32) e2 = ref_exp(ref);
    precond(s_f, x, e2);
#pragma unroll
    for (int r = 0; r < PPL; ++r)
        if (has[r]) s_x[slot][idx[r]] = x[r];
    __syncthreads();
    bool conv = !live;
    int sweeps = A.refine;   // sweeps this element needed
    double lastrel = 0.0;    // its estimated error left, relative to max |phi*|
    double prev = 0.0;       // max |y| of the previous sweep
    for (int it = 0; it < A.refine; ++it) {
        // residual r_p = phi*_p - (V x)_p, (V x)_p = sum_m b_m sum_l a_l x[m][l]
        double vx[PPL];
#pragma unroll
        for (int r = 0; r < PPL; ++r) vx[r] = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            double inner[PPL];
#pragma unroll
            for (int r = 0; r < PPL; ++r) inner[r] = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                const double xml = s_x[sl][l + N * m];
#pragma unroll
                for (int r = 0; r < PPL; ++r) inner[r] = fma(a[r][l], xml, inner[r]);
            }
#pragma unroll
            for (int r = 0; r < PPL; ++r) vx[r] = fma(b[r][m], inner[r], vx[r]);
        }
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (has[r]) s_r[slot][idx[r]] = sq[r] - vx[r];
        __syncthreads();  // s_x is no longer read in this sweep
        // clear the other parity's slot, last read before this sweep's first barrier
        if (t < E) s_nrm[(it + 1) & 1][t] = 0ull;
        precond(s_r, y, e2);
        double ny = 0.0;
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (has[r]) {
                if (!conv) x[r] += y[r];
                ny = fmax(ny, fabs(y[r]));
                s_x[slot][idx[r]] = x[r];
            }
        if (inblk) atomicMax(&s_nrm[it & 1][slot], (unsigned long long)__double_as_longlong(ny));
        __syncthreads();
        if (inblk) {
            const double eny = __longlong_as_double((long long)s_nrm[it & 1][slot]);
            if (P32 && eny > 0.0) e2 = ref_exp(eny);
            if (!conv) {
                // estimated error left: the correction times the observed contraction
                const double left = (it > 0 && prev > 0.0) ? fmin(eny, eny * eny / prev) : eny;
                lastrel = ref > 0.0 ? left / ref : 0.0;
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
        if (__syncthreads_and(conv)) break;
    }

    // edge traces of the remapped polynomial (eq. 2dx/2dy_bnd_interpolate):
    // t < N left (xi=0, eta_t), < 2N right, < 3N bottom (xi_k, eta=0), top
    int fl = 0;
    if (live) {
        if (out) fl |= FLAG_CONTAIN;
        if (!conv) fl |= FLAG_SINGULAR;
        if (q == 0) {
            atomicAdd(&s_sw_sum, sweeps);
            atomicMax(&s_sw_max, sweeps);
            atomicMax(&s_res, (unsigned long long)__double_as_longlong(lastrel));
        }
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (has[r]) {
                if (!isfinite(x[r])) fl |= FLAG_SINGULAR;
                A.phihat[(size_t)e * ND + idx[r]] = x[r];
            }
        for (int tt = q; tt < 4 * N; tt += L) {
            const int side = tt / N, k = tt % N;
            const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
            double tr = 0.0;
            if (side < 2)
                for (int c = 0; c < N; ++c) tr = fma(lv[c], s_x[slot][c + N * k], tr);
            else
                for (int c = 0; c < N; ++c) tr = fma(lv[c], s_x[slot][k + N * c], tr);
            A.rec[(size_t)e * 4 * N + tt] = tr;
        }
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[blockIdx.x] |= s_flag;
        // one block owns each slot row; launches on the stream are ordered
        double* sp = A.stat_part + (size_t)blockIdx.x * kStatSlots;
        sp[4] += (double)s_sw_sum;
        sp[5] = fmax(sp[5], (double)s_sw_max);
        sp[6] = fmax(sp[6], __longlong_as_double((long long)s_res));
    }
}

// ---------------------------------------------------------------------------
// boundary-constrained least squares (2D)
// ---------------------------------------------------------------------------
// persistent blocks: each loads the 4n x 4n table Q into LDS once and loops
// over chunks of E elements
constexpr int kConGrid = 2048;

template <int N>
__global__ __launch_bounds__(kBlock2) void k_constrain2d(Step2DArgs A)
{
    using O = Off2<N>;
    constexpr int ND = N * N;
    constexpr int E = kBlock2 / ND;
    constexpr int NQ = 16 * N * N;
    __shared__ double s_q[NQ];
    // per element: z, d_B - C_B phihat, d_B, phi
    __shared__ double s_d[E][4 * N], s_rb[E][4 * N], s_fv[E][4 * N], s_y[E][ND];
    __shared__ int s_flag;
    __shared__ unsigned long long s_stat;

    const int t = threadIdx.x;
    const int slot = t / ND, p = t - slot * ND;
    const bool inblk = slot < E;
    const double* __restrict__ tab = A.tab;
    const int kx = A.kx, ky = A.ky, K = A.K;
    const bool bnd = (A.cmask & SL_C_BOUNDARY) != 0;
    const double* Qg = tab + (A.mode == SL_MODE_HARD ? O::QH : O::QS);
    for (int k = t; k < NQ; k += kBlock2) s_q[k] = Qg[k];
    if (t == 0) {
        s_flag = 0;
        s_stat = 0ull;
    }
    const int i = p % N, j = p / N;
    const double l0i = tab[O::L0 + i], l1i = tab[O::L1 + i], l0j = tab[O::L0 + j], l1j = tab[O::L1 + j];
    const int nchunk = (K + E - 1) / E;

    for (int chunk = blockIdx.x; chunk < nchunk; chunk += gridDim.x) {
        const int e = chunk * E + slot;
        const bool live = inblk && e < K;
        const int ee = live ? e : 0;
        const size_t g = (size_t)ee * ND + p;
        const double ph = live ? A.phihat[g] : 0.0;

        // face value at the element's edge point tt: upwind of its own trace
        // and the neighbour's matching trace (eq. 4.12a); ghost values at the
        // domain boundary
        for (int tt = p; inblk && tt < 4 * N; tt += ND) {
            const int side = tt / N, k = tt % N;
            const int ex = ee % kx, ey = ee / kx;
            int nbe = -1, nbt = 0, gidx = 0;
            bool high = false;
            const int KL = ky * N, KB = kx * N;
            switch (side) {
            case 0:
                nbe = ex > 0 ? ee - 1 : (A.periodic ? ey * kx + kx - 1 : -1);
                nbt = N + k; gidx = ey * N + k; high = true;
                break;
            case 1:
                nbe = ex < kx - 1 ? ee + 1 : (A.periodic ? ey * kx : -1);
                nbt = k; gidx = KL + ey * N + k; high = false;
                break;
            case 2:
                nbe = ey > 0 ? ee - kx : (A.periodic ? (ky - 1) * kx + ex : -1);
                nbt = 3 * N + k; gidx = 2 * KL + ex * N + k; high = true;
                break;
            default:
                nbe = ey < ky - 1 ? ee + kx : (A.periodic ? ex : -1);
                nbt = 2 * N + k; gidx = 2 * KL + KB + ex * N + k; high = false;
                break;
            }
            const double mine = A.rec[(size_t)ee * 4 * N + tt];
            const double vmine = A.vedge[(size_t)ee * 4 * N + tt];
            double other, vn;
            if (nbe >= 0) {
                other = A.rec[(size_t)nbe * 4 * N + nbt];
                vn = 0.5 * (vmine + A.vedge[(size_t)nbe * 4 * N + nbt]);
            } else {
                other = A.gnext[gidx];
                vn = vmine;
            }
            if (fabs(vn) <= A.vzero) vn = 0.0;
            const double lo = high ? other : mine, hi = high ? mine : other;
            const double dv = upwind2(vn, lo, hi);
            s_fv[slot][tt] = dv;
            s_rb[slot][tt] = dv - mine;
        }
        __syncthreads();

        // phi = phihat + C_B^T z, z = Q (d_B - C_B phihat), Q = (C_B C_B^T)^+
        // (HARD) or (I + C_B C_B^T)^{-1} (SOFT); lanes t < 4n form z, then
        // every node applies C_B^T (four products)
        double phi = ph;
        if (bnd) {
            for (int tt = p; inblk && tt < 4 * N; tt += ND) {
                double z = 0.0;
                for (int q = 0; q < 4 * N; ++q) z = fma(s_q[tt * 4 * N + q], s_rb[slot][q], z);
                s_d[slot][tt] = z;
            }
            __syncthreads();
            if (inblk)
                phi = ph + l0i * s_d[slot][j] + l1i * s_d[slot][N + j] + l0j * s_d[slot][2 * N + i] +
                      l1j * s_d[slot][3 * N + i];
        }
        if (inblk) s_y[slot][p] = phi;
        __syncthreads();
        int fl = 0;
        if (live) {
            if (!isfinite(phi)) fl |= FLAG_NONFINITE;
            A.phi_out[g] = phi;
            for (int tt = p; bnd && tt < 4 * N; tt += ND) {
                const int side = tt / N, k = tt % N;
                const double* lv = tab + ((side & 1) ? O::L1 : O::L0);
                double tr = 0.0;
                if (side < 2)
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_y[slot][c + N * k], tr);
                else
                    for (int c = 0; c < N; ++c) tr = fma(lv[c], s_y[slot][k + N * c], tr);
                atomicMax(&s_stat, (unsigned long long)__double_as_longlong(fabs(tr - s_fv[slot][tt])));
            }
        }
        if (fl) atomicOr(&s_flag, fl);
        __syncthreads();  // s_fv, s_rb, s_d, s_y are rewritten by the next chunk
    }
    if (t == 0) {
        if (s_flag) A.flag_part[A.nblk + blockIdx.x] |= s_flag;
        double* sp = A.stat_part + (size_t)blockIdx.x * kStatSlots;
        sp[0] = fmax(sp[0], __longlong_as_double((long long)s_stat));
    }
}

template <int N>
int prep_n(int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM, double* vedge,
           const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s)
{
    const int bs = 64;
    hipLaunchKernelGGL(k_prep2d<N>, dim3((K + bs - 1) / bs), dim3(bs), 0, s, K, has_div, cons, aN, aM, divN, divM,
                       vedge, tab, 1.0 / dx, 1.0 / dy, vscale, vdeg);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int adv_n(const Step2DArgs& A, hipStream_t s)
{
    constexpr int E = Lanes2<N>::E;
    const dim3 grid((A.K + E - 1) / E);
    if (A.precision == SL_PREC_FP32_REFINED) hipLaunchKernelGGL((k_advect2d<N, true>), grid, dim3(kBlock2), 0, s, A);
    else hipLaunchKernelGGL((k_advect2d<N, false>), grid, dim3(kBlock2), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int con_n(const Step2DArgs& A, hipStream_t s)
{
    constexpr int E = kBlock2 / (N * N);
    const int nchunk = (A.K + E - 1) / E;
    hipLaunchKernelGGL(k_constrain2d<N>, dim3(nchunk < kConGrid ? nchunk : kConGrid), dim3(kBlock2), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace

int blocks2d(int n, int K)
{
    if (n < 2 || n > kMax2D) return 0;
    const int ppl = n >= 5 ? SL2D_PPL : 1;
    const int Ea = kBlock2 / ((n * n + ppl - 1) / ppl);  // advect elements per block
    const int Ec = kBlock2 / (n * n);                    // constrain elements per block
    const int a = (K + Ea - 1) / Ea, c = (K + Ec - 1) / Ec;
    return a > c ? a : c;
}

#define SL2D_SWITCH(n, CALL)                                                                                   \
    switch (n) {                                                                                               \
    case 2: return CALL(2); case 3: return CALL(3); case 4: return CALL(4); case 5: return CALL(5);            \
    case 6: return CALL(6); case 7: return CALL(7); case 8: return CALL(8); case 9: return CALL(9);            \
    case 10: return CALL(10); case 11: return CALL(11);                                                        \
    default: return 1;                                                                                         \
    }

int launch_prep2d(int n, int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM,
                  double* vedge, const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s)
{
#define PREP2(N) prep_n<N>(K, has_div, cons, aN, aM, divN, divM, vedge, tab, dx, dy, vscale, vdeg, s)
    SL2D_SWITCH(n, PREP2)
#undef PREP2
}

int launch_advect2d(int n, const Step2DArgs& A, hipStream_t s)
{
#define ADV2(N) adv_n<N>(A, s)
    SL2D_SWITCH(n, ADV2)
#undef ADV2
}

int launch_constrain2d(int n, const Step2DArgs& A, hipStream_t s)
{
#define CON2(N) con_n<N>(A, s)
    SL2D_SWITCH(n, CON2)
#undef CON2
}

}  // namespace sl
