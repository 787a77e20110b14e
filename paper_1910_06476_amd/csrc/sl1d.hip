// 1D explicit semi-Lagrangian step on gfx950 (FP64).
//
// Mapping: one lane per node ("particle"), the n lanes of an element
// adjacent, floor(256/n) elements packed into a 256-lane block, so loads and
// stores of the element-major fields are contiguous per block.  Element
// interpolants off the nodes are evaluated by Clenshaw recurrences on
// Chebyshev coefficients held in registers; the moved-point interpolant is
// evaluated in the division-free product (first barycentric) form.
//
// Two kernels per step:
//   advect    seed at the nodes (section 4.1), RK move (section 4.2, eq.
//             4.4a / 4.8), remap to the fixed nodes (eq. 4.9), own edge
//             traces (eq. remap_bnd), and the element-local parts of the mass
//             and energy targets (eq. quad, eq. remap_mass, eq.
//             remap_energy): M^n, E^n, the volume term, and the edge values
//             at the RK abscissae by backtracking (eq. 4.11).
//   constrain upwind face values (eq. 4.12a), the face fluxes of the
//             targets, and the constrained least squares (eq. matrix_a) as
//             a small Gram/Schur system per element, with the energy row
//             linearised by Picard iteration.
#include "sl_internal.h"

namespace sl {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool outside(double s) { return s < -1e-10 || s > 1.0 + 1e-10; }

template <int N>
__device__ __forceinline__ double clenshaw(const double (&c)[N], double x)
{
    double b1 = 0.0, b2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = N - 1; k >= 1; --k) {
        double b0 = fma(x2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(x, b1, c[0] - b2);
}

// One explicit RK step of length h for (s, q): ds/dt = dir * u(s) / dx and,
// in the conservative form, dq/dt = -div(s) q.  When have_first is set the
// first stage uses the given (nodal) values instead of an evaluation.
template <int N, bool CONS>
__device__ __forceinline__ void rk_move(const RKTab& T, const double (&ca)[N], const double (&cd)[N], double dir,
                                        double h, double invdx, double& s, double& q, bool& out, bool have_first,
                                        double u_first, double dv_first)
{
    double ks[4], kq[4];
    const double s0 = s, q0 = q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        ks[st] = 0.0;
        kq[st] = 0.0;
        if (st < T.s) {
            double ss = s0, qq = q0;
#pragma unroll
            for (int j = 0; j < st; ++j) {
                ss += h * T.a[st][j] * ks[j];
                if (CONS) qq += h * T.a[st][j] * kq[j];
            }
            double u, dv = 0.0;
            if (st == 0 && have_first) {
                u = u_first;
                dv = dv_first;
            } else {
                const double x = 2.0 * ss - 1.0;
                u = clenshaw<N>(ca, x);
                if (CONS) dv = clenshaw<N>(cd, x);
                out |= outside(ss);
            }
            ks[st] = dir * u * invdx;
            if (CONS) kq[st] = -dv * qq;
        }
    }
    double ds = 0.0, dq = 0.0;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        if (st < T.s) {
            ds += T.b[st] * ks[st];
            if (CONS) dq += T.b[st] * kq[st];
        }
    }
    s = s0 + h * ds;
    if (CONS) q = q0 + h * dq;
    out |= outside(s);
}

__device__ __forceinline__ double upwind(double vn, double lo, double hi)
{
    if (vn > 0.0) return lo;
    if (vn < 0.0) return hi;
    return 0.5 * (lo + hi);
}

// table layout of a 1D mesh: xi, w, l0, l1, Tinv (n x n), D (n x n)
template <int N> struct Off {
    static constexpr int XI = 0, W = N, L0 = 2 * N, L1 = 3 * N, TINV = 4 * N, DM = 4 * N + N * N;
};

// ---------------------------------------------------------------------------
// velocity preparation: Chebyshev coefficients, divergence, face velocities
// ---------------------------------------------------------------------------
template <int N>
__global__ void k_prep1d(int K, int periodic, int has_div, const double* __restrict__ aN, double* __restrict__ aM,
                         double* __restrict__ divN, double* __restrict__ divM, double* __restrict__ vface,
                         const double* __restrict__ tab, double invdx)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    using O = Off<N>;
    double a[N], dv[N];
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] = aN[(size_t)e * N + j];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) c = fma(tab[O::TINV + k * N + j], a[j], c);
        aM[(size_t)e * N + k] = c;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (!has_div) {
            double d = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) d = fma(tab[O::DM + i * N + j], a[j], d);
            dv[i] = d * invdx;
            divN[(size_t)e * N + i] = dv[i];
        } else {
            dv[i] = divN[(size_t)e * N + i];
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) c = fma(tab[O::TINV + k * N + j], dv[j], c);
        divM[(size_t)e * N + k] = c;
    }
    // face e sits between elements e-1 and e: mean of both sides' values
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) mine = fma(tab[O::L0 + j], a[j], mine);
    int em = e - 1;
    if (em < 0) em = periodic ? K - 1 : -1;
    if (em >= 0) {
        double other = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) other = fma(tab[O::L1 + j], aN[(size_t)em * N + j], other);
        vface[e] = 0.5 * (mine + other);
    } else {
        vface[e] = mine;
    }
    if (e == K - 1 && !periodic) {
        double r = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) r = fma(tab[O::L1 + j], a[j], r);
        vface[K] = r;
    }
}

// ---------------------------------------------------------------------------
// advect + remap + element-local target parts
// ---------------------------------------------------------------------------
template <int N, bool CONS>
__global__ __launch_bounds__(kBlock) void k_advect1d(Step1DArgs A)
{
    constexpr int E = kBlock / N;
    using O = Off<N>;
    __shared__ double s_a[E][N];
    __shared__ double s_d[E][N];
    __shared__ double s_p[E][N];
    __shared__ double s_q[E][N];
    __shared__ double s_x[E][N];
    __shared__ double s_c[E][N];
    __shared__ double s_r[4][E][N];
    __shared__ int s_flag;

    const int t = threadIdx.x;
    const int slot = t / N, i = t - slot * N;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const int e = blockIdx.x * E + slot;
    const bool live = inblk && e < A.K;
    const double* __restrict__ tab = A.tab;
    const size_t g = (size_t)(live ? e : 0) * N + i;
    if (t == 0) s_flag = 0;

    const double xi_i = tab[O::XI + i];
    const double W_i = A.dx * tab[O::W + i];
    double phi_i = 0.0, a_i = 0.0, dv_i = 0.0;
    if (live) {
        phi_i = A.phi[g];
        a_i = A.aN[g];
        if (A.targets || CONS) dv_i = A.divN[g];
    }
    if (inblk) {
        s_a[slot][i] = live ? A.aM[g] : 0.0;
        if (CONS) s_d[slot][i] = live ? A.divM[g] : 0.0;
        s_p[slot][i] = phi_i;
    }
    __syncthreads();
    if (A.targets && inblk) {
        double c = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) c = fma(tab[O::TINV + i * N + j], s_p[slot][j], c);
        s_q[slot][i] = c;
    }
    __syncthreads();

    double ca[N], cd[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ca[k] = s_a[sl][k];
        cd[k] = CONS ? s_d[sl][k] : 0.0;
    }
    bool out = false;
    // forward motion of particle i (section 4.2)
    double s = xi_i, q = phi_i;
    rk_move<N, CONS>(A.rk, ca, cd, 1.0, A.dt, 1.0 / A.dx, s, q, out, true, a_i, dv_i);

    // element-local target parts (needs phi^n coefficients)
    double m0 = 0.0, e0 = 0.0, vM = 0.0, vE = 0.0, FM = 0.0, FE = 0.0;
    if (A.targets) {
        double cp[N];
#pragma unroll
        for (int k = 0; k < N; ++k) cp[k] = s_q[sl][k];
        m0 = W_i * phi_i;
        e0 = W_i * phi_i * phi_i;
        if (A.vol) {
            for (int qd = 0; qd < A.rk.nq; ++qd) {
                const double cq = A.rk.cu[qd];
                double val = phi_i;
                if (cq != 0.0) {
                    double sb = xi_i, hq = 1.0;
                    rk_move<N, CONS>(A.rk, ca, cd, -1.0, cq * A.dt, 1.0 / A.dx, sb, hq, out, true, a_i, dv_i);
                    val = hq * clenshaw<N>(cp, 2.0 * sb - 1.0);
                }
                vM += A.rk.bu[qd] * (W_i * dv_i * val);
                vE += A.rk.bu[qd] * (W_i * dv_i * val * val);
            }
        }
        // edge values are needed only where this element is the upwind side
        // of the face (or the face is a stagnation point)
        bool need_edge = false;
        if (live && i == 0) {
            double vL = A.vface[e];
            need_edge = !(vL > A.vzero);
        } else if (live && i == N - 1) {
            double vR = A.vface[(A.periodic && e == A.K - 1) ? 0 : e + 1];
            need_edge = !(vR < -A.vzero);
        }
        if (need_edge) {
            const double xb = (i == 0) ? 0.0 : 1.0;
            for (int qd = 0; qd < A.rk.nq; ++qd) {
                const double cq = A.rk.cu[qd];
                double val;
                if (cq == 0.0) {
                    val = clenshaw<N>(cp, 2.0 * xb - 1.0);
                } else {
                    double sb = xb, hq = 1.0;
                    rk_move<N, CONS>(A.rk, ca, cd, -1.0, cq * A.dt, 1.0 / A.dx, sb, hq, out, false, 0.0, 0.0);
                    val = hq * clenshaw<N>(cp, 2.0 * sb - 1.0);
                }
                FM += A.rk.bu[qd] * val;
                FE += A.rk.bu[qd] * val * val;
            }
        }
        if (inblk) {
            s_r[0][slot][i] = m0;
            s_r[1][slot][i] = e0;
            s_r[2][slot][i] = vM;
            s_r[3][slot][i] = vE;
        }
    }

    // remap (eq. 4.9): phihat_i = sum_j c_j prod_{m != j} (xi_i - s_m),
    // c_j = phi*_j / prod_{m != j} (s_j - s_m)
    if (inblk) s_x[slot][i] = s;
    __syncthreads();
    double xs[N];
#pragma unroll
    for (int m = 0; m < N; ++m) xs[m] = s_x[sl][m];
    double pr = 1.0;
#pragma unroll
    for (int m = 0; m < N; ++m)
        if (m != i) pr *= (s - xs[m]);
    if (inblk) s_c[slot][i] = q / pr;
    __syncthreads();
    double cw[N];
#pragma unroll
    for (int m = 0; m < N; ++m) cw[m] = s_c[sl][m];
    double S = 0.0, P = 1.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double d = xi_i - xs[j];
        S = fma(S, d, cw[j] * P);
        P *= d;
    }
    const double phat = S;
    double tr = 0.0;
    if (i == 0 || i == N - 1) {
        const double xb = (i == 0) ? 0.0 : 1.0;
        double S2 = 0.0, P2 = 1.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const double d = xb - xs[j];
            S2 = fma(S2, d, cw[j] * P2);
            P2 *= d;
        }
        tr = S2;
    }

    int fl = 0;
    if (live) {
        if (out) fl |= FLAG_CONTAIN;
        if (!isfinite(phat)) fl |= FLAG_SINGULAR;
        A.phihat[g] = phat;
        double* r = A.rec + (size_t)e * 8;
        if (i == 0) {
            r[0] = tr;
            r[2] = FM;
            r[4] = FE;
        }
        if (i == N - 1) {
            r[1] = tr;
            r[3] = FM;
            r[5] = FE;
        }
    }
    if (A.targets) {
        // s_r was written before the barriers above
        if (live && i == 0) {
            double M = 0.0, En = 0.0, sM = 0.0, sE = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                M += s_r[0][slot][j];
                En += s_r[1][slot][j];
                sM += s_r[2][slot][j];
                sE += s_r[3][slot][j];
            }
            double* r = A.rec + (size_t)e * 8;
            r[6] = CONS ? M : M + A.dt * sM;
            r[7] = CONS ? En - A.dt * sE : En + A.dt * sE;
        }
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0 && s_flag) A.flag_part[blockIdx.x] |= s_flag;
}

// ---------------------------------------------------------------------------
// constrained least squares
// ---------------------------------------------------------------------------
// Cholesky solve of a 4x4 SPD system (upper triangle used)
__device__ __forceinline__ bool chol4(double G[4][4], double b[4])
{
    double L[4][4];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = G[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        ok = ok && (d > 0.0);
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        L[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
            double v = G[j][i];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / ljj;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double v = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i][k] * b[k];
        b[i] = v / L[i][i];
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        double v = b[i];
#pragma unroll
        for (int k = i + 1; k < 4; ++k) v -= L[k][i] * b[k];
        b[i] = v / L[i][i];
    }
    return ok;
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_constrain1d(Step1DArgs A)
{
    constexpr int E = kBlock / N;
    using O = Off<N>;
    __shared__ double s_r[5][E][N];
    __shared__ int s_flag;
    __shared__ unsigned long long s_stat[kStatSlots];

    const int t = threadIdx.x;
    const int slot = t / N, i = t - slot * N;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const int e = blockIdx.x * E + slot;
    const bool live = inblk && e < A.K;
    const int ee = live ? e : 0;
    const double* __restrict__ tab = A.tab;
    const size_t g = (size_t)ee * N + i;
    if (t < kStatSlots) s_stat[t] = 0ull;
    if (t == 0) s_flag = 0;

    const bool bnd = (A.cmask & SL_C_BOUNDARY) != 0;
    const bool mass = (A.cmask & SL_C_MASS) != 0;
    const bool energy = (A.cmask & SL_C_ENERGY) != 0;
    const double W_i = A.dx * tab[O::W + i];
    const double ph = live ? A.phihat[g] : 0.0;

    // neighbours and face values at t^{n+1}
    const int K = A.K;
    int em = ee - 1, ep = ee + 1;
    if (A.periodic) {
        if (em < 0) em = K - 1;
        if (ep >= K) ep = 0;
    } else {
        if (em < 0) em = -1;
        if (ep >= K) ep = -1;
    }
    double vL = A.vface[ee];
    double vR = A.vface[(A.periodic && ee == K - 1) ? 0 : ee + 1];
    if (fabs(vL) <= A.vzero) vL = 0.0;
    if (fabs(vR) <= A.vzero) vR = 0.0;
    const double* R = A.rec;
    const double* Re = R + (size_t)ee * 8;
    const double T1m = em >= 0 ? R[(size_t)em * 8 + 1] : A.gnext[0];
    const double T0p = ep >= 0 ? R[(size_t)ep * 8 + 0] : A.gnext[1];
    const double dB0 = upwind(vL, T1m, Re[0]);
    const double dB1 = upwind(vR, Re[1], T0p);
    double Mt = 0.0, Et = 0.0;
    if (A.targets) {
        double gM0 = 0.0, gE0 = 0.0, gM1 = 0.0, gE1 = 0.0;
        if (!A.periodic) {
            for (int qd = 0; qd < A.rk.nq; ++qd) {
                const double cq = A.rk.cu[qd];
                const double v0 = (1.0 - cq) * A.gnow[0] + cq * A.gnext[0];
                const double v1 = (1.0 - cq) * A.gnow[1] + cq * A.gnext[1];
                gM0 += A.rk.bu[qd] * v0;
                gE0 += A.rk.bu[qd] * v0 * v0;
                gM1 += A.rk.bu[qd] * v1;
                gE1 += A.rk.bu[qd] * v1 * v1;
            }
        }
        const double FMl = upwind(vL, em >= 0 ? R[(size_t)em * 8 + 3] : gM0, Re[2]);
        const double FEl = upwind(vL, em >= 0 ? R[(size_t)em * 8 + 5] : gE0, Re[4]);
        const double FMr = upwind(vR, Re[3], ep >= 0 ? R[(size_t)ep * 8 + 2] : gM1);
        const double FEr = upwind(vR, Re[5], ep >= 0 ? R[(size_t)ep * 8 + 4] : gE1);
        Mt = Re[6] + A.dt * (vL * FMl - vR * FMr);
        Et = Re[7] + A.dt * (vL * FEl - vR * FEr);
    }

    // rows: l(0), l(1), W, W*psi (energy); inactive rows are zero
    const double c0 = bnd ? tab[O::L0 + i] : 0.0;
    const double c1 = bnd ? tab[O::L1 + i] : 0.0;
    const double c2 = mass ? W_i : 0.0;
    double d[4] = {bnd ? dB0 : 0.0, bnd ? dB1 : 0.0, mass ? Mt : 0.0, energy ? Et : 0.0};
    double Gc[3][3] = {{bnd ? A.g00 : 0.0, bnd ? A.g01 : 0.0, (bnd && mass) ? A.g02 : 0.0},
                       {0.0, bnd ? A.g11 : 0.0, (bnd && mass) ? A.g12 : 0.0},
                       {0.0, 0.0, mass ? A.g22 : 0.0}};
    const bool act[4] = {bnd, bnd, mass, false};

    // C phihat for the constant rows
    if (inblk) {
        s_r[0][slot][i] = c0 * ph;
        s_r[1][slot][i] = c1 * ph;
        s_r[2][slot][i] = c2 * ph;
    }
    __syncthreads();
    double Cph[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < N; ++j) {
        Cph[0] += s_r[0][sl][j];
        Cph[1] += s_r[1][sl][j];
        Cph[2] += s_r[2][sl][j];
    }
    __syncthreads();

    bool singular = false;
    // one constrained solve with energy row c3 (inactive if !use_e)
    auto solve = [&](bool use_e, double c3, const double (&red)[5]) -> double {
        double G[4][4];
        G[0][0] = Gc[0][0]; G[0][1] = Gc[0][1]; G[0][2] = Gc[0][2];
        G[1][1] = Gc[1][1]; G[1][2] = Gc[1][2]; G[2][2] = Gc[2][2];
        G[0][3] = use_e ? red[0] : 0.0;
        G[1][3] = use_e ? red[1] : 0.0;
        G[2][3] = use_e ? red[2] : 0.0;
        G[3][3] = use_e ? red[3] : 0.0;
        const double cph3 = use_e ? red[4] : 0.0;
        const double dd[4] = {d[0], d[1], d[2], use_e ? d[3] : 0.0};
        const bool ac[4] = {act[0], act[1], act[2], use_e};
        double rhs[4];
        const double cp[4] = {Cph[0], Cph[1], Cph[2], cph3};
        if (A.mode == SL_MODE_HARD) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                rhs[a] = cp[a] - dd[a];
                if (!ac[a]) G[a][a] = 1.0;
            }
        } else {
            // (I + G) z = C phihat + G d ; y = z - d
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double s = cp[a];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double gab = (a <= b) ? G[a][b] : G[b][a];
                    s += gab * dd[b];
                }
                rhs[a] = s;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) G[a][a] += 1.0;
        }
        singular |= !chol4(G, rhs);
        double y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) y[a] = (A.mode == SL_MODE_HARD) ? rhs[a] : rhs[a] - dd[a];
        return ph - (c0 * y[0] + c1 * y[1] + c2 * y[2] + (use_e ? c3 * y[3] : 0.0));
    };

    const double zero5[5] = {0, 0, 0, 0, 0};
    double phi = solve(false, 0.0, zero5);
    int iters = 0;
    bool done = !(energy && live);
    bool conv = false;
    if (energy) {
        const bool center = (A.mode == SL_MODE_HARD) && mass;
        double older = phi;
        const double Et0 = d[3];
        for (int k = 1; k <= A.emaxit; ++k) {
            if (__syncthreads_and(done)) break;
            double c3 = W_i * phi;
            if (center) {
                // energy row orthogonal to the mass row (same constraint set)
                if (inblk) s_r[0][slot][i] = c3 * c2;
                __syncthreads();
                double gw = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) gw += s_r[0][sl][j];
                __syncthreads();
                const double mu = gw / A.g22;
                c3 -= mu * c2;
                d[3] = Et0 - mu * Mt;
            }
            if (inblk) {
                s_r[0][slot][i] = c3 * c0;
                s_r[1][slot][i] = c3 * c1;
                s_r[2][slot][i] = c3 * c2;
                s_r[3][slot][i] = c3 * c3;
                s_r[4][slot][i] = c3 * ph;
            }
            __syncthreads();
            double red[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < N; ++j) {
#pragma unroll
                for (int r = 0; r < 5; ++r) red[r] += s_r[r][sl][j];
            }
            __syncthreads();
            const double nphi = solve(true, c3, red);
            if (inblk) {
                s_r[0][slot][i] = fabs(nphi - phi);
                s_r[1][slot][i] = fabs(nphi - older);
            }
            __syncthreads();
            double diff = 0.0, back = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                diff = fmax(diff, s_r[0][sl][j]);
                back = fmax(back, s_r[1][sl][j]);
            }
            __syncthreads();
            if (!done) {
                older = phi;
                phi = nphi;
                iters = k;
                if (diff < A.etol) {
                    done = true;
                    conv = true;
                } else if (k >= 2 && back < A.etol) {
                    done = true;  // 2-cycle: further sweeps repeat
                }
            }
        }
    }

    // residuals of the rows actually imposed
    if (inblk) {
        s_r[0][slot][i] = tab[O::L0 + i] * phi;
        s_r[1][slot][i] = tab[O::L1 + i] * phi;
        s_r[2][slot][i] = W_i * phi;
        s_r[3][slot][i] = W_i * phi * phi;
    }
    __syncthreads();
    int fl = 0;
    if (live) {
        double r0 = 0, r1 = 0, r2 = 0, r3 = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            r0 += s_r[0][slot][j];
            r1 += s_r[1][slot][j];
            r2 += s_r[2][slot][j];
            r3 += s_r[3][slot][j];
        }
        if (i == 0) {
            const double rb = bnd ? fmax(fabs(r0 - dB0), fabs(r1 - dB1)) : 0.0;
            const double rm = mass ? fabs(r2 - Mt) : 0.0;
            const double re = energy ? fabs(r3 - Et) : 0.0;
            atomicMax(&s_stat[0], (unsigned long long)__double_as_longlong(rb));
            atomicMax(&s_stat[1], (unsigned long long)__double_as_longlong(rm));
            atomicMax(&s_stat[2], (unsigned long long)__double_as_longlong(re));
            atomicMax(&s_stat[3], (unsigned long long)iters);
            if (energy && !conv && A.etol > 0.0) fl |= FLAG_NOCONV;
        }
        if (singular) fl |= FLAG_SINGULAR;
        if (!isfinite(phi)) fl |= FLAG_NONFINITE;
        A.phi_out[g] = phi;
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0) {
        if (s_flag) A.flag_part[gridDim.x + blockIdx.x] |= s_flag;
        double* sp = A.stat_part + (size_t)blockIdx.x * kStatSlots;
#pragma unroll
        for (int k = 0; k < 3; ++k) sp[k] = fmax(sp[k], __longlong_as_double((long long)s_stat[k]));
        sp[3] = fmax(sp[3], (double)s_stat[3]);
    }
}

template <int N>
int launch_prep_n(int K, int periodic, int has_div, const double* aN, double* aM, double* divN, double* divM,
                  double* vface, const double* tab, double dx, hipStream_t s)
{
    const int bs = 128;
    hipLaunchKernelGGL(k_prep1d<N>, dim3((K + bs - 1) / bs), dim3(bs), 0, s, K, periodic, has_div, aN, aM, divN,
                       divM, vface, tab, 1.0 / dx);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int launch_adv_n(const Step1DArgs& A, hipStream_t s)
{
    constexpr int E = kBlock / N;
    dim3 grid((A.K + E - 1) / E);
    if (A.cons) hipLaunchKernelGGL((k_advect1d<N, true>), grid, dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL((k_advect1d<N, false>), grid, dim3(kBlock), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int launch_con_n(const Step1DArgs& A, hipStream_t s)
{
    constexpr int E = kBlock / N;
    dim3 grid((A.K + E - 1) / E);
    hipLaunchKernelGGL(k_constrain1d<N>, grid, dim3(kBlock), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

#define SL_DISPATCH_1D(n, CALL)                                                                                 \
    switch (n) {                                                                                                \
    case 2: return CALL<2>; case 3: return CALL<3>; case 4: return CALL<4>; case 5: return CALL<5>;             \
    case 6: return CALL<6>; case 7: return CALL<7>; case 8: return CALL<8>; case 9: return CALL<9>;             \
    case 10: return CALL<10>; case 11: return CALL<11>; case 12: return CALL<12>; case 13: return CALL<13>;     \
    case 14: return CALL<14>; case 15: return CALL<15>; case 16: return CALL<16>; case 17: return CALL<17>;     \
    default: return 1;                                                                                          \
    }

}  // namespace

int blocks1d(int n, int K)
{
    if (n < 2 || n > kMax1D) return 0;
    const int E = kBlock / n;
    return (K + E - 1) / E;
}

#define PREP_CALL(N) launch_prep_n<N>(K, periodic, has_div, aN, aM, divN, divM, vface, tab, dx, s)
int launch_prep1d(int n, int K, int periodic, int has_div, const double* aN, double* aM, double* divN,
                  double* divM, double* vface, const double* tab, double dx, hipStream_t s)
{
    switch (n) {
    case 2: return PREP_CALL(2); case 3: return PREP_CALL(3); case 4: return PREP_CALL(4);
    case 5: return PREP_CALL(5); case 6: return PREP_CALL(6); case 7: return PREP_CALL(7);
    case 8: return PREP_CALL(8); case 9: return PREP_CALL(9); case 10: return PREP_CALL(10);
    case 11: return PREP_CALL(11); case 12: return PREP_CALL(12); case 13: return PREP_CALL(13);
    case 14: return PREP_CALL(14); case 15: return PREP_CALL(15); case 16: return PREP_CALL(16);
    case 17: return PREP_CALL(17);
    default: return 1;
    }
}
#undef PREP_CALL

int launch_advect1d(int n, const Step1DArgs& A, hipStream_t s)
{
    switch (n) {
    case 2: return launch_adv_n<2>(A, s); case 3: return launch_adv_n<3>(A, s);
    case 4: return launch_adv_n<4>(A, s); case 5: return launch_adv_n<5>(A, s);
    case 6: return launch_adv_n<6>(A, s); case 7: return launch_adv_n<7>(A, s);
    case 8: return launch_adv_n<8>(A, s); case 9: return launch_adv_n<9>(A, s);
    case 10: return launch_adv_n<10>(A, s); case 11: return launch_adv_n<11>(A, s);
    case 12: return launch_adv_n<12>(A, s); case 13: return launch_adv_n<13>(A, s);
    case 14: return launch_adv_n<14>(A, s); case 15: return launch_adv_n<15>(A, s);
    case 16: return launch_adv_n<16>(A, s); case 17: return launch_adv_n<17>(A, s);
    default: return 1;
    }
}

int launch_constrain1d(int n, const Step1DArgs& A, hipStream_t s)
{
    switch (n) {
    case 2: return launch_con_n<2>(A, s); case 3: return launch_con_n<3>(A, s);
    case 4: return launch_con_n<4>(A, s); case 5: return launch_con_n<5>(A, s);
    case 6: return launch_con_n<6>(A, s); case 7: return launch_con_n<7>(A, s);
    case 8: return launch_con_n<8>(A, s); case 9: return launch_con_n<9>(A, s);
    case 10: return launch_con_n<10>(A, s); case 11: return launch_con_n<11>(A, s);
    case 12: return launch_con_n<12>(A, s); case 13: return launch_con_n<13>(A, s);
    case 14: return launch_con_n<14>(A, s); case 15: return launch_con_n<15>(A, s);
    case 16: return launch_con_n<16>(A, s); case 17: return launch_con_n<17>(A, s);
    default: return 1;
    }
}

}  // namespace sl
