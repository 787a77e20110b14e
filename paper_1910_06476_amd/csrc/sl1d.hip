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
#include "sl_batch.h"
#include "sl_internal.h"

namespace sl {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool outside(double s) { return s < -1e-10 || s > 1.0 + 1e-10; }

// sum_{k < M} c_k T_k(x) by Clenshaw's recurrence (the first M of N terms)
template <int N, int M>
__device__ __forceinline__ double clenshaw_n(const double (&c)[N], double x)
{
    static_assert(M >= 1 && M <= N, "term count");
    double b1 = 0.0, b2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = M - 1; k >= 1; --k) {
        double b0 = fma(x2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(x, b1, c[0] - b2);
}

// the same over coefficients in LDS (read as the recurrence needs them)
template <int N>
__device__ __forceinline__ double clenshaw_p(const double* __restrict__ c, double x)
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

// clenshaw_p at P points at once: each coefficient is read once for all of
// them, and the P recurrences are independent (the same operations per
// point as clenshaw_p)
template <int N, int P>
__device__ __forceinline__ void clenshaw_multi(const double* __restrict__ c, const double (&x)[P], double (&v)[P])
{
    double b1[P], b2[P], x2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        b1[p] = b2[p] = 0.0;
        x2[p] = 2.0 * x[p];
    }
#pragma unroll
    for (int k = N - 1; k >= 1; --k) {
        const double ck = c[k];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double b0 = fma(x2[p], b1[p], ck - b2[p]);
            b2[p] = b1[p];
            b1[p] = b0;
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = fma(x[p], b1[p], c[0] - b2[p]);
}

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

// Effective degree of a Chebyshev series: the largest k whose tail
// sum_{j >= k} |c_j| exceeds 2^-46 (1.4e-14) of max(sum_j |c_j|, scale).
// Coefficients obtained from nodal values carry rounding noise of about
// 1e-16 of the nodal magnitudes; a tail below this threshold is that noise,
// and skipping it moves the evaluated series by no more than its own
// rounding error.  `scale` is the mesh-wide magnitude of the field (max
// |a| for the velocity): where the field nearly vanishes in one element,
// its noise is measured against the field, not against the element's own
// tiny coefficients.
template <int N>
__device__ __forceinline__ int cheb_degree(const double (&c)[N], double scale = 0.0)
{
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) tot += fabs(c[k]);
    const double thr = fmax(tot, scale) * 0x1p-46;
    double tail = 0.0;
    int d = 0;
#pragma unroll
    for (int k = N - 1; k >= 1; --k) {
        tail += fabs(c[k]);
        if (d == 0 && tail > thr) d = k;
    }
    return d;
}

// One explicit RK step of length h for (s, q): ds/dt = dir * u(s) / dx and,
// in the conservative form, dq/dt = -div(s) q.  When have_first is set the
// first stage uses the given (nodal) values instead of an evaluation.
// (NA: number of leading Chebyshev coefficients of the velocity and
// divergence series that are evaluated; the rest are negligible, see
// cheb_degree)
// Tableau access: RKS = 0 reads the runtime tableau, RKS = 4 is the
// classical fourth-order tableau at compile time (its zero entries vanish
// from the code; the distinct abscissae are 0, 1/2, 1 with weights
// 1/6, 2/3, 1/6).
template <int RKS> struct Tab {
    const RKTab& T;
    __device__ int s() const { return T.s; }
    __device__ double a(int i, int j) const { return T.a[i][j]; }
    __device__ double b(int i) const { return T.b[i]; }
    __device__ int nq() const { return T.nq; }
    __device__ double cu(int k) const { return T.cu[k]; }
    __device__ double bu(int k) const { return T.bu[k]; }
};
template <> struct Tab<4> {
    const RKTab& T;
    __device__ constexpr int s() const { return 4; }
    __device__ constexpr double a(int i, int j) const
    {
        return (i == 1 && j == 0) || (i == 2 && j == 1) ? 0.5 : (i == 3 && j == 2) ? 1.0 : 0.0;
    }
    __device__ constexpr double b(int i) const { return (i == 0 || i == 3) ? 1.0 / 6 : 1.0 / 3; }
    __device__ constexpr int nq() const { return 3; }
    __device__ constexpr double cu(int k) const { return k == 0 ? 0.0 : k == 1 ? 0.5 : 1.0; }
    __device__ constexpr double bu(int k) const { return k == 1 ? 2.0 / 3 : 1.0 / 6; }
};

template <int N, bool CONS, int NA = N, int RKS = 0>
__device__ __forceinline__ void rk_move(const RKTab& TT, const double (&ca)[N], const double (&cd)[N], double dir,
                                        double h, double invdx, double& s, double& q, bool& out, bool have_first,
                                        double u_first, double dv_first)
{
    const Tab<RKS> T{TT};
    double ks[4], kq[4];
    const double s0 = s, q0 = q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        ks[st] = 0.0;
        kq[st] = 0.0;
        if (st < T.s()) {
            double ss = s0, qq = q0;
#pragma unroll
            for (int j = 0; j < st; ++j) {
                if (T.a(st, j) == 0.0) continue;
                ss += h * T.a(st, j) * ks[j];
                if (CONS) qq += h * T.a(st, j) * kq[j];
            }
            double u, dv = 0.0;
            if (st == 0 && have_first) {
                u = u_first;
                dv = dv_first;
            } else {
                const double x = 2.0 * ss - 1.0;
                u = clenshaw_n<N, NA>(ca, x);
                if (CONS) dv = clenshaw_n<N, NA>(cd, x);
                out |= outside(ss);
            }
            ks[st] = dir * u * invdx;
            if (CONS) kq[st] = -dv * qq;
        }
    }
    double ds = 0.0, dq = 0.0;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        if (st < T.s()) {
            ds += T.b(st) * ks[st];
            if (CONS) dq += T.b(st) * kq[st];
        }
    }
    s = s0 + h * ds;
    if (CONS) q = q0 + h * dq;
    out |= outside(s);
}

// The first NA (<= 4) Chebyshev terms on x = 2s - 1 rewritten as a
// polynomial in s and multiplied by `scale`: T1 = 2s - 1, T2 = 8s^2 - 8s + 1,
// T3 = 32s^3 - 48s^2 + 18s - 1.  Horner's rule on it costs NA - 1 FMAs per
// evaluation against Clenshaw's 2(NA - 1) + 2 operations.  The absolute
// coefficient sums of T1..T3 in s are 3, 17 and 99, which bounds how much the
// rewriting can magnify the rounding of each term.
template <int NA, int N>
__device__ __forceinline__ void cheb_to_mono(const double (&c)[N], double scale, double (&m)[NA])
{
    static_assert(NA >= 1 && NA <= 4 && NA <= N, "term count");
    const double c0 = c[0];
    const double c1 = NA > 1 ? c[NA > 1 ? 1 : 0] : 0.0;
    const double c2 = NA > 2 ? c[NA > 2 ? 2 : 0] : 0.0;
    const double c3 = NA > 3 ? c[NA > 3 ? 3 : 0] : 0.0;
    const double mm[4] = {c0 - c1 + c2 - c3, 2.0 * c1 - 8.0 * c2 + 18.0 * c3, 8.0 * c2 - 48.0 * c3, 32.0 * c3};
#pragma unroll
    for (int k = 0; k < NA; ++k) m[k] = scale * mm[k];
}

template <int NA>
__device__ __forceinline__ double horner(const double (&m)[NA], double s)
{
    double u = m[NA - 1];
#pragma unroll
    for (int k = NA - 2; k >= 0; --k) u = fma(u, s, m[k]);
    return u;
}

// rk_move with the velocity (and divergence) as polynomials in s from
// cheb_to_mono: mu is the velocity over dx, hs = dir * h the signed step of
// the position, h the step of q; k_first = the first stage's mu value
template <bool CONS, int NA, int RKS>
__device__ __forceinline__ void rk_move_mono(const RKTab& TT, const double (&mu)[NA], const double (&md)[NA],
                                             double hs, double h, double& s, double& q, bool& out,
                                             bool have_first, double k_first, double dv_first)
{
    const Tab<RKS> T{TT};
    double ks[4], kq[4];
    const double s0 = s, q0 = q;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        ks[st] = 0.0;
        kq[st] = 0.0;
        if (st < T.s()) {
            double ss = s0, qq = q0;
#pragma unroll
            for (int j = 0; j < st; ++j) {
                if (T.a(st, j) == 0.0) continue;
                ss += hs * T.a(st, j) * ks[j];
                if (CONS) qq += h * T.a(st, j) * kq[j];
            }
            double u, dv = 0.0;
            if (st == 0 && have_first) {
                u = k_first;
                dv = dv_first;
            } else {
                u = horner<NA>(mu, ss);
                if (CONS) dv = horner<NA>(md, ss);
                out |= outside(ss);
            }
            ks[st] = u;
            if (CONS) kq[st] = -dv * qq;
        }
    }
    double ds = 0.0, dq = 0.0;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        if (st < T.s()) {
            ds += T.b(st) * ks[st];
            if (CONS) dq += T.b(st) * kq[st];
        }
    }
    s = s0 + hs * ds;
    if (CONS) q = q0 + h * dq;
    out |= outside(s);
}

// value of a Chebyshev series at x = 1 (edge 1) or x = -1 (edge 0), where
// T_k is 1 or (-1)^k
template <int N>
__device__ __forceinline__ double cheb_end(const double* __restrict__ c, int edge)
{
    double ev = c[0], od = N > 1 ? c[1] : 0.0;
#pragma unroll
    for (int k = 2; k < N; ++k) {
        if (k & 1) od += c[k];
        else ev += c[k];
    }
    return edge ? ev + od : ev - od;
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
                         double* __restrict__ divN, double* __restrict__ divM, double* __restrict__ aM4,
                         double* __restrict__ divM4, double* __restrict__ vface, const double* __restrict__ tab,
                         double invdx, int cons, double vscale, int* __restrict__ vdeg)
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
        if (k < 4) aM4[(size_t)e * 4 + k] = c;
    }
    for (int k = N; k < 4; ++k) aM4[(size_t)e * 4 + k] = 0.0;
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
        if (k < 4) divM4[(size_t)e * 4 + k] = c;
    }
    for (int k = N; k < 4; ++k) divM4[(size_t)e * 4 + k] = 0.0;
    // effective degree of the velocity (and divergence) series
    {
        double c[N], cdv[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            c[k] = aM[(size_t)e * N + k];
            cdv[k] = divM[(size_t)e * N + k];
        }
        // the divergence series is evaluated off the nodes only in the
        // conservative form
        const int d = cons ? max(cheb_degree<N>(c, vscale), cheb_degree<N>(cdv)) : cheb_degree<N>(c, vscale);
        atomicMax(vdeg, d);
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
//
// n + 1 lanes per element: n node lanes and one edge lane.  The edge lane
// runs the backtraces from the element's upwind edge(s) in the same
// instruction stream as the node lanes' backtraces from the nodes, evaluates
// the remapped polynomial at 0 while the node lanes evaluate it at the nodes,
// and sums l(1) . phihat while node lanes 0 and 1 sum the mass and energy
// targets.
// ---------------------------------------------------------------------------
// (No occupancy attribute: the edge lane stores its stage sums as soon as
// they are complete, which keeps the per-lane state small enough for the
// default allocation to hold five waves per SIMD at order 16 with a short
// velocity series.)
template <int N, bool CONS, int NA, int RKS>
__device__ __forceinline__ void advect1d_body(const Step1DArgs& A, const int bid)
{
    const Tab<RKS> RK{A.rk};
    constexpr int L = N + 1;
    constexpr int E = kBlock / L;
    using O = Off<N>;
    __shared__ double s_a[E][N];
    __shared__ double s_d[E][N];
    __shared__ double s_p[E][N];
    __shared__ double s_q[E][N];
    __shared__ double s_x[E][N];
    __shared__ double s_c[E][N];
    __shared__ double s_r[2][E][N];
    __shared__ double s_ti[N * N];  // nodal-to-Chebyshev matrix (row k: coefficient k)
    __shared__ int s_flag;

    const int t = threadIdx.x;
    const int slot = t / L, i = t - slot * L;
    const bool inblk = slot < E;
    const int sl = inblk ? slot : 0;
    const bool node = i < N;
    const int in = node ? i : 0;
    const int e = bid * E + slot;
    const bool live = inblk && e < A.K;
    const double* __restrict__ tab = A.tab;
    const size_t g = (size_t)(live ? e : 0) * N + in;
    if (t == 0) s_flag = 0;

    // a velocity series of at most four terms is evaluated as a polynomial
    // in the element coordinate (cheb_to_mono), longer ones by Clenshaw;
    // only the coefficients that are evaluated are read
    constexpr bool MONO = NA <= 4;
    const double xi_i = tab[O::XI + in];
    const double invdx = A.invdx;
    double phi_i = 0.0, a_i = 0.0, dv_i = 0.0;
    if (live && node) {
        phi_i = A.phi[g];
        a_i = A.aN[g];
        if (A.targets || CONS) dv_i = A.divN[g];
    }
    if (inblk && node) {
        // a series of at most four terms reads the contiguous [K][4] copies:
        // whole lines of used coefficients instead of a few from each row
        const bool used = live && i < NA;
        const size_t g4 = (size_t)(live ? e : 0) * 4 + (i < 4 ? i : 0);
        s_a[slot][i] = used ? (MONO ? A.aM4[g4] : A.aM[g]) : 0.0;
        if (CONS) s_d[slot][i] = used ? (MONO ? A.divM4[g4] : A.divM[g]) : 0.0;
        s_p[slot][i] = phi_i;
    }
    const bool bt = A.iface == SL_IFACE_BACKTRACK;  // edge values by backtracking (eq. 4.11)
    const bool need_cp = A.targets || bt;           // phi^n off the nodes is evaluated
    if (need_cp)
        for (int k = t; k < N * N; k += kBlock) s_ti[k] = tab[O::TINV + k];
    __syncthreads();
    // Chebyshev coefficients of phi^n (for its values at backtraced feet);
    // zero when no foot is evaluated, so that LDS holds defined values
    if (inblk && node) {
        double c = 0.0;
        if (need_cp) {
#pragma unroll
            for (int j = 0; j < N; ++j) c = fma(s_ti[i * N + j], s_p[slot][j], c);
        }
        s_q[slot][i] = c;
    }

    double ca[N], cd[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ca[k] = (k < NA) ? s_a[sl][k] : 0.0;
        cd[k] = (CONS && k < NA) ? s_d[sl][k] : 0.0;
    }
    constexpr int NM = MONO ? NA : 1;
    double mu[NM], md[NM];
    if constexpr (MONO) {
        cheb_to_mono<NA, N>(ca, invdx, mu);
        cheb_to_mono<NA, N>(cd, 1.0, md);
    }
    const double k_i = a_i * invdx;
    bool out = false;
    // forward motion of particle i (section 4.2)
    double s = xi_i, q = phi_i;
    if (node) {
        if constexpr (MONO) rk_move_mono<CONS, NA, RKS>(A.rk, mu, md, A.dt, A.dt, s, q, out, true, k_i, dv_i);
        else rk_move<N, CONS, NA, RKS>(A.rk, ca, cd, 1.0, A.dt, invdx, s, q, out, true, a_i, dv_i);
    }
    __syncthreads();  // s_q complete
    const double* cp = s_q[sl];  // phi^n coefficients, read from LDS where used

    // element-local target parts: M^n, E^n, volume term at the RK abscissae
    // (node lanes), edge values at the RK abscissae on the upwind edges (edge
    // lane); backtracking as in eq. 4.11
    // upwind edges of the element (edge lane): where the flow leaves it, or
    // the face speed vanishes
    int first = -1, second = -1;
    if (need_cp && !node && live) {
        const double vL = A.vface[e];
        const double vR = A.vface[(A.periodic && e == A.K - 1) ? 0 : e + 1];
        const bool needL = !(vL > A.vzero), needR = !(vR < -A.vzero);
        first = needL ? 0 : (needR ? 1 : -1);
        second = (needL && needR) ? 1 : -1;
    }
    // the element's mean at t^n, c = M^n / sum W: the energy balance is
    // taken for the deviation phi - c (same law as for phi^2 in the PDE,
    // computed from differences of like size)
    double cmean = 0.0;
    if (A.targets) {
        double sw = 0.0;
        const double* pn = s_p[sl];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            cmean = fma(tab[O::W + j], pn[j], cmean);
            sw += tab[O::W + j];
        }
        cmean /= sw;
    }
    double vM = 0.0, vE = 0.0;
    if (A.targets) {
        const double W_i = A.dx * tab[O::W + in];
        if (!node && live) {
            // an edge without backtraces has zero stage sums
            double* rc = A.rec + (size_t)e * kRec1;
            if (first != 0 && second != 0) rc[2] = rc[4] = 0.0;
            if (first != 1 && second != 1) rc[3] = rc[5] = 0.0;
            rc[8] = cmean;
        }
        for (int r = 0; r < 2; ++r) {
            const int edge = (r == 0) ? first : second;
            const bool act = node ? (r == 0 && A.vol && live) : (edge >= 0);
            if (!act) continue;
            const double x0 = node ? xi_i : (double)edge;
            // sum_q bu_q v_q, sum_q bu_q (v_q - c) and sum_q bu_q (v_q - c)^2
            double am = 0.0, ad = 0.0, ae = 0.0;
            if constexpr (RKS == 4 && MONO) {
                // abscissae 0, 1/2, 1: both backtraces first, then phi^n at
                // the two feet in one pass over its coefficients
                double sb[2] = {x0, x0}, hq[2] = {1.0, 1.0}, xf[2], vf[2];
#pragma unroll
                for (int z = 0; z < 2; ++z) {
                    const double h = RK.cu(z + 1) * A.dt;
                    rk_move_mono<CONS, NA, RKS>(A.rk, mu, md, -h, h, sb[z], hq[z], out, node, k_i, dv_i);
                    xf[z] = 2.0 * sb[z] - 1.0;
                }
                clenshaw_multi<N, 2>(cp, xf, vf);
                const double val[3] = {node ? phi_i : cheb_end<N>(cp, edge), hq[0] * vf[0], hq[1] * vf[1]};
#pragma unroll
                for (int qd = 0; qd < 3; ++qd) {
                    const double dq = val[qd] - cmean;
                    am += RK.bu(qd) * val[qd];
                    ad += RK.bu(qd) * dq;
                    ae += RK.bu(qd) * dq * dq;
                }
            } else {
#pragma unroll
            for (int qd = 0; qd < 4; ++qd) {
                if (qd >= RK.nq()) break;
                const double cq = RK.cu(qd);
                double val;
                if (cq == 0.0) {
                    val = node ? phi_i : cheb_end<N>(cp, edge);
                } else {
                    double sb = x0, hq = 1.0;
                    const double h = cq * A.dt;
                    if constexpr (MONO) rk_move_mono<CONS, NA, RKS>(A.rk, mu, md, -h, h, sb, hq, out, node, k_i, dv_i);
                    else rk_move<N, CONS, NA, RKS>(A.rk, ca, cd, -1.0, h, invdx, sb, hq, out, node, a_i, dv_i);
                    val = hq * clenshaw_p<N>(cp, 2.0 * sb - 1.0);
                }
                const double bq = RK.bu(qd);
                const double dq = val - cmean;
                am += bq * val;
                ad += bq * dq;
                ae += bq * dq * dq;
            }
            }
            // node: volume terms (mass: + int (div a) phi in the advective
            // form; deviation energy: + int (div a) psi^2 advective,
            // - int (div a)(psi^2 + 2 c psi) conservative); edge lane: the
            // edge's stage sums, stored now
            if (node) {
                vM = W_i * dv_i * am;
                vE = W_i * dv_i * (CONS ? -fma(2.0 * cmean, ad, ae) : ae);
            } else {
                double* rc = A.rec + (size_t)e * kRec1;
                rc[2 + edge] = ad;
                rc[4 + edge] = ae;
            }
        }
        // per-node parts of the mass and deviation energy targets with their
        // volume terms: M^n (+ dt V_M) and sum W (phi^n - c)^2 + dt V_E
        if (inblk && node) {
            const double dn = phi_i - cmean;
            s_r[0][slot][i] = CONS ? W_i * phi_i : fma(A.dt, vM, W_i * phi_i);
            s_r[1][slot][i] = fma(A.dt, vE, W_i * dn * dn);
        }
    }

    // backtracking interface values (eq. 4.11): phi^n at the foot of the
    // characteristic through each upwind edge over the whole step, stored as
    // that edge's trace (the remap below leaves those slots alone)
    if (bt && !node && live) {
        for (int r = 0; r < 2; ++r) {
            const int edge = (r == 0) ? first : second;
            if (edge < 0) continue;
            double sb = (double)edge, hq = 1.0;
            if constexpr (MONO) rk_move_mono<CONS, NA, RKS>(A.rk, mu, md, -A.dt, A.dt, sb, hq, out, false, k_i, dv_i);
            else rk_move<N, CONS, NA, RKS>(A.rk, ca, cd, -1.0, A.dt, invdx, sb, hq, out, false, a_i, dv_i);
            A.rec[(size_t)e * kRec1 + edge] = hq * clenshaw_p<N>(cp, 2.0 * sb - 1.0);
        }
    }
    const bool bt0 = bt && (first == 0 || second == 0), bt1 = bt && (first == 1 || second == 1);

    // remap (eq. 4.9): phihat_i = sum_j c_j prod_{m != j} (xi_i - s_m),
    // c_j = phi*_j / prod_{m != j} (s_j - s_m); the edge lane evaluates the
    // same polynomial at 0, and its value at 1 is l(1) . phihat (eq.
    // remap_bnd; the polynomial has degree n - 1, so its nodal interpolant is
    // itself)
    if (inblk && node) s_x[slot][i] = s;
    __syncthreads();
    const double* xs = s_x[sl];  // moved positions, read from LDS where used
    if (node) {
        // pr = prod_{m != i} (s_i - s_m) = l'(s_i) for l(x) = prod_m (x - s_m),
        // by the product rule over the partial products P: the factor
        // s_i - s_i is exactly zero, after which D carries P_i times the
        // remaining factors, rounded as the direct product.  No test of m
        // against i, so every read of s_m is unconditional.
        double P = 1.0, D = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const double d = s - xs[m];
            D = fma(D, d, P);
            P *= d;
        }
        if (inblk) s_c[slot][i] = q / D;
    }
    __syncthreads();
    const double* cw = s_c[sl];
    const double xe = node ? xi_i : 0.0;
    double S = 0.0, P = 1.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double d = xe - xs[j];
        S = fma(S, d, cw[j] * P);
        P *= d;
    }
    // s_p (phi^n, read before the second barrier) takes l(1)_i phihat_i
    // store what is final before the last barrier
    int fl = 0;
    if (live) {
        if (out) fl |= FLAG_CONTAIN;
        if (node) {
            if (!isfinite(S)) fl |= FLAG_SINGULAR;
            A.phihat[g] = S;
        } else if (!bt0) {
            A.rec[(size_t)e * kRec1] = S;
        }
    }
    // s_p (phi^n, read before the second barrier) takes l(1)_i phihat_i
    if (inblk && node) s_p[slot][i] = tab[O::L1 + i] * S;
    __syncthreads();
    // one sum over the element's nodes in three lanes at once: the trace at 1
    // (edge lane, record slot 1), the mass target (node lane 0, slot 6) and
    // the energy target (node lane 1, slot 7), each summed in node order
    if (live && ((!node && !bt1) || (A.targets && i < 2))) {
        const double* src = node ? s_r[i][sl] : s_p[sl];
        double sum = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) sum += src[j];
        A.rec[(size_t)e * kRec1 + (node ? 6 + i : 1)] = sum;
    }
    if (fl) atomicOr(&s_flag, fl);
    __syncthreads();
    if (t == 0 && s_flag) A.flag_part[bid] |= s_flag;
}

template <int N, bool CONS, int NA, int RKS>
__global__ __launch_bounds__(kBlock) void k_advect1d(Step1DArgs A)
{
    advect1d_body<N, CONS, NA, RKS>(A, blockIdx.x);
}

// One step of several meshes in one launch: the blocks of request r are
// start[r] .. start[r + 1] - 1, each running the kernel above on the
// request's own arguments As[r] (its own buffers and statistics)
template <int N, bool CONS, int NA, int RKS>
__global__ __launch_bounds__(kBlock) void k_advect1d_batch(const Step1DArgs* __restrict__ As,
                                                           const int* __restrict__ start, int nreq)
{
    const int r = batch_request(start, nreq, blockIdx.x);
    advect1d_body<N, CONS, NA, RKS>(As[r], blockIdx.x - start[r]);
}

// ---------------------------------------------------------------------------
// constrained least squares: one lane per element, values in registers
// ---------------------------------------------------------------------------
constexpr int kConBlock = 64;  // one wave
constexpr int kConQ = 2;       // lanes per element (a pair)
constexpr int kConElems = kConBlock / kConQ;

// value of the lane whose index differs in bit 0 (CTRL 0xB1, quad_perm
// [1,0,3,2]): a DPP move within the pair, no LDS traffic
template <int CTRL>
__device__ __forceinline__ double lane_swap(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// sum over the element's pair of lanes (2k, 2k+1), the same in both
// (v0 + v1 = v1 + v0 exactly)
__device__ __forceinline__ double pair_sum(double v) { return v + lane_swap<0xB1>(v); }
__device__ __forceinline__ double pair_max(double v) { return fmax(v, lane_swap<0xB1>(v)); }

// Two lanes per element: lane r of the pair holds nodes r, r+2, r+4, ...
// (NP of them); row products are pair sums, and the small KKT / least-squares
// solve is repeated in both lanes.  32 elements per wave: at order 16 the
// kernel takes about 250 VGPRs (two waves per SIMD), and a 65536-element
// launch (2048 waves) is resident at once; with four lanes per element its
// 4096 waves at three per SIMD needed a second, mostly idle round.
template <int N>
__device__ __forceinline__ void constrain1d_body(const Step1DArgs& A, const int bid)
{
    using O = Off<N>;
    constexpr int NP = (N + kConQ - 1) / kConQ;
    constexpr int NR = (kConElems + 2) * kRec1;  // records of elements e0 - 1 .. e0 + kConElems
    constexpr int NF = kConElems + 1;        // faces e0 .. e0 + kConElems
    static_assert(3 * kConQ * NP <= kConBlock && NF <= kConBlock, "one table entry / face per lane");
    __shared__ double s_buf[kConElems * N];
    __shared__ double s_rec[NR];
    __shared__ double s_vf[NF];
    __shared__ double s_tab[3][kConQ][NP];  // l(0), l(1), w at node r + 2k of lane r ([row][r][k])
    __shared__ double s_st[kConElems][4];  // per-element statistics, reduced by four lanes
    __shared__ int s_fq[kConElems];
    const int t = threadIdx.x;
    const int le = t / kConQ, r = t % kConQ;
    const int e0 = bid * kConElems;
    const int K = A.K;
    const int e = e0 + le;
    const bool live = e < K;
    const int ee = live ? e : K - 1;
    const double* __restrict__ tab = A.tab;

    // every global load is a coalesced block load issued before the first
    // wait: phihat, the records of the block's elements and of one neighbour
    // on each side, the face speeds, and the table rows; the element's values
    // are then read from LDS
    constexpr int kStage = (kConElems * N + kConBlock - 1) / kConBlock;
    constexpr int kRStage = (NR + kConBlock - 1) / kConBlock;
    const int cnt = (K - e0 < kConElems ? K - e0 : kConElems) * N;
    double v[kStage], rv[kRStage];
#pragma unroll
    for (int r2 = 0; r2 < kStage; ++r2) {
        const int k = t + r2 * kConBlock;
        v[r2] = k < cnt ? A.phihat[(size_t)e0 * N + k] : 0.0;
    }
    // periodic wrap of an element or face index within [e0 - 1, e0 + kConElems]
    // (a division only on meshes smaller than the staged window)
    const bool small = K < kConElems + 2;
    auto wrap = [&](int i) { return small ? ((i % K) + K) % K : (i < 0 ? i + K : (i >= K ? i - K : i)); };
#pragma unroll
    for (int r3 = 0; r3 < kRStage; ++r3) {
        const int j = t + r3 * kConBlock;
        const int jr = j / kRec1;
        int ge = e0 + jr - 1;  // element of this record entry
        if (A.periodic) ge = wrap(ge);
        rv[r3] = (j < NR && ge >= 0 && ge < K) ? A.rec[(size_t)ge * kRec1 + (j - jr * kRec1)] : 0.0;
    }
    double fv = 0.0;
    if (t < NF) {
        // face e0 + t; on a periodic mesh face K is face 0, elsewhere the
        // K + 1 faces end at K
        const int f = e0 + t;
        fv = A.vface[A.periodic ? wrap(f) : (f < K ? f : K)];
    }
    double tv = 0.0;
    if (t < 3 * kConQ * NP) {
        // one load per lane, no branch on the row
        static_assert(O::L1 == O::L0 + N, "table layout");
        const int row = t / (kConQ * NP), j = (t / NP) % kConQ + kConQ * (t % NP);
        const int at = row == 2 ? O::W + j : O::L0 + row * N + j;
        if (j < N) tv = tab[at];
    }
    // ghost values at t^n and t^{n+1} (a bounded mesh only; scalar loads)
    double gw0 = 0.0, gw1 = 0.0, gn0 = 0.0, gn1 = 0.0;
    if (!A.periodic) {
        gn0 = A.gnext[0];
        gn1 = A.gnext[1];
        if (A.targets) {
            gw0 = A.gnow[0];
            gw1 = A.gnow[1];
        }
    }

    const bool bnd = (A.cmask & SL_C_BOUNDARY) != 0;
    const bool mass = (A.cmask & SL_C_MASS) != 0;
    const bool energy = (A.cmask & SL_C_ENERGY) != 0;

#pragma unroll
    for (int r2 = 0; r2 < kStage; ++r2) {
        const int k = t + r2 * kConBlock;
        if (k < kConElems * N) s_buf[k] = v[r2];
    }
#pragma unroll
    for (int r3 = 0; r3 < kRStage; ++r3) {
        const int j = t + r3 * kConBlock;
        if (j < NR) s_rec[j] = rv[r3];
    }
    if (t < NF) s_vf[t] = fv;
    if (t < 3 * kConQ * NP) (&s_tab[0][0][0])[t] = tv;
    __syncthreads();

    double l0[NP], l1[NP], Wn[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        l0[k] = s_tab[0][r][k];
        l1[k] = s_tab[1][r][k];
        Wn[k] = A.dx * s_tab[2][r][k];
    }

    // neighbours and face values at t^{n+1} (eq. 4.12a); the records of
    // element le - 1, le, le + 1 of the block sit at rows le, le + 1, le + 2
    int em = ee - 1, ep = ee + 1;
    if (A.periodic) {
        if (em < 0) em = K - 1;
        if (ep >= K) ep = 0;
    } else {
        if (em < 0) em = -1;
        if (ep >= K) ep = -1;
    }
    double vL = s_vf[le];
    double vR = s_vf[le + 1];
    if (fabs(vL) <= A.vzero) vL = 0.0;
    if (fabs(vR) <= A.vzero) vR = 0.0;
    const double* Rm = s_rec + le * kRec1;
    const double* Re = Rm + kRec1;
    const double* Rp = Re + kRec1;
    const double T1m = em >= 0 ? Rm[1] : gn0;
    const double T0p = ep >= 0 ? Rp[0] : gn1;
    const double dB0 = upwind(vL, T1m, Re[0]);
    const double dB1 = upwind(vR, Re[1], T0p);

    // targets: M^{n+1} and the deviation energy Ed^{n+1} = sum W (phi - c)^2
    // about the element's mean c at t^n, from the own record's volume parts
    // and the upwind edge sums.  A neighbour's sums are about its own mean
    // c'; with delta = c' - c, sum_q b_q (v_q - c)^2 = S2 + delta (2 S1 +
    // delta) and sum_q b_q v_q = S1 + c' (the weights b_q sum to one).
    // E^{n+1} = Ed + 2 c M - c^2 sum W is the energy target of phi^2.
    double Mt = 0.0, Edt = 0.0, Et = 0.0;
    const double cr = Re[8];
    if (A.targets) {
        double gM0 = 0.0, gE0 = 0.0, gM1 = 0.0, gE1 = 0.0;
        if (!A.periodic) {
            for (int qd = 0; qd < A.rk.nq; ++qd) {
                const double cq = A.rk.cu[qd];
                const double v0 = (1.0 - cq) * gw0 + cq * gn0;
                const double v1 = (1.0 - cq) * gw1 + cq * gn1;
                gM0 += A.rk.bu[qd] * v0;
                gE0 += A.rk.bu[qd] * (v0 - cr) * (v0 - cr);
                gM1 += A.rk.bu[qd] * v1;
                gE1 += A.rk.bu[qd] * (v1 - cr) * (v1 - cr);
            }
        }
        const double dm = Rm[8] - cr, dp = Rp[8] - cr;
        const double FMl = upwind(vL, em >= 0 ? Rm[3] + Rm[8] : gM0, Re[2] + cr);
        const double FEl = upwind(vL, em >= 0 ? fma(dm, fma(2.0, Rm[3], dm), Rm[5]) : gE0, Re[4]);
        const double FMr = upwind(vR, Re[3] + cr, ep >= 0 ? Rp[2] + Rp[8] : gM1);
        const double FEr = upwind(vR, Re[5], ep >= 0 ? fma(dp, fma(2.0, Rp[2], dp), Rp[4]) : gE1);
        Mt = Re[6] + A.dt * (vL * FMl - vR * FMr);
        Edt = Re[7] + A.dt * (vL * FEl - vR * FEr);
        Et = Edt + cr * (2.0 * Mt - cr * A.sumW);
    }

    // this lane's nodes (absent nodes are zero rows)
    double ph[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int j = r + kConQ * k;
        ph[k] = (live && j < N) ? s_buf[le * N + j] : 0.0;
    }
    __syncthreads();
    // rows l(0), l(1), W (mass), W*psi (energy); inactive rows are zero
    double Cph[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        Cph[0] = fma(l0[k], ph[k], Cph[0]);
        Cph[1] = fma(l1[k], ph[k], Cph[1]);
        Cph[2] = fma(Wn[k], ph[k], Cph[2]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) Cph[a] = pair_sum(Cph[a]);
    const double dd0 = bnd ? dB0 : 0.0, dd1 = bnd ? dB1 : 0.0, dd2 = mass ? Mt : 0.0;
    const double s0 = bnd ? 1.0 : 0.0, s1 = bnd ? 1.0 : 0.0, s2 = mass ? 1.0 : 0.0;
    bool singular = false;

    // one constrained solve.  The 3x3 block of rows l(0), l(1), W is the
    // same for every element (its inverse g3i comes with the launch); the
    // energy row borders it with its Gram entries red[0..3] (against l0,
    // l1, W, itself), its product with phihat red[4] and target d3, and is
    // eliminated through the Schur complement.  HARD: G y = C phihat - d;
    // SOFT: (I + G) z = C phihat + G d, y = z - d.  Returns false when the
    // energy row's Schur complement vanishes (the row lies in the span of the
    // others): then y4 = 0 and num holds the energy row's residual.
    auto solve = [&](bool use_e, const double (&red)[5], double d3, double (&y)[4], double& num) {
        const double ge[3] = {use_e ? red[0] * s0 : 0.0, use_e ? red[1] * s1 : 0.0, use_e ? red[2] * s2 : 0.0};
        const double gam = use_e ? red[3] : 0.0;
        const double dd[4] = {dd0, dd1, dd2, use_e ? d3 : 0.0};
        double r3[3] = {Cph[0] * s0, Cph[1] * s1, Cph[2] * s2};
        double r4 = use_e ? red[4] : 0.0;
        const bool soft = A.mode == SL_MODE_SOFT;
        if (soft) {
            const double G3[3][3] = {{bnd ? A.g00 : 0.0, bnd ? A.g01 : 0.0, (bnd && mass) ? A.g02 : 0.0},
                                     {bnd ? A.g01 : 0.0, bnd ? A.g11 : 0.0, (bnd && mass) ? A.g12 : 0.0},
                                     {(bnd && mass) ? A.g02 : 0.0, (bnd && mass) ? A.g12 : 0.0, mass ? A.g22 : 0.0}};
#pragma unroll
            for (int a = 0; a < 3; ++a) r3[a] += G3[a][0] * dd[0] + G3[a][1] * dd[1] + G3[a][2] * dd[2] + ge[a] * dd[3];
            r4 += ge[0] * dd[0] + ge[1] * dd[1] + ge[2] * dd[2] + gam * dd[3];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) r3[a] -= dd[a];
            r4 -= dd[3];
        }
        double z[3], w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            z[a] = A.g3i[3 * a] * r3[0] + A.g3i[3 * a + 1] * r3[1] + A.g3i[3 * a + 2] * r3[2];
            w[a] = A.g3i[3 * a] * ge[0] + A.g3i[3 * a + 1] * ge[1] + A.g3i[3 * a + 2] * ge[2];
        }
        double y4 = 0.0;
        bool ok = true;
        num = 0.0;
        if (use_e) {
            const double sch = (soft ? gam + 1.0 : gam) - (ge[0] * w[0] + ge[1] * w[1] + ge[2] * w[2]);
            num = r4 - (ge[0] * z[0] + ge[1] * z[1] + ge[2] * z[2]);
            ok = sch > 0.0;
            y4 = ok ? num / sch : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) y[a] = z[a] - w[a] * y4;
        y[3] = y4;
        if (soft)
#pragma unroll
            for (int a = 0; a < 4; ++a) y[a] -= dd[a];
        return ok;
    };

    double phi[NP], y[4], num;
    const double zero5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    solve(false, zero5, 0.0, y, num);
#pragma unroll
    for (int k = 0; k < NP; ++k) phi[k] = ph[k] - (l0[k] * s0 * y[0] + l1[k] * s1 * y[1] + Wn[k] * s2 * y[2]);

    // the energy row (section "Local energy conservation").  SOFT: the
    // paper's linearisation sum W phi^(k-1) phi = E^{n+1}, stacked with the
    // other rows.  HARD: its fixed point, reached by Newton's linearisation
    // of the same row, written for y = phi - sh with the target T:
    //   sum W y^(k-1) y = (T + sum W (y^(k-1))^2) / 2,
    // with a mass row as the deviation from the element's mean (sh = c,
    // T = Ed^{n+1}: the same constraint on the mass row's level set),
    // otherwise sh = 0, T = E^{n+1}.  Each sweep solves from phihat; stop
    // when max |phi^(k) - phi^(k-1)| < tol (strict, as printed).
    const bool hard = A.mode == SL_MODE_HARD;
    const bool devf = hard && mass;
    const double sh = devf ? cr : 0.0;
    int iters = 0;
    bool conv = false;
    if (energy && live) {
        const double Tt = devf ? Edt : Et;
        for (int it = 1; it <= A.emaxit; ++it) {
            double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, en = 0.0;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double yk = phi[k] - sh;
                const double c3 = Wn[k] * yk;
                red[0] += c3 * l0[k];
                red[1] += c3 * l1[k];
                red[2] += c3 * Wn[k];
                red[3] += c3 * c3;
                red[4] += c3 * (ph[k] - sh);
                en += c3 * yk;
            }
#pragma unroll
            for (int a = 0; a < 5; ++a) red[a] = pair_sum(red[a]);
            en = pair_sum(en);
            const bool ok = solve(true, red, hard ? 0.5 * (Tt + en) : Et, y, num);
            double diff = 0.0;
            if (ok) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double c3 = Wn[k] * (phi[k] - sh);
                    const double nv = ph[k] - (l0[k] * s0 * y[0] + l1[k] * s1 * y[1] + Wn[k] * s2 * y[2] + c3 * y[3]);
                    diff = fmax(diff, fabs(nv - phi[k]));
                    phi[k] = nv;
                }
            } else if (num != 0.0) {
                singular = true;
            }
            diff = pair_max(diff);
            iters = it;
            if (diff < A.etol) {
                conv = true;
                break;
            }
        }
    }

    // residuals of the rows actually imposed (energy: HARD with a mass row
    // in the deviation form, otherwise sum W phi^2 against E^{n+1})
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        r0 = fma(l0[k], phi[k], r0);
        r1 = fma(l1[k], phi[k], r1);
        r2 = fma(Wn[k], phi[k], r2);
        r3 = fma(Wn[k] * (phi[k] - sh), phi[k] - sh, r3);
        finite = finite && isfinite(phi[k]);
    }
    r0 = pair_sum(r0);
    r1 = pair_sum(r1);
    r2 = pair_sum(r2);
    r3 = pair_sum(r3);
    double rb = (live && bnd) ? fmax(fabs(r0 - dB0), fabs(r1 - dB1)) : 0.0;
    double rm = (live && mass) ? fabs(r2 - Mt) : 0.0;
    double re = (live && energy) ? fabs(r3 - (devf ? Edt : Et)) : 0.0;
    double pic = live ? (double)iters : 0.0;
    int fl = 0;
    if (live) {
        if (energy && !conv && A.etol > 0.0) fl |= FLAG_NOCONV;
        if (singular) fl |= FLAG_SINGULAR;
        if (!finite) fl |= FLAG_NONFINITE;
    }
    // per-element statistics (the same in the pair's two lanes), reduced
    // over the block after the next barrier
    if (r == 0) {
        s_st[le][0] = rb;
        s_st[le][1] = rm;
        s_st[le][2] = re;
        s_st[le][3] = pic;
        s_fq[le] = fl;
    }

    // coalesced store of phi^{n+1}
    if (live) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int j = r + kConQ * k;
            if (j < N) s_buf[le * N + j] = phi[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r2 = 0; r2 < kStage; ++r2) {
        const int k = t + r2 * kConBlock;
        if (k < cnt) A.phi_out[(size_t)e0 * N + k] = s_buf[k];
    }
    if (t < 4) {  // lane a: statistic a
        double m = 0.0;
#pragma unroll
        for (int q = 0; q < kConElems; ++q) m = fmax(m, s_st[q][t]);
        double* sp = A.stat_part + (size_t)bid * kStatSlots;
        sp[t] = fmax(sp[t], m);
    } else if (t == 4) {
        int f = 0;
#pragma unroll
        for (int q = 0; q < kConElems; ++q) f |= s_fq[q];
        if (f) A.flag_part[A.nblk + bid] |= f;
    }
}

template <int N>
__global__ __launch_bounds__(kConBlock) void k_constrain1d(Step1DArgs A)
{
    constrain1d_body<N>(A, blockIdx.x);
}

template <int N>
__global__ __launch_bounds__(kConBlock) void k_constrain1d_batch(const Step1DArgs* __restrict__ As,
                                                                 const int* __restrict__ start, int nreq)
{
    const int r = batch_request(start, nreq, blockIdx.x);
    constrain1d_body<N>(As[r], blockIdx.x - start[r]);
}

template <int N>
int launch_prep_n(int K, int periodic, int has_div, const double* aN, double* aM, double* divN, double* divM,
                  double* aM4, double* divM4, double* vface, const double* tab, double dx, int cons, double vscale,
                  int* vdeg, hipStream_t s)
{
    const int bs = 128;
    hipLaunchKernelGGL(k_prep1d<N>, dim3((K + bs - 1) / bs), dim3(bs), 0, s, K, periodic, has_div, aN, aM, divN,
                       divM, aM4, divM4, vface, tab, 1.0 / dx, cons, vscale, vdeg);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N, int NA>
void launch_adv_na(const Step1DArgs& A, dim3 grid, hipStream_t s)
{
    const bool rk4 = A.rk.s == 4;  // the classical tableau, the only 4-stage one
    if (A.cons) {
        if (rk4) launch_timed((k_advect1d<N, true, NA, 4>), grid, dim3(kBlock), 0, s, A);
        else launch_timed((k_advect1d<N, true, NA, 0>), grid, dim3(kBlock), 0, s, A);
    } else {
        if (rk4) launch_timed((k_advect1d<N, false, NA, 4>), grid, dim3(kBlock), 0, s, A);
        else launch_timed((k_advect1d<N, false, NA, 0>), grid, dim3(kBlock), 0, s, A);
    }
}

// velocity series evaluated with 4, 8 or all n Chebyshev terms: the fewest
// that cover the mesh-wide effective degree
template <int N>
int launch_adv_n(const Step1DArgs& A, hipStream_t s)
{
    constexpr int E = kBlock / (N + 1);
    dim3 grid((A.K + E - 1) / E);
    const int need = A.vdeg + 1;
    if (N > 4 && need <= 4) launch_adv_na<N, (N > 4 ? 4 : N)>(A, grid, s);
    else if (N > 8 && need <= 8) launch_adv_na<N, (N > 8 ? 8 : N)>(A, grid, s);
    else launch_adv_na<N, N>(A, grid, s);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int launch_con_n(const Step1DArgs& A, hipStream_t s)
{
    dim3 grid((A.K + kConElems - 1) / kConElems);
    launch_timed(k_constrain1d<N>, grid, dim3(kConBlock), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

// batched launches: the advect's template variant is chosen as for one
// mesh (launch_adv_n) from A0, which every member shares (advect1d_variant)
template <int N, int NA>
void launch_adv_batch_na(const Step1DArgs& A0, const Step1DArgs* As, const int* start, int nreq, int nblocks,
                         hipStream_t s)
{
    const bool rk4 = A0.rk.s == 4;
    const dim3 grid(nblocks), block(kBlock);
    if (A0.cons) {
        if (rk4) hipLaunchKernelGGL((k_advect1d_batch<N, true, NA, 4>), grid, block, 0, s, As, start, nreq);
        else hipLaunchKernelGGL((k_advect1d_batch<N, true, NA, 0>), grid, block, 0, s, As, start, nreq);
    } else {
        if (rk4) hipLaunchKernelGGL((k_advect1d_batch<N, false, NA, 4>), grid, block, 0, s, As, start, nreq);
        else hipLaunchKernelGGL((k_advect1d_batch<N, false, NA, 0>), grid, block, 0, s, As, start, nreq);
    }
}

// number of velocity series terms the advect evaluates (launch_adv_n's choice)
template <int N>
int adv_terms_n(int vdeg)
{
    const int need = vdeg + 1;
    return (N > 4 && need <= 4) ? 4 : (N > 8 && need <= 8) ? 8 : N;
}

template <int N>
int launch_adv_batch_n(const Step1DArgs& A0, const Step1DArgs* As, const int* start, int nreq, int nblocks,
                       hipStream_t s)
{
    const int na = adv_terms_n<N>(A0.vdeg);
    if (na == 4) launch_adv_batch_na<N, (N > 4 ? 4 : N)>(A0, As, start, nreq, nblocks, s);
    else if (na == 8) launch_adv_batch_na<N, (N > 8 ? 8 : N)>(A0, As, start, nreq, nblocks, s);
    else launch_adv_batch_na<N, N>(A0, As, start, nreq, nblocks, s);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

template <int N>
int launch_con_batch_n(const Step1DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_constrain1d_batch<N>, dim3(nblocks), dim3(kConBlock), 0, s, As, start, nreq);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace

int blocks1d(int n, int K)
{
    if (n < 2 || n > kMax1D) return 0;
    const int E = kBlock / (n + 1);
    const int a = (K + E - 1) / E, c = (K + kConElems - 1) / kConElems;
    return a > c ? a : c;
}

#define PREP_CALL(N) \
    launch_prep_n<N>(K, periodic, has_div, aN, aM, divN, divM, aM4, divM4, vface, tab, dx, cons, vscale, vdeg, s)
int launch_prep1d(int n, int K, int periodic, int has_div, const double* aN, double* aM, double* divN,
                  double* divM, double* aM4, double* divM4, double* vface, const double* tab, double dx, int cons,
                  double vscale, int* vdeg, hipStream_t s)
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

#define SL1D_CASES(F)                                                                                    \
    case 2: return F(2); case 3: return F(3); case 4: return F(4); case 5: return F(5);                  \
    case 6: return F(6); case 7: return F(7); case 8: return F(8); case 9: return F(9);                  \
    case 10: return F(10); case 11: return F(11); case 12: return F(12); case 13: return F(13);           \
    case 14: return F(14); case 15: return F(15); case 16: return F(16); case 17: return F(17);

// template variant of the advect for A: the members of one batched launch
// share it (series terms evaluated, form, the classical RK4 tableau or not)
int advect1d_variant(int n, const Step1DArgs& A)
{
    int na = -1;
    switch (n) {
#define TERMS(N) \
    case N: na = adv_terms_n<N>(A.vdeg); break;
        TERMS(2) TERMS(3) TERMS(4) TERMS(5) TERMS(6) TERMS(7) TERMS(8) TERMS(9)
        TERMS(10) TERMS(11) TERMS(12) TERMS(13) TERMS(14) TERMS(15) TERMS(16) TERMS(17)
#undef TERMS
    default: break;
    }
    if (na < 0) return -1;
    return na * 4 + (A.cons ? 2 : 0) + (A.rk.s == 4 ? 1 : 0);
}

int advect1d_blocks(int n, int K) { return (K + kBlock / (n + 1) - 1) / (kBlock / (n + 1)); }

int constrain1d_blocks(int K) { return (K + kConElems - 1) / kConElems; }

int launch_advect1d_batch(int n, const Step1DArgs& A0, const Step1DArgs* As, const int* start, int nreq,
                          int nblocks, hipStream_t s)
{
    switch (n) {
#define ADVB(N) launch_adv_batch_n<N>(A0, As, start, nreq, nblocks, s)
        SL1D_CASES(ADVB)
#undef ADVB
    default: return 1;
    }
}

int launch_constrain1d_batch(int n, const Step1DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s)
{
    switch (n) {
#define CONB(N) launch_con_batch_n<N>(As, start, nreq, nblocks, s)
        SL1D_CASES(CONB)
#undef CONB
    default: return 1;
    }
}
#undef SL1D_CASES


}  // namespace sl
