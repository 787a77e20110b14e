/*
 * sl_oracle.c -- plain, slow, FP64 CPU reference of one explicit
 * semi-Lagrangian spectral (DSEM-SL) step, after Natarajan & Jacobs,
 * "An explicit semi-Lagrangian, spectral method for solution of Lagrangian
 * transport equations in Eulerian-Lagrangian formulations" (arXiv 1910.06476).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library: every table here is recomputed from its mathematical definition.
 *
 * The routes are chosen to be obviously correct, not fast:
 *   - Lagrange basis in product form (section 3, eq. 3.5; section 4.1 eq. 4.3),
 *   - the remap (eq. 4.9 in 1D, eq. 5.4 in 2D) as a dense solve of the
 *     moved-point Vandermonde system by LU with partial pivoting,
 *   - the constrained least squares (eq. matrix_a) as the full KKT system
 *     (HARD) or the normal equations of the stacked system (SOFT), both by LU,
 *   - the 2D boundary pseudo-inverse from a cyclic Jacobi eigen-decomposition.
 *
 * Readings of the paper (where it is silent or garbled) are listed in the
 * design notes of the repository; each is marked "reading" where used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Public parameter block (mirrored by oracle/__init__.py).                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;          /* 1 or 2 */
    int32_t kx, ky;       /* elements per direction (ky = 1 in 1D) */
    int32_t n;            /* nodes per direction (order N = n - 1) */
    int32_t family;       /* 0 Gauss-Legendre, 1 Chebyshev-Gauss (eq. gaussquad) */
    int32_t bc;           /* 0 periodic, 1 ghost values at the domain boundary;  */
                          /* 2D only: 2 periodic in x, ghost values on the       */
                          /* bottom and top sides; 3 ghost values on the left    */
                          /* and right sides, periodic in y                      */
    int32_t form;         /* 0 advective u_t + a.grad u = 0, 1 conservative (eq. 2.3) */
    int32_t rk;           /* tableau id, see rk_tableau() */
    int32_t cmask;        /* bit0 boundary, bit1 mass, bit2 energy */
    int32_t mode;         /* 0 HARD (KKT), 1 SOFT (stacked least squares, eq. matrix_a) */
    int32_t energy_maxit; /* Picard iterations cap */
    int32_t vel_kind;     /* 0 nodal arrays; >0 analytic field (paper pins only) */
    double x0, x1, y0, y1;
    double energy_tol;    /* Picard stop: max |phi^(k) - phi^(k-1)| < tol */
    double vel_param[4];
    int32_t iface;        /* interface values: 0 interpolation (eq. remap_bnd),
                             1 backtracking (eq. 4.11) */
} ora_params;

typedef struct {
    double resid_boundary; /* max |C_B phi - d_B| (least-squares sense in 2D) */
    double resid_mass;     /* max |W.phi - M^{n+1}| */
    double resid_energy;   /* max |W.phi^2 - E^{n+1}| */
    int32_t max_picard;    /* largest number of energy-row solves */
    int32_t flags;         /* bit0 non-finite, bit1 particle left element,
                              bit2 singular system, bit3 Picard not converged */
} ora_stats;

enum { F_NONFINITE = 1, F_CONTAIN = 2, F_SINGULAR = 4, F_NOCONV = 8 };
enum { C_BOUND = 1, C_MASS = 2, C_ENERGY = 4 };

/* ------------------------------------------------------------------------ */
/* Node families on the unit reference interval [0, 1].                      */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre: the n roots of P_n, found by Newton iteration on the
 * three-term recurrence in long double; weight 2/((1-t^2) P_n'(t)^2) on
 * [-1,1], halved for [0,1].  Returned in ascending order. */
static void gl_rule(int n, double* xi, double* w)
{
    for (int i = 0; i < n; ++i) {
        long double t = cosl((long double)M_PI * (i + 0.75L) / (n + 0.5L));
        long double pn = 0, dp = 1;
        for (int it = 0; it < 200; ++it) {
            long double p0 = 1.0L, p1 = t;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pn = p1;
            dp = (n == 1) ? 1.0L : n * (t * p1 - p0) / (t * t - 1.0L);
            long double step = pn / dp;
            t -= step;
            if (fabsl(step) < 1e-20L) break;
        }
        /* re-evaluate at the converged root for the weight */
        {
            long double p0 = 1.0L, p1 = t;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = (n == 1) ? 1.0L : n * (t * p1 - p0) / (t * t - 1.0L);
        }
        long double wt = 2.0L / ((1.0L - t * t) * dp * dp);
        /* t descends with i, so x = (1 - t)/2 ascends */
        xi[i] = (double)((1.0L - t) * 0.5L);
        w[i] = (double)(wt * 0.5L);
    }
}

/* Chebyshev-Gauss (section 3, eq. gaussquad with n = N+1 points; reading:
 * angle (j+1/2) pi / n): xi_j = (1 - cos theta_j)/2.  Weights are the
 * interpolatory ones, w_j = int_0^1 l_j, in closed form (Fejer's first rule):
 * on [-1,1], w_j = (2/n) [1 - 2 sum_{k=1}^{n/2} cos(2 k theta_j)/(4k^2-1)]. */
static void cg_rule(int n, double* xi, double* w)
{
    for (int j = 0; j < n; ++j) {
        double th = M_PI * (j + 0.5) / n;
        xi[j] = 0.5 * (1.0 - cos(th));
        double s = 0.0;
        for (int k = 1; k <= n / 2; ++k) s += cos(2.0 * k * th) / (4.0 * k * k - 1.0);
        w[j] = 0.5 * (2.0 / n) * (1.0 - 2.0 * s);
    }
}

int ora_nodes(int family, int n, double* xi, double* w)
{
    if (n < 1 || n > 64) return 1;
    if (family == 0) gl_rule(n, xi, w);
    else if (family == 1) cg_rule(n, xi, w);
    else return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lagrange basis in product form (eq. 3.5 / eq. 4.3).                       */
/* ------------------------------------------------------------------------ */
static void lag_basis(int n, const double* x, double t, double* l)
{
    for (int j = 0; j < n; ++j) {
        double num = 1.0, den = 1.0;
        for (int m = 0; m < n; ++m) {
            if (m == j) continue;
            num *= (t - x[m]);
            den *= (x[j] - x[m]);
        }
        l[j] = num / den;
    }
}

/* d/dt of each basis polynomial: sum over the dropped factor k of the
 * remaining product (product rule), no division by (t - x_k). */
static void lag_basis_deriv(int n, const double* x, double t, double* dl)
{
    for (int j = 0; j < n; ++j) {
        double den = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) den *= (x[j] - x[m]);
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            if (k == j) continue;
            double p = 1.0;
            for (int m = 0; m < n; ++m)
                if (m != j && m != k) p *= (t - x[m]);
            s += p;
        }
        dl[j] = s / den;
    }
}

int ora_lagrange(int n, const double* x, double t, double* l)
{
    lag_basis(n, x, t, l);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting: solves A x = b in place (A n-by-n, row    */
/* major, destroyed; b overwritten by x).  Returns 1 if a zero pivot shows.  */
/* ------------------------------------------------------------------------ */
static int lu_solve(int n, double* A, double* b, int nrhs)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        if (best == 0.0 || !isfinite(best)) return 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
            for (int r = 0; r < nrhs; ++r) { double t = b[k * nrhs + r]; b[k * nrhs + r] = b[p * nrhs + r]; b[p * nrhs + r] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int r = 0; r < nrhs; ++r) b[i * nrhs + r] -= f * b[k * nrhs + r];
        }
    }
    for (int r = 0; r < nrhs; ++r) {
        for (int i = n - 1; i >= 0; --i) {
            double s = b[i * nrhs + r];
            for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j * nrhs + r];
            b[i * nrhs + r] = s / A[i * n + i];
        }
    }
    return 0;
}

/* Symmetric eigen-decomposition by cyclic Jacobi rotations (A n-by-n,
 * destroyed; eigenvalues on return in lam, eigenvectors in columns of Q). */
static void jacobi_eig(int n, double* A, double* lam, double* Q)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) { /* columns p, q */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* rows p, q */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - s * qkq;
                    Q[k * n + q] = s * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

/* ------------------------------------------------------------------------ */
/* Explicit Runge-Kutta tableaux.  Ids 1..4 are the ones the method uses     */
/* (Euler, Heun, Kutta's third order, classical fourth order); 5..7 are      */
/* alternative second/third-order tableaux kept for the paper-pin study.     */
/* ------------------------------------------------------------------------ */
typedef struct { int s; double a[4][4], b[4], c[4]; } tableau;

static int rk_tableau(int id, tableau* T)
{
    memset(T, 0, sizeof(*T));
    switch (id) {
    case 1: T->s = 1; T->b[0] = 1; return 0;
    case 2: /* Heun / explicit trapezoid */
        T->s = 2; T->a[1][0] = 1; T->b[0] = 0.5; T->b[1] = 0.5; T->c[1] = 1; return 0;
    case 3: /* Kutta third order */
        T->s = 3; T->a[1][0] = 0.5; T->a[2][0] = -1; T->a[2][1] = 2;
        T->b[0] = 1.0 / 6; T->b[1] = 2.0 / 3; T->b[2] = 1.0 / 6;
        T->c[1] = 0.5; T->c[2] = 1; return 0;
    case 4: /* classical fourth order */
        T->s = 4; T->a[1][0] = 0.5; T->a[2][1] = 0.5; T->a[3][2] = 1;
        T->b[0] = 1.0 / 6; T->b[1] = 1.0 / 3; T->b[2] = 1.0 / 3; T->b[3] = 1.0 / 6;
        T->c[1] = 0.5; T->c[2] = 0.5; T->c[3] = 1; return 0;
    case 5: /* explicit midpoint */
        T->s = 2; T->a[1][0] = 0.5; T->b[1] = 1; T->c[1] = 0.5; return 0;
    case 6: /* SSP third order (Shu-Osher) */
        T->s = 3; T->a[1][0] = 1; T->a[2][0] = 0.25; T->a[2][1] = 0.25;
        T->b[0] = 1.0 / 6; T->b[1] = 1.0 / 6; T->b[2] = 2.0 / 3;
        T->c[1] = 1; T->c[2] = 0.5; return 0;
    case 7: /* Ralston second order */
        T->s = 2; T->a[1][0] = 2.0 / 3; T->b[0] = 0.25; T->b[1] = 0.75; T->c[1] = 2.0 / 3; return 0;
    default: return 1;
    }
}

/* distinct abscissae of a tableau with their summed weights: the balance
 * laws for mass and energy depend on time only, so the tableau reduces to
 * the quadrature sum_s b_s R(t^n + c_s dt). */
static int rk_nodes(const tableau* T, double* cu, double* bu)
{
    int m = 0;
    for (int s = 0; s < T->s; ++s) {
        int f = -1;
        for (int q = 0; q < m; ++q)
            if (cu[q] == T->c[s]) f = q;
        if (f < 0) { cu[m] = T->c[s]; bu[m] = T->b[s]; ++m; }
        else bu[f] += T->b[s];
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Context shared by the phases of one step.                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const ora_params* p;
    int n, nd, K;          /* nodes per dir, nodes per element, elements */
    double dx, dy;
    double xi[64], w[64];  /* reference nodes / weights on [0,1] */
    double l0[64], l1[64]; /* l_j(0), l_j(1) */
    const double* a;       /* nodal velocity, component-major [dim][K][nd] */
    double* div;           /* nodal divergence [K][nd] */
    tableau T;
    double dt;
    double vzero;          /* face speeds with |v| <= vzero count as zero */
} ctx;

/* physical velocity and divergence at reference point (s, r) of element e */
static void vel_eval(const ctx* c, int e, double s, double r, double* u, double* v, double* dv)
{
    const ora_params* p = c->p;
    int n = c->n;
    if (p->vel_kind == 0) {
        double ls[64], lr[64];
        lag_basis(n, c->xi, s, ls);
        if (p->dim == 1) {
            double su = 0, sd = 0;
            for (int j = 0; j < n; ++j) {
                su += c->a[e * n + j] * ls[j];
                sd += c->div[e * n + j] * ls[j];
            }
            *u = su; *v = 0; *dv = sd;
        } else {
            lag_basis(n, c->xi, r, lr);
            const double* au = c->a + (size_t)e * c->nd;
            const double* av = c->a + (size_t)c->K * c->nd + (size_t)e * c->nd;
            const double* dd = c->div + (size_t)e * c->nd;
            double su = 0, sv = 0, sd = 0;
            for (int jj = 0; jj < n; ++jj)
                for (int ii = 0; ii < n; ++ii) {
                    double h = ls[ii] * lr[jj];
                    su += au[ii + n * jj] * h;
                    sv += av[ii + n * jj] * h;
                    sd += dd[ii + n * jj] * h;
                }
            *u = su; *v = sv; *dv = sd;
        }
        return;
    }
    /* analytic fields, physical coordinates */
    int ex = (p->dim == 1) ? e : e % p->kx, ey = (p->dim == 1) ? 0 : e / p->kx;
    double x = p->x0 + (ex + s) * c->dx;
    double y = p->y0 + (ey + r) * c->dy;
    const double* q = p->vel_param;
    switch (p->vel_kind) {
    case 1: *u = q[0]; *v = q[1]; *dv = 0; break;                      /* constant */
    case 2: *u = -sin(x); *v = 0; *dv = -cos(x); break;                  /* u = -sin x */
    case 3: *u = 1.0 + 0.5 * sin(M_PI * x); *v = 0; *dv = 0.5 * M_PI * cos(M_PI * x); break;
    case 4: *u = -(y - 0.5); *v = x - 0.5; *dv = 0; break;               /* rotation */
    case 5: {                                                            /* swirl */
        double sx = sin(M_PI * x), sy = sin(M_PI * y);
        *u = sx * sx * sin(2 * M_PI * y);
        *v = -sy * sy * sin(2 * M_PI * x);
        *dv = 0;
        break;
    }
    default: *u = *v = *dv = 0;
    }
}

/* value of the nodal field f (one element, nd values) at (s, r) */
static double field_eval(const ctx* c, const double* f, double s, double r)
{
    int n = c->n;
    double ls[64], lr[64];
    lag_basis(n, c->xi, s, ls);
    if (c->p->dim == 1) {
        double acc = 0;
        for (int j = 0; j < n; ++j) acc += f[j] * ls[j];
        return acc;
    }
    lag_basis(n, c->xi, r, lr);
    double acc = 0;
    for (int jj = 0; jj < n; ++jj)
        for (int ii = 0; ii < n; ++ii) acc += f[ii + n * jj] * ls[ii] * lr[jj];
    return acc;
}

/* containment test of a reference coordinate, with a 1e-10 allowance for
 * traces that start on a face where the face velocity vanishes */
static int outside(double s) { return s < -1e-10 || s > 1.0 + 1e-10; }

/* One RK step of length h for Y = (s, r, q) of element e.
 * dir = +1: forward particle motion, ds/dt = u/dx, dr/dt = v/dy and, in the
 *           conservative form, dq/dt = -div * q (section 4.2, eq. 4.4a, 4.8).
 * dir = -1: backward trace, ds/dt = -u/dx, dr/dt = -v/dy, dq/dt = -div * q
 *           (q is then the source factor accumulated along the path).
 * Returns 1 if a stage position (or the result) leaves [0,1]^d. */
static int rk_move(const ctx* c, int e, int dir, double h, double* s, double* r, double* q)
{
    const tableau* T = &c->T;
    int cons = (c->p->form == 1), d2 = (c->p->dim == 2);
    double ks[4], kr[4], kq[4];
    int out = 0;
    for (int st = 0; st < T->s; ++st) {
        double ss = *s, rr = *r, qq = *q;
        for (int j = 0; j < st; ++j) {
            ss += h * T->a[st][j] * ks[j];
            rr += h * T->a[st][j] * kr[j];
            qq += h * T->a[st][j] * kq[j];
        }
        if (outside(ss) || (d2 && outside(rr))) out = 1;
        double u, v, dv;
        vel_eval(c, e, ss, d2 ? rr : 0.0, &u, &v, &dv);
        ks[st] = dir * u / c->dx;
        kr[st] = d2 ? dir * v / c->dy : 0.0;
        kq[st] = cons ? -dv * qq : 0.0;
    }
    for (int st = 0; st < T->s; ++st) {
        *s += h * T->b[st] * ks[st];
        *r += h * T->b[st] * kr[st];
        *q += h * T->b[st] * kq[st];
    }
    if (outside(*s) || (d2 && outside(*r))) out = 1;
    return out;
}

/* value of phi^n of element e carried along the backward trace of length h
 * from reference point (s, r): phi^n(foot) times the source factor */
static double backtrace_value(const ctx* c, int e, const double* phin, double h, double s, double r, int* flags)
{
    double q = 1.0;
    if (h > 0 && rk_move(c, e, -1, h, &s, &r, &q)) *flags |= F_CONTAIN;
    return q * field_eval(c, phin + (size_t)e * c->nd, s, r);
}

static double upwind(double vn, double left, double right)
{
    if (vn > 0) return left;
    if (vn < 0) return right;
    return 0.5 * (left + right);
}

/* ------------------------------------------------------------------------ */
/* Constrained least squares (section "Least-squares solution of the        */
/* constrained system", eq. matrix_a).                                       */
/*   HARD: min ||phi - phihat||  s.t.  C phi = d      (full KKT, LU)         */
/*   SOFT: min ||phi - phihat||^2 + ||C phi - d||^2  ((I + C^T C) phi = ...) */
/* ------------------------------------------------------------------------ */
static int cls_solve(int nd, int m, const double* C, const double* d, const double* phihat, int mode, double* phi)
{
    if (mode == 0) {
        int N = nd + m;
        double* A = calloc((size_t)N * N, sizeof(double));
        double* b = calloc((size_t)N, sizeof(double));
        for (int i = 0; i < nd; ++i) { A[i * N + i] = 1.0; b[i] = phihat[i]; }
        for (int r = 0; r < m; ++r) {
            for (int i = 0; i < nd; ++i) {
                A[(nd + r) * N + i] = C[r * nd + i];
                A[i * N + nd + r] = C[r * nd + i];
            }
            b[nd + r] = d[r];
        }
        int bad = lu_solve(N, A, b, 1);
        for (int i = 0; i < nd; ++i) phi[i] = b[i];
        free(A); free(b);
        return bad;
    } else {
        double* A = calloc((size_t)nd * nd, sizeof(double));
        double* b = calloc((size_t)nd, sizeof(double));
        for (int i = 0; i < nd; ++i) {
            A[i * nd + i] = 1.0;
            b[i] = phihat[i];
            for (int r = 0; r < m; ++r) b[i] += C[r * nd + i] * d[r];
            for (int j = 0; j < nd; ++j)
                for (int r = 0; r < m; ++r) A[i * nd + j] += C[r * nd + i] * C[r * nd + j];
        }
        int bad = lu_solve(nd, A, b, 1);
        for (int i = 0; i < nd; ++i) phi[i] = b[i];
        free(A); free(b);
        return bad;
    }
}

/* ------------------------------------------------------------------------ */
/* 2D boundary rows: C_B (4n x n^2), ordered left j, right j, bottom i,      */
/* top i; node index i + n j with i along x.  Row space has dimension 4n-4  */
/* (one dependency per corner), so the boundary data are imposed through    */
/* the pseudo-inverse (reading of the one-sentence 2D remap).               */
/* ------------------------------------------------------------------------ */
static void build_CB(const ctx* c, double* CB)
{
    int n = c->n, nd = c->nd;
    memset(CB, 0, sizeof(double) * 4 * n * nd);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            CB[(0 * n + j) * nd + i + n * j] = c->l0[i];
            CB[(1 * n + j) * nd + i + n * j] = c->l1[i];
            CB[(2 * n + i) * nd + i + n * j] = c->l0[j];
            CB[(3 * n + i) * nd + i + n * j] = c->l1[j];
        }
}

/* CBp = C_B^+ (n^2 x 4n) = C_B^T (C_B C_B^T)^+, with the Gram pseudo-inverse
 * from its eigen-decomposition (eigenvalues below 1e-12 * max dropped). */
static void build_CBpinv(const ctx* c, const double* CB, double* CBp)
{
    int n = c->n, nd = c->nd, m = 4 * n;
    double* G = malloc(sizeof(double) * m * m);
    double* Q = malloc(sizeof(double) * m * m);
    double* lam = malloc(sizeof(double) * m);
    double* Gp = malloc(sizeof(double) * m * m);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0;
            for (int i = 0; i < nd; ++i) s += CB[a * nd + i] * CB[b * nd + i];
            G[a * m + b] = s;
        }
    jacobi_eig(m, G, lam, Q);
    double lmax = 0;
    for (int a = 0; a < m; ++a) lmax = fmax(lmax, fabs(lam[a]));
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0;
            for (int k = 0; k < m; ++k)
                if (lam[k] > 1e-12 * lmax) s += Q[a * m + k] * Q[b * m + k] / lam[k];
            Gp[a * m + b] = s;
        }
    for (int i = 0; i < nd; ++i)
        for (int b = 0; b < m; ++b) {
            double s = 0;
            for (int a = 0; a < m; ++a) s += CB[a * nd + i] * Gp[a * m + b];
            CBp[i * m + b] = s;
        }
    free(G); free(Q); free(lam); free(Gp);
}

/* ------------------------------------------------------------------------ */
/* Per-step work arrays.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double* phihat;  /* [K][nd] remapped values, eq. remap_advect / eq. 5.4 */
    double* tr;      /* [K][4n] own traces of phihat: left j, right j, bottom i, top i (1D: 2) */
    double* fv;      /* face value at t^{n+1} seen by element: same layout as tr */
    double* vn;      /* face velocity at the element's face points, same layout */
    double* Mt;      /* mass target M^{n+1} */
    double* Et;      /* energy target E^{n+1} (sum W phi^2) */
    double* Ec;      /* energy target of the deviation from cref: sum W (phi - cref)^2 */
    double* cref;    /* the element's mean at t^n, M^n / sum W */
} work;

static int ntr(const ctx* c) { return c->p->dim == 1 ? 2 : 4 * c->n; }

/* whether the left/right (x) and bottom/top (y) sides of the domain wrap
 * around to each other (otherwise their faces take ghost values) */
static int periodic_x(const ora_params* p) { return p->bc == 0 || p->bc == 2; }
static int periodic_y(const ora_params* p) { return p->bc == 0 || p->bc == 3; }

/* element neighbours; -1 = outside (ghost) */
static int nb_left(const ctx* c, int e)
{
    const ora_params* p = c->p;
    int ex = e % p->kx, ey = e / p->kx;
    if (ex > 0) return e - 1;
    return periodic_x(p) ? ey * p->kx + p->kx - 1 : -1;
}
static int nb_right(const ctx* c, int e)
{
    const ora_params* p = c->p;
    int ex = e % p->kx, ey = e / p->kx;
    if (ex < p->kx - 1) return e + 1;
    return periodic_x(p) ? ey * p->kx : -1;
}
static int nb_down(const ctx* c, int e)
{
    const ora_params* p = c->p;
    int ex = e % p->kx, ey = e / p->kx;
    if (ey > 0) return e - p->kx;
    return periodic_y(p) ? (p->ky - 1) * p->kx + ex : -1;
}
static int nb_up(const ctx* c, int e)
{
    const ora_params* p = c->p;
    int ex = e % p->kx, ey = e / p->kx;
    if (ey < p->ky - 1) return e + p->kx;
    return periodic_y(p) ? ex : -1;
}

/* reference coordinates of trace point t (layout of work.tr) */
static void trace_point(const ctx* c, int t, double* s, double* r)
{
    int n = c->n;
    if (c->p->dim == 1) { *s = (t == 0) ? 0.0 : 1.0; *r = 0; return; }
    int side = t / n, k = t % n;
    switch (side) {
    case 0: *s = 0; *r = c->xi[k]; break;
    case 1: *s = 1; *r = c->xi[k]; break;
    case 2: *s = c->xi[k]; *r = 0; break;
    default: *s = c->xi[k]; *r = 1; break;
    }
}

/* For trace point t of element e: the neighbour across that face, the
 * matching trace point index in the neighbour, and the ghost index (when the
 * neighbour is outside).  'low' tells whether e sits on the high side of the
 * face (its left/bottom face), so that the neighbour is the low side. */
static void face_partner(const ctx* c, int e, int t, int* nbe, int* nbt, int* gidx, int* e_is_high)
{
    const ora_params* p = c->p;
    int n = c->n;
    int ex = e % p->kx, ey = e / p->kx;
    if (p->dim == 1) {
        if (t == 0) { *nbe = nb_left(c, e); *nbt = 1; *gidx = 0; *e_is_high = 1; }
        else { *nbe = nb_right(c, e); *nbt = 0; *gidx = 1; *e_is_high = 0; }
        return;
    }
    int side = t / n, k = t % n;
    int KL = p->ky * n, KB = p->kx * n;
    switch (side) {
    case 0: *nbe = nb_left(c, e); *nbt = 1 * n + k; *gidx = ey * n + k; *e_is_high = 1; break;
    case 1: *nbe = nb_right(c, e); *nbt = 0 * n + k; *gidx = KL + ey * n + k; *e_is_high = 0; break;
    case 2: *nbe = nb_down(c, e); *nbt = 3 * n + k; *gidx = 2 * KL + ex * n + k; *e_is_high = 1; break;
    default: *nbe = nb_up(c, e); *nbt = 2 * n + k; *gidx = 2 * KL + KB + ex * n + k; *e_is_high = 0; break;
    }
}

/* face-normal velocity component of element e at its trace point t */
static double vel_normal(const ctx* c, int e, int t)
{
    double s, r, u, v, dv;
    trace_point(c, t, &s, &r);
    vel_eval(c, e, s, r, &u, &v, &dv);
    if (c->p->dim == 1) return u;
    return (t / c->n) < 2 ? u : v;
}

/* ------------------------------------------------------------------------ */
/* Phase 1: seed, advect and remap one element (sections 4.1-4.3; the 2D    */
/* scheme, eq. 5.1 and eq. 5.4).  Particles start at the fixed nodes, move  */
/* with one RK step of length dt, and the polynomial through the moved     */
/* points is brought back to the fixed nodes by solving V* phihat = phi*   */
/* with V*_{p,q} = H_q(moved point p) -- identical in exact arithmetic to  */
/* evaluating the moved-point Lagrange interpolant at the fixed nodes.     */
/* ------------------------------------------------------------------------ */
static double face_velocity(const ctx* c, int e, int t);
static void face_partner(const ctx* c, int e, int t, int* nbe, int* nbt, int* gidx, int* e_is_high);

static int advect_remap(const ctx* c, int e, const double* phin, work* W)
{
    int n = c->n, nd = c->nd, d2 = (c->p->dim == 2);
    int flags = 0;
    double* V = malloc(sizeof(double) * nd * nd);
    double* rhs = malloc(sizeof(double) * nd);
    double ls[64], lr[64];
    for (int jj = 0; jj < (d2 ? n : 1); ++jj)
        for (int ii = 0; ii < n; ++ii) {
            int pidx = ii + n * jj;
            double s = c->xi[ii], r = d2 ? c->xi[jj] : 0.0;
            double q = phin[(size_t)e * nd + pidx];
            if (rk_move(c, e, +1, c->dt, &s, &r, &q)) flags |= F_CONTAIN;
            rhs[pidx] = q; /* phi* at the moved particle */
            lag_basis(n, c->xi, s, ls);
            if (d2) lag_basis(n, c->xi, r, lr);
            for (int mm = 0; mm < (d2 ? n : 1); ++mm)
                for (int ll = 0; ll < n; ++ll)
                    V[pidx * nd + ll + n * mm] = ls[ll] * (d2 ? lr[mm] : 1.0);
        }
    if (lu_solve(nd, V, rhs, 1)) flags |= F_SINGULAR;
    double* ph = W->phihat + (size_t)e * nd;
    for (int i = 0; i < nd; ++i) ph[i] = rhs[i];
    /* own traces of the remapped polynomial (eq. remap_bnd; 2D: eq.
     * 2dx_bnd_interpolate and eq. 2dy_bnd_interpolate) */
    double* tr = W->tr + (size_t)e * ntr(c);
    for (int t = 0; t < ntr(c); ++t) {
        double s, r;
        trace_point(c, t, &s, &r);
        tr[t] = field_eval(c, ph, s, r);
    }
    /* Backtracking interface values (eq. 4.11): the characteristic through
     * the trace point is traced back over dt with the particles' RK tableau,
     * and phi^n of this element is evaluated at its foot (times the source
     * factor in the conservative form).  Computed where this element is the
     * upwind side of the face (both sides where the face velocity vanishes);
     * elsewhere the upwind rule (eq. 4.12a) never selects this element's value,
     * and the interpolated one stays. */
    if (c->p->iface == 1) {
        for (int t = 0; t < ntr(c); ++t) {
            int nbe, nbt, gidx, high;
            face_partner(c, e, t, &nbe, &nbt, &gidx, &high);
            double vn = face_velocity(c, e, t);
            int up = high ? (vn <= 0) : (vn >= 0);
            if (!up) continue;
            double s, r;
            trace_point(c, t, &s, &r);
            tr[t] = backtrace_value(c, e, phin, c->dt, s, r, &flags);
        }
    }
    free(V); free(rhs);
    return flags;
}

/* quadrature weight of the element's trace point t on its face (physical) */
static double face_weight(const ctx* c, int t)
{
    if (c->p->dim == 1) return 1.0;
    int side = t / c->n, k = t % c->n;
    return (side < 2 ? c->dy : c->dx) * c->w[k];
}

static double ghost_value(const double* ghost, int gidx) { return ghost ? ghost[gidx] : 0.0; }

/* ghost value at t^n + c dt: linear in time between the rows for t^n and
 * t^{n+1} (reading: the paper gives ghost values only as boundary data) */
static double ghost_at(const double* g_now, const double* g_next, int gidx, double cfrac)
{
    return (1.0 - cfrac) * ghost_value(g_now, gidx) + cfrac * ghost_value(g_next, gidx);
}

/* Face velocity and the low/high sides of the face through trace point t of
 * element e.  Reading: the face velocity is the mean of the two sides'
 * interpolants (interior side only at a ghost boundary). */
static double face_velocity(const ctx* c, int e, int t)
{
    int nbe, nbt, gidx, high;
    face_partner(c, e, t, &nbe, &nbt, &gidx, &high);
    double mine = vel_normal(c, e, t);
    double v = (nbe < 0) ? mine : 0.5 * (mine + vel_normal(c, nbe, nbt));
    /* reading: a face speed at rounding level (a stagnation point) has no
     * upwind side; it is treated as zero, i.e. the mean of both traces */
    return fabs(v) <= c->vzero ? 0.0 : v;
}

/* ------------------------------------------------------------------------ */
/* Phase 2a: unique upwind face values at t^{n+1} seen by element e         */
/* (eq. 4.12a; ghost values at the domain boundary).                        */
/* ------------------------------------------------------------------------ */
static void face_values(const ctx* c, int e, const double* ghost, work* W)
{
    int nt = ntr(c);
    for (int t = 0; t < nt; ++t) {
        int nbe, nbt, gidx, high;
        face_partner(c, e, t, &nbe, &nbt, &gidx, &high);
        double vn = face_velocity(c, e, t);
        double mine = W->tr[(size_t)e * nt + t];
        double other = (nbe >= 0) ? W->tr[(size_t)nbe * nt + nbt] : ghost_value(ghost, gidx);
        /* e is the high side (its left/bottom face): low side = other */
        double lo = high ? other : mine, hi = high ? mine : other;
        W->fv[(size_t)e * nt + t] = upwind(vn, lo, hi);
        W->vn[(size_t)e * nt + t] = vn;
    }
}

/* ------------------------------------------------------------------------ */
/* Phase 2b: mass and energy targets (section "Mass and Energy              */
/* Conservation", eq. 4.14, eq. quad, eq. remap_mass, eq. remap_energy).    */
/* Reading: the balance laws dM/dt = inflow - outflow (+ volume term) are   */
/* integrated over dt with the quadrature of the RK tableau; stage values   */
/* at time t^n + c dt come from backtracking over c dt (eq. 4.11) in the    */
/* upwind element; with c = 0 and Euler this is the paper's first-order     */
/* update exactly.                                                          */
/*                                                                          */
/* Reading (energy): the balance law is taken for the deviation psi =       */
/* phi - c from the element's mean c = M^n / sum W, held fixed over the     */
/* step.  In the advective form psi obeys the same transport equation as    */
/* phi, so d/dt int psi^2 = inflow - outflow of psi^2 + int (div a) psi^2;  */
/* in the conservative form psi_t + div(a psi) = -c div a, which gives the  */
/* volume term -int (div a)(psi^2 + 2 c psi).  For the PDE this is the same */
/* law as the one for phi^2.  Discretely the two differ by c^2 dt times the */
/* element's divergence defect (net face inflow speed + int div a, zero by  */
/* the divergence theorem), a rounding-level quantity for a resolved        */
/* velocity that the phi^2 form would multiply by the field's square and    */
/* that a near-constant element's energy row amplifies without bound.  The  */
/* energy target is E^{n+1} = Ec + 2 c M^{n+1} - c^2 sum W, where Ec is the  */
/* deviation target; Ec itself is what HARD imposes next to a mass row.     */
/* ------------------------------------------------------------------------ */
static int targets(const ctx* c, int e, const double* phin, const double* ghost, const double* ghost_next,
                   work* W)
{
    const ora_params* p = c->p;
    int n = c->n, nd = c->nd, d2 = (p->dim == 2), nt = ntr(c), flags = 0;
    double cu[4], bu[4];
    int nq = rk_nodes(&c->T, cu, bu);
    const double* ph = phin + (size_t)e * nd;
    double M = 0, SW = 0;
    for (int jj = 0; jj < (d2 ? n : 1); ++jj)
        for (int ii = 0; ii < n; ++ii) {
            int pidx = ii + n * jj;
            double Wp = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
            M += Wp * ph[pidx];
            SW += Wp;
        }
    const double cr = M / SW;
    double Ed = 0;
    for (int jj = 0; jj < (d2 ? n : 1); ++jj)
        for (int ii = 0; ii < n; ++ii) {
            int pidx = ii + n * jj;
            double Wp = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
            Ed += Wp * (ph[pidx] - cr) * (ph[pidx] - cr);
        }
    double dM = 0, dE = 0;
    for (int q = 0; q < nq; ++q) {
        double h = cu[q] * c->dt;
        double fM = 0, fE = 0;
        for (int t = 0; t < nt; ++t) {
            int nbe, nbt, gidx, high;
            face_partner(c, e, t, &nbe, &nbt, &gidx, &high);
            double vn = face_velocity(c, e, t);
            /* only the upwind side is traced (both when vn == 0) */
            int use_lo = (vn >= 0), use_hi = (vn <= 0);
            double lo = 0, hi = 0, s, r;
            int lo_e = high ? nbe : e, hi_e = high ? e : nbe;
            int lo_t = high ? nbt : t, hi_t = high ? t : nbt;
            if (use_lo) {
                if (lo_e >= 0) { trace_point(c, lo_t, &s, &r); lo = backtrace_value(c, lo_e, phin, h, s, r, &flags); }
                else lo = ghost_at(ghost, ghost_next, gidx, cu[q]);
            }
            if (use_hi) {
                if (hi_e >= 0) { trace_point(c, hi_t, &s, &r); hi = backtrace_value(c, hi_e, phin, h, s, r, &flags); }
                else hi = ghost_at(ghost, ghost_next, gidx, cu[q]);
            }
            double val = upwind(vn, lo, hi);
            double sign = high ? 1.0 : -1.0; /* inflow positive */
            double fw = face_weight(c, t);
            fM += sign * vn * val * fw;
            fE += sign * vn * (val - cr) * (val - cr) * fw;
        }
        double vM = 0, vE = 0;
        for (int jj = 0; jj < (d2 ? n : 1); ++jj)
            for (int ii = 0; ii < n; ++ii) {
                int pidx = ii + n * jj;
                double Wp = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
                double s = c->xi[ii], r = d2 ? c->xi[jj] : 0.0, u, v, dv;
                if (p->vel_kind == 0) dv = c->div[(size_t)e * nd + pidx];
                else vel_eval(c, e, s, r, &u, &v, &dv);
                if (dv == 0.0) continue;
                double val = backtrace_value(c, e, phin, h, s, r, &flags);
                double dev = val - cr;
                vM += Wp * dv * val;
                /* advective: + int (div a) psi^2; conservative: - int (div a)(psi^2 + 2 c psi) */
                vE += Wp * dv * (p->form == 0 ? dev * dev : -(dev * dev + 2.0 * cr * dev));
            }
        double RM = fM + (p->form == 0 ? vM : 0.0);
        double RE = fE + vE;
        dM += bu[q] * RM;
        dE += bu[q] * RE;
    }
    W->Mt[e] = M + c->dt * dM;
    W->Ec[e] = Ed + c->dt * dE;
    W->cref[e] = cr;
    W->Et[e] = W->Ec[e] + 2.0 * cr * W->Mt[e] - cr * cr * SW;
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Phase 3: constrained least squares for one element.                      */
/* ------------------------------------------------------------------------ */
typedef struct { double rb, rm, re; int picard, flags; } cls_out;

/* rows of element e other than the 2D boundary block: boundary (1D), mass,
 * energy (with linearisation point prev).  Returns the number of rows. */
static int assemble_rows(const ctx* c, int e, const work* W, const double* prev, int with_energy,
                         int with_boundary, double* C, double* d)
{
    const ora_params* p = c->p;
    int n = c->n, nd = c->nd, d2 = (p->dim == 2), m = 0;
    if (with_boundary && !d2) {
        for (int i = 0; i < n; ++i) { C[m * nd + i] = c->l0[i]; C[(m + 1) * nd + i] = c->l1[i]; }
        d[m] = W->fv[(size_t)e * 2 + 0];
        d[m + 1] = W->fv[(size_t)e * 2 + 1];
        m += 2;
    }
    if (p->cmask & C_MASS) {
        for (int jj = 0; jj < (d2 ? n : 1); ++jj)
            for (int ii = 0; ii < n; ++ii)
                C[m * nd + ii + n * jj] = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
        d[m] = W->Mt[e];
        ++m;
    }
    if (with_energy) {
        /* the paper's linearised energy row sum W phi^(k-1) phi = E^{n+1}
         * (used by SOFT; HARD imposes the energy row in constrain()) */
        for (int jj = 0; jj < (d2 ? n : 1); ++jj)
            for (int ii = 0; ii < n; ++ii) {
                int pidx = ii + n * jj;
                C[m * nd + pidx] = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0) * prev[pidx];
            }
        d[m] = W->Et[e];
        ++m;
    }
    return m;
}

/* one solve with the current rows; 2D HARD uses the boundary pseudo-inverse
 * first and then imposes the remaining rows inside the null space of C_B */
static int solve_once(const ctx* c, int e, const work* W, const double* CB, const double* CBp,
                      const double* PB, const double* prev, int with_energy, double* out)
{
    const ora_params* p = c->p;
    int n = c->n, nd = c->nd, d2 = (p->dim == 2), bound = (p->cmask & C_BOUND) != 0;
    const double* ph = W->phihat + (size_t)e * nd;
    double C[4 * 256]; /* at most 4 rows of at most 256 nodes */
    double d[8];
    int bad = 0;
    if (!d2) {
        int m = assemble_rows(c, e, W, prev, with_energy, bound, C, d);
        if (m == 0) { memcpy(out, ph, sizeof(double) * nd); return 0; }
        return cls_solve(nd, m, C, d, ph, p->mode, out);
    }
    /* 2D */
    if (p->mode == 1) { /* SOFT: stack everything (eq. matrix_a) */
        int mb = bound ? 4 * n : 0;
        double* Cs = malloc(sizeof(double) * (mb + 2) * nd);
        double* ds = malloc(sizeof(double) * (mb + 2));
        if (bound) {
            memcpy(Cs, CB, sizeof(double) * mb * nd);
            for (int t = 0; t < mb; ++t) ds[t] = W->fv[(size_t)e * mb + t];
        }
        int m2 = assemble_rows(c, e, W, prev, with_energy, 0, Cs + (size_t)mb * nd, ds + mb);
        bad = cls_solve(nd, mb + m2, Cs, ds, ph, 1, out);
        free(Cs); free(ds);
        return bad;
    }
    /* HARD, prioritised: phi1 = phihat + C_B^+ (d_B - C_B phihat) */
    double* phi1 = malloc(sizeof(double) * nd);
    memcpy(phi1, ph, sizeof(double) * nd);
    if (bound) {
        int mb = 4 * n;
        double rb[256];
        for (int t = 0; t < mb; ++t) {
            double s = 0;
            for (int i = 0; i < nd; ++i) s += CB[t * nd + i] * ph[i];
            rb[t] = W->fv[(size_t)e * mb + t] - s;
        }
        for (int i = 0; i < nd; ++i) {
            double s = 0;
            for (int t = 0; t < mb; ++t) s += CBp[i * mb + t] * rb[t];
            phi1[i] += s;
        }
    }
    int m2 = assemble_rows(c, e, W, prev, with_energy, 0, C, d);
    if (m2 == 0) { memcpy(out, phi1, sizeof(double) * nd); free(phi1); return 0; }
    /* G = C^T (nd x m2); PG = P_B G; solve (G^T P_B G) y = G^T phi1 - h */
    double* PG = malloc(sizeof(double) * nd * m2);
    for (int r = 0; r < m2; ++r)
        for (int i = 0; i < nd; ++i) {
            double s = 0;
            if (bound) for (int k = 0; k < nd; ++k) s += PB[i * nd + k] * C[r * nd + k];
            else s = C[r * nd + i];
            PG[i * m2 + r] = s;
        }
    double S[4], y[2];
    for (int a = 0; a < m2; ++a) {
        for (int b = 0; b < m2; ++b) {
            double s = 0;
            for (int i = 0; i < nd; ++i) s += C[a * nd + i] * PG[i * m2 + b];
            S[a * m2 + b] = s;
        }
        double g = 0;
        for (int i = 0; i < nd; ++i) g += C[a * nd + i] * phi1[i];
        y[a] = g - d[a];
    }
    bad = lu_solve(m2, S, y, 1);
    for (int i = 0; i < nd; ++i) {
        double s = 0;
        for (int r = 0; r < m2; ++r) s += PG[i * m2 + r] * y[r];
        out[i] = phi1[i] - s;
    }
    free(PG); free(phi1);
    return bad;
}

/* Orthonormal basis of the span of the rows of R (m x nd) by modified
 * Gram-Schmidt, applied twice per row; a row whose remainder falls below
 * 1e-10 of its own norm depends on the earlier ones and is dropped.  Returns
 * the number of basis vectors written to Q (rank x nd). */
static int row_basis(int m, int nd, const double* R, double* Q)
{
    int k = 0;
    for (int r = 0; r < m; ++r) {
        double* q = Q + (size_t)k * nd;
        double n0 = 0, n1 = 0;
        for (int i = 0; i < nd; ++i) { q[i] = R[(size_t)r * nd + i]; n0 += q[i] * q[i]; }
        for (int pass = 0; pass < 2; ++pass)
            for (int b = 0; b < k; ++b) {
                const double* qb = Q + (size_t)b * nd;
                double s = 0;
                for (int i = 0; i < nd; ++i) s += qb[i] * q[i];
                for (int i = 0; i < nd; ++i) q[i] -= s * qb[i];
            }
        for (int i = 0; i < nd; ++i) n1 += q[i] * q[i];
        if (n1 <= 1e-20 * n0 || n1 == 0.0) continue;
        n1 = sqrt(n1);
        for (int i = 0; i < nd; ++i) q[i] /= n1;
        ++k;
    }
    return k;
}

/* HARD energy row (section "Local energy conservation", eq. remap_energy).
 * Reading: the paper's fixed-point iteration sum W phi^(k-1) phi^(k) = E
 * is kept as the definition of the result -- its fixed point is the point
 * of the constraint set {linear rows, sum W phi^2 = E} nearest phihat (the
 * KKT point of the quadratic row) -- but under HARD that map is 2-periodic
 * (it sends the no-energy solution phi1 to a point phi2 and phi2 back to
 * phi1, because sum W phi2 phi1 = E holds by construction).  The fixed point
 * is reached instead by Newton's linearisation of the same row,
 *   2 sum W y^(k-1) y = T + sum W (y^(k-1))^2,
 * i.e. the paper's row with its target replaced by the mean of T and the
 * current energy; each sweep is the nearest point to phihat (equivalently
 * to phi1, the solution without the energy row) that satisfies the linear
 * rows and the linearised one.  A fixed point of the sweep satisfies the
 * energy row exactly and is stationary for the distance, so it is the
 * paper's fixed point.  y = phi - s: with a mass row the row is written for
 * the deviation from the element's mean (s = cref, T = Ec), the same
 * constraint set on the mass row's level set, and computed from differences
 * of like size; without a mass row s = 0 and T = E^{n+1}.  Stop when
 * max |y^(k) - y^(k-1)| < tol (strict, as printed), y^(0) = y1.
 *   linear rows: 1D l(0), l(1) (boundary), W (mass); 2D C_B, W.
 * Returns the number of sweeps; *conv set when the stop rule was met;
 * *sing set when the linearised row lies in the span of the linear rows
 * (no correction possible) while the energy is not met. */
static int energy_newton_core(int nd, int m, const double* R, const double* Wq, double s, double T,
                              const double* phi1, double tol, int maxit, double* out, int* conv, int* sing)
{
    double* Q = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * nd);
    double* y1 = malloc(sizeof(double) * nd);
    double* y = malloc(sizeof(double) * nd);
    double* g = malloc(sizeof(double) * nd);
    int rank = row_basis(m, nd, R, Q);
    for (int i = 0; i < nd; ++i) { y1[i] = phi1[i] - s; y[i] = y1[i]; }
    int k = 0;
    *conv = 0;
    *sing = 0;
    for (k = 1; k <= maxit; ++k) {
        /* gradient direction w = W y (half the gradient of sum W y^2),
         * projected onto the null space of the linear rows (twice) */
        double en = 0;
        for (int i = 0; i < nd; ++i) { g[i] = Wq[i] * y[i]; en += Wq[i] * y[i] * y[i]; }
        double wy1 = 0;
        for (int i = 0; i < nd; ++i) wy1 += g[i] * y1[i];
        for (int pass = 0; pass < 2; ++pass)
            for (int b = 0; b < rank; ++b) {
                const double* qb = Q + (size_t)b * nd;
                double t = 0;
                for (int i = 0; i < nd; ++i) t += qb[i] * g[i];
                for (int i = 0; i < nd; ++i) g[i] -= t * qb[i];
            }
        double gg = 0;
        for (int i = 0; i < nd; ++i) gg += g[i] * g[i];
        const double rhs = 0.5 * (T + en) - wy1; /* w.(y - y1) required */
        double diff = 0;
        if (gg > 0.0) {
            const double a = rhs / gg;
            for (int i = 0; i < nd; ++i) {
                double nv = y1[i] + a * g[i];
                diff = fmax(diff, fabs(nv - y[i]));
                y[i] = nv;
            }
        } else if (rhs != 0.0) {
            *sing = 1;
        }
        if (diff < tol) { *conv = 1; break; }
    }
    if (k > maxit) k = maxit;
    for (int i = 0; i < nd; ++i) out[i] = y[i] + s;
    free(Q); free(y1); free(y); free(g);
    return k;
}

/* the element's linear rows and weights for energy_newton_core */
static int energy_newton(const ctx* c, int e, const work* W, const double* CB, const double* phi1, double* out,
                         int* conv, int* sing)
{
    const ora_params* p = c->p;
    int n = c->n, nd = c->nd, d2 = (p->dim == 2);
    int bound = (p->cmask & C_BOUND) != 0, mass = (p->cmask & C_MASS) != 0;
    int mr = (bound ? (d2 ? 4 * n : 2) : 0) + (mass ? 1 : 0);
    double* R = malloc(sizeof(double) * (size_t)(mr > 0 ? mr : 1) * nd);
    double* Wq = malloc(sizeof(double) * nd);
    for (int jj = 0; jj < (d2 ? n : 1); ++jj)
        for (int ii = 0; ii < n; ++ii) Wq[ii + n * jj] = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
    int m = 0;
    if (bound) {
        if (d2) { memcpy(R, CB, sizeof(double) * 4 * n * nd); m = 4 * n; }
        else {
            for (int i = 0; i < nd; ++i) { R[i] = c->l0[i]; R[nd + i] = c->l1[i]; }
            m = 2;
        }
    }
    if (mass) { memcpy(R + (size_t)m * nd, Wq, sizeof(double) * nd); ++m; }
    const double s = mass ? W->cref[e] : 0.0;
    const double T = mass ? W->Ec[e] : W->Et[e];
    int k = energy_newton_core(nd, m, R, Wq, s, T, phi1, p->energy_tol, p->energy_maxit, out, conv, sing);
    free(R); free(Wq);
    return k;
}

static cls_out constrain(const ctx* c, int e, const work* W, const double* CB, const double* CBp,
                         const double* PB, double* out)
{
    const ora_params* p = c->p;
    int n = c->n, nd = c->nd, d2 = (p->dim == 2);
    cls_out o = {0, 0, 0, 0, 0};
    double* prev = malloc(sizeof(double) * nd);
    double* cur = malloc(sizeof(double) * nd);
    if (solve_once(c, e, W, CB, CBp, PB, NULL, 0, prev)) o.flags |= F_SINGULAR;
    if ((p->cmask & C_ENERGY) && p->mode == 0) {
        int conv, sing;
        o.picard = energy_newton(c, e, W, CB, prev, cur, &conv, &sing);
        memcpy(prev, cur, sizeof(double) * nd);
        if (sing) o.flags |= F_SINGULAR;
        if (!conv && p->energy_tol > 0) o.flags |= F_NOCONV;
    } else if (p->cmask & C_ENERGY) {
        /* SOFT: Picard on the paper's linearised energy row (section "Local
         * energy conservation"), stacked with the other rows; stop when the
         * change is below tol (strict, as printed) */
        int conv = 0;
        for (int k = 1; k <= p->energy_maxit; ++k) {
            if (solve_once(c, e, W, CB, CBp, PB, prev, 1, cur)) o.flags |= F_SINGULAR;
            double diff = 0;
            for (int i = 0; i < nd; ++i) diff = fmax(diff, fabs(cur[i] - prev[i]));
            memcpy(prev, cur, sizeof(double) * nd);
            o.picard = k;
            if (diff < p->energy_tol) { conv = 1; break; }
        }
        if (!conv && p->energy_tol > 0) o.flags |= F_NOCONV;
    }
    memcpy(out, prev, sizeof(double) * nd);
    /* residuals */
    int nt = ntr(c);
    if (p->cmask & C_BOUND) {
        for (int t = 0; t < nt; ++t) {
            double s, r;
            trace_point(c, t, &s, &r);
            double v = field_eval(c, out, s, r);
            o.rb = fmax(o.rb, fabs(v - W->fv[(size_t)e * nt + t]));
        }
    }
    /* energy residual of the row as imposed: HARD with a mass row in the
     * deviation form, otherwise sum W phi^2 against E^{n+1} */
    const int dev = (p->mode == 0) && (p->cmask & C_MASS);
    const double s0 = dev ? W->cref[e] : 0.0;
    double M = 0, E = 0;
    for (int jj = 0; jj < (d2 ? n : 1); ++jj)
        for (int ii = 0; ii < n; ++ii) {
            double Wp = c->dx * c->w[ii] * (d2 ? c->dy * c->w[jj] : 1.0);
            double v = out[ii + n * jj];
            M += Wp * v;
            E += Wp * (v - s0) * (v - s0);
        }
    if (p->cmask & C_MASS) o.rm = fabs(M - W->Mt[e]);
    if (p->cmask & C_ENERGY) o.re = fabs(E - (dev ? W->Ec[e] : W->Et[e]));
    free(prev); free(cur);
    return o;
}

/* ------------------------------------------------------------------------ */
/* Driver: nsteps steps of length dt.                                        */
/*   a      nodal velocity, component-major [dim][K][nd] (unused if analytic)*/
/*   div    nodal divergence [K][nd], or NULL for D.a from the interpolant   */
/*   ghost  ghost rows [ghost_rows][nghost] (NULL if periodic): row i holds  */
/*          the outside values at t0 + i dt; step i reads rows i and i+1    */
/*          (clamped).  1D: [left, right]; 2D: left (ky*n), right (ky*n),    */
/*          bottom (kx*n), top (kx*n)                                        */
/*   phi    in: phi^n [K][nd]; out: phi^{n+nsteps}                          */
/*   want   optional element mask (nsteps must be 1): only these elements   */
/*          are written; the others keep their input values                 */
/* Returns 0, or 1 on invalid parameters.                                    */
/* ------------------------------------------------------------------------ */
int ora_ghost_count(const ora_params* p)
{
    if (p->dim == 1) return 2;
    return 2 * p->ky * p->n + 2 * p->kx * p->n;
}

int ora_step(const ora_params* p, const double* a, const double* div, const double* ghost, int ghost_rows,
             double dt, int nsteps, double* phi, const uint8_t* want, ora_stats* st)
{
    if (p->dim != 1 && p->dim != 2) return 1;
    if (p->n < 1 || p->n > (p->dim == 1 ? 64 : 17)) return 1;
    if (p->kx < 1 || p->ky < 1 || (p->dim == 1 && p->ky != 1)) return 1;
    if (p->bc < 0 || p->bc > (p->dim == 1 ? 1 : 3)) return 1;
    if (want && nsteps != 1) return 1;
    /* 2D HARD: the rows after the boundary block are imposed inside
     * null(C_B), of dimension (n-2)^2 since C_B has rank 4n-4; more rows
     * than that cannot all hold, so the step is refused (SOFT stacks them
     * and is always defined) */
    if (p->dim == 2 && p->mode == 0 && (p->cmask & C_BOUND)) {
        int extra = ((p->cmask & C_MASS) != 0) + ((p->cmask & C_ENERGY) != 0);
        if (extra > (p->n - 2) * (p->n - 2)) return 1;
    }
    ctx c;
    memset(&c, 0, sizeof(c));
    c.p = p;
    c.n = p->n;
    c.nd = p->dim == 1 ? p->n : p->n * p->n;
    c.K = p->kx * p->ky;
    c.dx = (p->x1 - p->x0) / p->kx;
    c.dy = p->dim == 2 ? (p->y1 - p->y0) / p->ky : 1.0;
    c.dt = dt;
    c.a = a;
    if (ora_nodes(p->family, p->n, c.xi, c.w)) return 1;
    if (rk_tableau(p->rk, &c.T)) return 1;
    lag_basis(c.n, c.xi, 0.0, c.l0);
    lag_basis(c.n, c.xi, 1.0, c.l1);
    int n = c.n, nd = c.nd, K = c.K, nt = ntr(&c);

    /* stagnation threshold: 1e-12 of the largest nodal speed (1e-12 for the
     * analytic fields, whose speeds are of order one) */
    c.vzero = 1e-12;
    if (p->vel_kind == 0) {
        double am = 0;
        for (size_t i = 0; i < (size_t)p->dim * K * nd; ++i) am = fmax(am, fabs(a[i]));
        c.vzero = 1e-12 * am;
    }

    /* nodal divergence: given, or the derivative of the velocity interpolant */
    c.div = malloc(sizeof(double) * (size_t)K * nd);
    if (p->vel_kind == 0) {
        if (div) memcpy(c.div, div, sizeof(double) * (size_t)K * nd);
        else {
            double D[64 * 64];
            for (int i = 0; i < n; ++i) lag_basis_deriv(n, c.xi, c.xi[i], D + i * n);
            for (int e = 0; e < K; ++e)
                for (int jj = 0; jj < (p->dim == 2 ? n : 1); ++jj)
                    for (int ii = 0; ii < n; ++ii) {
                        double s = 0;
                        if (p->dim == 1) {
                            for (int l = 0; l < n; ++l) s += D[ii * n + l] * a[(size_t)e * nd + l];
                            s /= c.dx;
                        } else {
                            const double* au = a + (size_t)e * nd;
                            const double* av = a + (size_t)K * nd + (size_t)e * nd;
                            double sx = 0, sy = 0;
                            for (int l = 0; l < n; ++l) sx += D[ii * n + l] * au[l + n * jj];
                            for (int m = 0; m < n; ++m) sy += D[jj * n + m] * av[ii + n * m];
                            s = sx / c.dx + sy / c.dy;
                        }
                        c.div[(size_t)e * nd + ii + n * jj] = s;
                    }
        }
    } else {
        memset(c.div, 0, sizeof(double) * (size_t)K * nd);
    }

    /* 2D boundary block tables (constant per n) */
    double *CB = NULL, *CBp = NULL, *PB = NULL;
    if (p->dim == 2) {
        CB = malloc(sizeof(double) * 4 * n * nd);
        CBp = malloc(sizeof(double) * 4 * n * nd);
        PB = malloc(sizeof(double) * nd * nd);
        build_CB(&c, CB);
        build_CBpinv(&c, CB, CBp);
        for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nd; ++j) {
                double s = 0;
                for (int t = 0; t < 4 * n; ++t) s += CBp[i * 4 * n + t] * CB[t * nd + j];
                PB[i * nd + j] = (i == j ? 1.0 : 0.0) - s;
            }
    }

    work W;
    W.phihat = malloc(sizeof(double) * (size_t)K * nd);
    W.tr = malloc(sizeof(double) * (size_t)K * nt);
    W.fv = malloc(sizeof(double) * (size_t)K * nt);
    W.vn = malloc(sizeof(double) * (size_t)K * nt);
    W.Mt = calloc((size_t)K, sizeof(double));
    W.Et = calloc((size_t)K, sizeof(double));
    W.Ec = calloc((size_t)K, sizeof(double));
    W.cref = calloc((size_t)K, sizeof(double));
    double* out = malloc(sizeof(double) * (size_t)K * nd);
    uint8_t* need = NULL;
    if (want) {
        /* phase 1 is needed on the wanted elements and their face neighbours */
        need = calloc((size_t)K, 1);
        for (int e = 0; e < K; ++e) {
            if (!want[e]) continue;
            need[e] = 1;
            for (int t = 0; t < nt; ++t) {
                int nbe, nbt, gidx, high;
                face_partner(&c, e, t, &nbe, &nbt, &gidx, &high);
                if (nbe >= 0) need[nbe] = 1;
            }
        }
    }
    int nghost = ora_ghost_count(p);
    ora_stats S;
    memset(&S, 0, sizeof(S));

    for (int step = 0; step < nsteps; ++step) {
        /* ghost rows hold boundary values at t0, t0 + dt, ...; this step runs
         * from row 'step' to row 'step + 1' (both clamped to the last row) */
        const double *g = NULL, *gn = NULL;
        if (p->bc != 0 && ghost) {
            g = ghost + (size_t)nghost * (step < ghost_rows ? step : ghost_rows - 1);
            gn = ghost + (size_t)nghost * (step + 1 < ghost_rows ? step + 1 : ghost_rows - 1);
        }
        int flags = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
        for (int e = 0; e < K; ++e) {
            if (need && !need[e]) continue;
            flags |= advect_remap(&c, e, phi, &W);
        }
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
        for (int e = 0; e < K; ++e) {
            if (want && !want[e]) continue;
            face_values(&c, e, gn, &W);
            if (p->cmask & (C_MASS | C_ENERGY)) flags |= targets(&c, e, phi, g, gn, &W);
        }
        double rb = 0, rm = 0, re = 0;
        int pic = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags) reduction(max : rb, rm, re, pic)
        for (int e = 0; e < K; ++e) {
            if (want && !want[e]) continue;
            cls_out o = constrain(&c, e, &W, CB, CBp, PB, out + (size_t)e * nd);
            flags |= o.flags;
            rb = fmax(rb, o.rb); rm = fmax(rm, o.rm); re = fmax(re, o.re);
            if (o.picard > pic) pic = o.picard;
        }
        for (int e = 0; e < K; ++e) {
            if (want && !want[e]) continue;
            for (int i = 0; i < nd; ++i) {
                double v = out[(size_t)e * nd + i];
                if (!isfinite(v)) flags |= F_NONFINITE;
                phi[(size_t)e * nd + i] = v;
            }
        }
        S.flags |= flags;
        S.resid_boundary = fmax(S.resid_boundary, rb);
        S.resid_mass = fmax(S.resid_mass, rm);
        S.resid_energy = fmax(S.resid_energy, re);
        if (pic > S.max_picard) S.max_picard = pic;
    }
    if (st) *st = S;
    free(c.div); free(CB); free(CBp); free(PB);
    free(W.phihat); free(W.tr); free(W.fv); free(W.vn); free(W.Mt); free(W.Et); free(W.Ec); free(W.cref);
    free(out); free(need);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mixed orders in 2D: every element has its own number of nodes n_e.       */
/*                                                                          */
/* Each element is handled as a one-element mesh with its own box and     */
/* order (a "view"), so the element-local steps above apply unchanged: the */
/* particle motion and the remap of eq. 5.4, the traces, and the boundary  */
/* least squares.  What couples elements of different orders is the face  */
/* value: the upwind side's remapped polynomial is evaluated at this        */
/* element's own edge nodes (reading: the neighbour's edge polynomial       */
/* evaluated at the element's edge points), and the face speed is the mean  */
/* of the two sides' velocity interpolants at the same physical point.     */
/* Periodic meshes, boundary rows only (HARD or SOFT).                      */
/*                                                                          */
/*   orders  [K] nodes per direction of each element, element e = ix+kx*iy  */
/*   a       nodal velocity: all u values (element by element, n_e^2 each,  */
/*           node i + n_e j), then all v values                             */
/*   phi     in/out, element by element (n_e^2 values each)                 */
/* Returns 0, or 1 on invalid parameters.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    ora_params p;   /* the element as a 1x1 mesh */
    ctx c;
    double* au;     /* [2][nd] velocity of the element (u then v) */
    double* div;    /* [nd] */
    double *CB, *CBp, *PB;
} elem_view;

static int view_init(const ora_params* p, int e, int n, const double* a_u, const double* a_v, double dt,
                     double vzero, elem_view* v)
{
    memset(v, 0, sizeof(*v));
    v->p = *p;
    int ex = e % p->kx, ey = e / p->kx;
    double dx = (p->x1 - p->x0) / p->kx, dy = (p->y1 - p->y0) / p->ky;
    v->p.kx = v->p.ky = 1;
    v->p.n = n;
    v->p.x0 = p->x0 + ex * dx;
    v->p.x1 = v->p.x0 + dx;
    v->p.y0 = p->y0 + ey * dy;
    v->p.y1 = v->p.y0 + dy;
    ctx* c = &v->c;
    c->p = &v->p;
    c->n = n;
    c->nd = n * n;
    c->K = 1;
    c->dx = dx;
    c->dy = dy;
    c->dt = dt;
    c->vzero = vzero;
    if (ora_nodes(p->family, n, c->xi, c->w)) return 1;
    if (rk_tableau(p->rk, &c->T)) return 1;
    lag_basis(n, c->xi, 0.0, c->l0);
    lag_basis(n, c->xi, 1.0, c->l1);
    int nd = n * n;
    v->au = malloc(sizeof(double) * 2 * nd);
    v->div = malloc(sizeof(double) * nd);
    if (p->vel_kind == 0) {
        memcpy(v->au, a_u, sizeof(double) * nd);
        memcpy(v->au + nd, a_v, sizeof(double) * nd);
        /* divergence of the velocity interpolant at the nodes */
        double D[64 * 64];
        for (int i = 0; i < n; ++i) lag_basis_deriv(n, c->xi, c->xi[i], D + i * n);
        for (int jj = 0; jj < n; ++jj)
            for (int ii = 0; ii < n; ++ii) {
                double sx = 0, sy = 0;
                for (int l = 0; l < n; ++l) sx += D[ii * n + l] * a_u[l + n * jj];
                for (int m = 0; m < n; ++m) sy += D[jj * n + m] * a_v[ii + n * m];
                v->div[ii + n * jj] = sx / dx + sy / dy;
            }
    } else {
        memset(v->au, 0, sizeof(double) * 2 * nd);
        memset(v->div, 0, sizeof(double) * nd);
    }
    c->a = v->au;
    c->div = v->div;
    v->CB = malloc(sizeof(double) * 4 * n * nd);
    v->CBp = malloc(sizeof(double) * 4 * n * nd);
    v->PB = malloc(sizeof(double) * nd * nd);
    build_CB(c, v->CB);
    build_CBpinv(c, v->CB, v->CBp);
    for (int i = 0; i < nd; ++i)
        for (int j = 0; j < nd; ++j) {
            double sum = 0;
            for (int t = 0; t < 4 * n; ++t) sum += v->CBp[i * 4 * n + t] * v->CB[t * nd + j];
            v->PB[i * nd + j] = (i == j ? 1.0 : 0.0) - sum;
        }
    return 0;
}

static void view_free(elem_view* v)
{
    free(v->au); free(v->div); free(v->CB); free(v->CBp); free(v->PB);
}

/* normal velocity component of view v at its reference point (s, r):
 * u on x-faces (sides 0, 1), v on y-faces */
static double view_normal(const elem_view* v, int side, double s, double r)
{
    double u, w, dv;
    vel_eval(&v->c, 0, s, r, &u, &w, &dv);
    return side < 2 ? u : w;
}

int ora_step_mixed(const ora_params* p, const int32_t* orders, const double* a, double dt, int nsteps,
                   double* phi, ora_stats* st)
{
    /* interpolated interface values only (the backtracking variant is
     * defined here for meshes of one order) */
    if (p->dim != 2 || p->bc != 0 || (p->cmask & ~C_BOUND) || p->kx < 1 || p->ky < 1 || p->iface != 0) return 1;
    int K = p->kx * p->ky;
    size_t* off = malloc(sizeof(size_t) * (K + 1));
    off[0] = 0;
    for (int e = 0; e < K; ++e) {
        if (orders[e] < 2 || orders[e] > 17) { free(off); return 1; }
        off[e + 1] = off[e] + (size_t)orders[e] * orders[e];
    }
    size_t tot = off[K];
    /* stagnation threshold: 1e-12 of the largest nodal speed */
    double vzero = 1e-12;
    if (p->vel_kind == 0) {
        double am = 0;
        for (size_t i = 0; i < 2 * tot; ++i) am = fmax(am, fabs(a[i]));
        vzero = 1e-12 * am;
    }
    elem_view* V = calloc((size_t)K, sizeof(elem_view));
    int bad = 0;
    for (int e = 0; e < K && !bad; ++e)
        bad = view_init(p, e, orders[e], a + off[e], a + tot + off[e], dt, vzero, &V[e]);
    if (bad) {
        for (int e = 0; e < K; ++e) view_free(&V[e]);
        free(V); free(off);
        return 1;
    }
    double* phihat = malloc(sizeof(double) * tot);
    double* tr = malloc(sizeof(double) * 4 * 16 * (size_t)K);   /* each view's own traces */
    double* fv = malloc(sizeof(double) * 4 * 16 * (size_t)K);
    double* out = malloc(sizeof(double) * tot);
    ora_stats S;
    memset(&S, 0, sizeof(S));
    for (int step = 0; step < nsteps; ++step) {
        int flags = 0;
        /* phase 1: seed, move and remap each element in its own view */
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
        for (int e = 0; e < K; ++e) {
            work W;
            memset(&W, 0, sizeof(W));
            W.phihat = phihat + off[e];
            W.tr = tr + (size_t)64 * e;
            flags |= advect_remap(&V[e].c, 0, phi + off[e], &W);
        }
        /* phase 2: face values at each element's own edge points; phase 3:
         * the element's boundary least squares */
        double rb = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags) reduction(max : rb)
        for (int e = 0; e < K; ++e) {
            const elem_view* me = &V[e];
            int n = orders[e], ex = e % p->kx, ey = e / p->kx;
            double* f = fv + (size_t)64 * e;
            for (int t = 0; t < 4 * n; ++t) {
                int side = t / n;
                double s, r;
                trace_point(&me->c, t, &s, &r);
                /* neighbour across the face (periodic) and the same physical
                 * point in its reference frame */
                int nb;
                double s2 = s, r2 = r;
                switch (side) {
                case 0: nb = ey * p->kx + (ex + p->kx - 1) % p->kx; s2 = 1.0; break;
                case 1: nb = ey * p->kx + (ex + 1) % p->kx; s2 = 0.0; break;
                case 2: nb = ((ey + p->ky - 1) % p->ky) * p->kx + ex; r2 = 1.0; break;
                default: nb = ((ey + 1) % p->ky) * p->kx + ex; r2 = 0.0; break;
                }
                const elem_view* ot = &V[nb];
                double v = 0.5 * (view_normal(me, side, s, r) + view_normal(ot, side, s2, r2));
                if (fabs(v) <= vzero) v = 0.0;
                double mine = field_eval(&me->c, phihat + off[e], s, r);
                double other = field_eval(&ot->c, phihat + off[nb], s2, r2);
                int high = (side == 0 || side == 2);
                f[t] = upwind(v, high ? other : mine, high ? mine : other);
            }
            work W;
            memset(&W, 0, sizeof(W));
            W.phihat = phihat + off[e];
            W.fv = f;
            cls_out o = constrain(&me->c, 0, &W, me->CB, me->CBp, me->PB, out + off[e]);
            flags |= o.flags;
            rb = fmax(rb, o.rb);
        }
        for (size_t i = 0; i < tot; ++i) {
            if (!isfinite(out[i])) flags |= F_NONFINITE;
            phi[i] = out[i];
        }
        S.flags |= flags;
        S.resid_boundary = fmax(S.resid_boundary, rb);
    }
    if (st) *st = S;
    for (int e = 0; e < K; ++e) view_free(&V[e]);
    free(V); free(off); free(phihat); free(tr); free(fv); free(out);
    return 0;
}

/* Exposed pieces for unit tests of the oracle itself. */
int ora_rk_tableau(int id, int* s, double* a16, double* b4, double* c4)
{
    tableau T;
    if (rk_tableau(id, &T)) return 1;
    *s = T.s;
    for (int i = 0; i < 4; ++i) {
        b4[i] = T.b[i];
        c4[i] = T.c[i];
        for (int j = 0; j < 4; ++j) a16[i * 4 + j] = T.a[i][j];
    }
    return 0;
}

int ora_cls(int nd, int m, const double* C, const double* d, const double* phihat, int mode, double* phi)
{
    return cls_solve(nd, m, C, d, phihat, mode, phi);
}

/* HARD least squares with one quadratic row (the energy row as imposed by
 * constrain()): min ||phi - phihat|| s.t. C phi = d (m x nd, full row rank)
 * and sum_i Wq_i (phi_i - s)^2 = T, by the LSE solution of the linear rows
 * followed by energy_newton_core.  Returns the sweep count; flags get
 * F_NOCONV (tol > 0, not met) and F_SINGULAR. */
int ora_energy_hard(int nd, int m, const double* C, const double* d, const double* Wq, double s, double T,
                    const double* phihat, double tol, int maxit, double* phi, int* flags)
{
    double* phi1 = malloc(sizeof(double) * nd);
    int conv, sing;
    *flags = 0;
    if (m > 0) {
        if (cls_solve(nd, m, C, d, phihat, 0, phi1)) *flags |= F_SINGULAR;
    } else {
        memcpy(phi1, phihat, sizeof(double) * nd);
    }
    int k = energy_newton_core(nd, m, C, Wq, s, T, phi1, tol, maxit, phi, &conv, &sing);
    if (sing) *flags |= F_SINGULAR;
    if (!conv && tol > 0) *flags |= F_NOCONV;
    free(phi1);
    return k;
}

int ora_boundary_pinv(int family, int n, double* CB, double* CBp)
{
    ora_params p;
    memset(&p, 0, sizeof(p));
    p.dim = 2; p.n = n; p.family = family;
    ctx c;
    memset(&c, 0, sizeof(c));
    c.p = &p; c.n = n; c.nd = n * n;
    if (ora_nodes(family, n, c.xi, c.w)) return 1;
    lag_basis(n, c.xi, 0.0, c.l0);
    lag_basis(n, c.xi, 1.0, c.l1);
    build_CB(&c, CB);
    build_CBpinv(&c, CB, CBp);
    return 0;
}
