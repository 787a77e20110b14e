// Reference-element tables of the semi-Lagrangian step (host, FP64).
//
// Node families on the reference interval [0,1] (paper section 3):
//   - Gauss-Legendre: roots of P_n located by bisection on the Sturm
//     sequence of the Legendre three-term recurrence, then polished by two
//     Newton steps; weights 1/((1 - t^2) P_n'(t)^2) on [0,1].
//   - Chebyshev-Gauss: the closed form of eq. gaussquad with n = N + 1
//     points, xi_j = (1 - cos((j + 1/2) pi / n)) / 2; weights are the
//     integrals of the Lagrange basis, obtained through the Chebyshev
//     expansion of each basis polynomial.
// Derived tables (all per node family and n):
//   - barycentric weights lambda_j = 1 / prod_{m != j} (xi_j - xi_m),
//   - l_j(0), l_j(1): the basis at the element edges (eq. remap_bnd),
//   - D_ij = l_j'(xi_i): derivative of the interpolant at the nodes,
//   - Tinv: nodal values -> coefficients in Chebyshev polynomials of
//     x = 2 xi - 1, the inverse of T_k(x_j) (used for Clenshaw evaluation of
//     the element interpolant off the nodes).
#include "sl_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace sl {

namespace {

// number of roots of P_n strictly below x, from the sign changes of the
// Sturm sequence P_0(x), P_1(x), ..., P_n(x) of the three-term recurrence
int legendre_roots_below(int n, double x)
{
    double p0 = 1.0, p1 = x;
    int changes = 0;
    auto sgn = [](double v) { return v > 0 ? 1 : (v < 0 ? -1 : 0); };
    int prev = sgn(p0);
    int s1 = sgn(p1);
    if (s1 != 0 && s1 != prev) ++changes;
    if (s1 != 0) prev = s1;
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
        int s = sgn(p1);
        if (s != 0 && s != prev) ++changes;
        if (s != 0) prev = s;
    }
    // sign changes count the roots above x; the rest lie below
    return n - changes;
}

void legendre_eval(int n, double x, double* pn, double* dpn)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *dpn = (n == 1) ? 1.0 : n * (p0 - x * p1) / (1.0 - x * x);
}

void gauss_legendre(int n, double* xi, double* w)
{
    for (int r = 0; r < n; ++r) {
        // root r (ascending on [-1,1]): the point where the count reaches r+1
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 80; ++it) {
            double mid = 0.5 * (lo + hi);
            if (legendre_roots_below(n, mid) >= r + 1) hi = mid;
            else lo = mid;
        }
        double t = 0.5 * (lo + hi), pn, dp;
        for (int it = 0; it < 2; ++it) {
            legendre_eval(n, t, &pn, &dp);
            if (dp != 0.0) t -= pn / dp;
        }
        legendre_eval(n, t, &pn, &dp);
        xi[r] = 0.5 * (t + 1.0);
        w[r] = 1.0 / ((1.0 - t * t) * dp * dp);
    }
}

}  // namespace

// Gauss-Jordan inverse with partial pivoting; returns false if singular
bool invert(int n, const double* A, double* Ainv)
{
    std::vector<double> M(static_cast<size_t>(n) * 2 * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            M[i * 2 * n + j] = A[i * n + j];
            M[i * 2 * n + n + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r * 2 * n + c]) > std::fabs(M[p * 2 * n + c])) p = r;
        if (M[p * 2 * n + c] == 0.0) return false;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(M[c * 2 * n + j], M[p * 2 * n + j]);
        double piv = M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) M[c * 2 * n + j] /= piv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = M[r * 2 * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; ++j) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i * 2 * n + n + j];
    return true;
}

bool node_rule(int family, int n, double* xi, double* w)
{
    if (n < 1 || n > kMaxTableN) return false;
    if (family == 0) {
        gauss_legendre(n, xi, w);
        return true;
    }
    if (family != 1) return false;
    for (int j = 0; j < n; ++j) xi[j] = 0.5 * (1.0 - std::cos(M_PI * (j + 0.5) / n));
    // w_j = int_0^1 l_j = sum_k Tinv[k][j] * int_0^1 T_k(2 xi - 1) dxi,
    // int_0^1 T_k(2 xi - 1) dxi = 1/(1 - k^2) for even k, 0 for odd k
    std::vector<double> T(n * n), Ti(n * n);
    for (int j = 0; j < n; ++j) {
        double x = 2.0 * xi[j] - 1.0, t0 = 1.0, t1 = x;
        for (int k = 0; k < n; ++k) {
            double tk = (k == 0) ? 1.0 : (k == 1 ? x : 2.0 * x * t1 - t0);
            if (k >= 2) { t0 = t1; t1 = tk; }
            T[j * n + k] = tk;
        }
    }
    if (!invert(n, T.data(), Ti.data())) return false;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; k += 2) s += Ti[k * n + j] / (1.0 - double(k) * k);
        w[j] = s;
    }
    return true;
}

bool build_tables(int family, int n, Tables* T)
{
    std::memset(T, 0, sizeof(*T));
    T->n = n;
    if (!node_rule(family, n, T->xi, T->w)) return false;
    for (int j = 0; j < n; ++j) {
        double p = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) p *= (T->xi[j] - T->xi[m]);
        T->lam[j] = 1.0 / p;
    }
    // edge values of the basis by the barycentric formula (second form)
    for (int e = 0; e < 2; ++e) {
        double x = e ? 1.0 : 0.0, den = 0.0;
        double* l = e ? T->l1 : T->l0;
        for (int j = 0; j < n; ++j) den += T->lam[j] / (x - T->xi[j]);
        for (int j = 0; j < n; ++j) l[j] = (T->lam[j] / (x - T->xi[j])) / den;
    }
    // differentiation matrix (barycentric form)
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d = (T->lam[j] / T->lam[i]) / (T->xi[i] - T->xi[j]);
            T->D[i * n + j] = d;
            diag -= d;
        }
        T->D[i * n + i] = diag;
    }
    // Chebyshev-Vandermonde inverse
    std::vector<double> V(n * n);
    for (int j = 0; j < n; ++j) {
        double x = 2.0 * T->xi[j] - 1.0, t0 = 1.0, t1 = x;
        for (int k = 0; k < n; ++k) {
            double tk = (k == 0) ? 1.0 : (k == 1 ? x : 2.0 * x * t1 - t0);
            if (k >= 2) { t0 = t1; t1 = tk; }
            V[j * n + k] = tk;
        }
    }
    if (!invert(n, V.data(), T->Tinv)) return false;
    return true;
}

// 2D boundary rows C_B (4n x n^2): left edge j, right edge j, bottom edge
// i, top edge i; node index i + n j.  Both constrained fits are
//   phi = phihat + C_B^T Q (d_B - C_B phihat),
// HARD: Q = G^+ (then C_B^T Q = C_B^+), SOFT: Q = (I + G)^{-1} (Woodbury form
// of (I + C_B^T C_B)^{-1}(phihat + C_B^T d_B)), with G = C_B C_B^T (4n x 4n).
// G has rank 4n - 4: each corner value is reachable from two edges.  Its
// pseudo-inverse is built from the four corner combinations spanning null(G):
//   z_BL = l(0) on left - l(0) on bottom,  z_TL = l(1) on left - l(0) on top,
//   z_BR = l(0) on right - l(1) on bottom, z_TR = l(1) on right - l(1) on top;
// with Z their orthonormal basis, G^+ = (G + Z Z^T)^{-1} - Z Z^T.
bool build_boundary_tables(const Tables& T, double* Qhard, double* Qsoft, double* Zhard, double* Zsoft)
{
    const int n = T.n, nd = n * n, m = 4 * n;
    std::vector<double> CB((size_t)m * nd, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            CB[(size_t)(0 * n + j) * nd + i + n * j] = T.l0[i];
            CB[(size_t)(1 * n + j) * nd + i + n * j] = T.l1[i];
            CB[(size_t)(2 * n + i) * nd + i + n * j] = T.l0[j];
            CB[(size_t)(3 * n + i) * nd + i + n * j] = T.l1[j];
        }
    std::vector<double> G((size_t)m * m, 0.0);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int q = 0; q < nd; ++q) s += CB[(size_t)a * nd + q] * CB[(size_t)b * nd + q];
            G[(size_t)a * m + b] = s;
        }
    std::vector<double> Z((size_t)4 * m, 0.0);
    for (int k = 0; k < n; ++k) {
        Z[0 * m + 0 * n + k] = T.l0[k]; Z[0 * m + 2 * n + k] = -T.l0[k];
        Z[1 * m + 0 * n + k] = T.l1[k]; Z[1 * m + 3 * n + k] = -T.l0[k];
        Z[2 * m + 1 * n + k] = T.l0[k]; Z[2 * m + 2 * n + k] = -T.l1[k];
        Z[3 * m + 1 * n + k] = T.l1[k]; Z[3 * m + 3 * n + k] = -T.l1[k];
    }
    for (int a = 0; a < 4; ++a) {  // modified Gram-Schmidt, twice
        for (int pass = 0; pass < 2; ++pass)
            for (int b = 0; b < a; ++b) {
                double d = 0.0;
                for (int q = 0; q < m; ++q) d += Z[a * m + q] * Z[b * m + q];
                for (int q = 0; q < m; ++q) Z[a * m + q] -= d * Z[b * m + q];
            }
        double nr = 0.0;
        for (int q = 0; q < m; ++q) nr += Z[a * m + q] * Z[a * m + q];
        nr = std::sqrt(nr);
        if (!(nr > 0.0)) return false;
        for (int q = 0; q < m; ++q) Z[a * m + q] /= nr;
    }
    std::vector<double> H((size_t)m * m);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double zz = 0.0;
            for (int k = 0; k < 4; ++k) zz += Z[k * m + a] * Z[k * m + b];
            H[(size_t)a * m + b] = G[(size_t)a * m + b] + zz;
        }
    if (!invert(m, H.data(), Qhard)) return false;
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double zz = 0.0;
            for (int k = 0; k < 4; ++k) zz += Z[k * m + a] * Z[k * m + b];
            Qhard[(size_t)a * m + b] -= zz;
        }
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) H[(size_t)a * m + b] = G[(size_t)a * m + b] + (a == b ? 1.0 : 0.0);
    if (!invert(m, H.data(), Qsoft)) return false;
    // reference mass row g = w (x) w, projected: Z = g - C_B^T Q C_B g
    std::vector<double> g(nd), cg(m), qcg(m);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) g[i + n * j] = T.w[i] * T.w[j];
    for (int a = 0; a < m; ++a) {
        double s = 0.0;
        for (int q = 0; q < nd; ++q) s += CB[(size_t)a * nd + q] * g[q];
        cg[a] = s;
    }
    for (int pass = 0; pass < 2; ++pass) {
        const double* Q = pass == 0 ? Qhard : Qsoft;
        double* Z = pass == 0 ? Zhard : Zsoft;
        for (int a = 0; a < m; ++a) {
            double s = 0.0;
            for (int b = 0; b < m; ++b) s += Q[(size_t)a * m + b] * cg[b];
            qcg[a] = s;
        }
        for (int q = 0; q < nd; ++q) {
            double s = 0.0;
            for (int a = 0; a < m; ++a) s += CB[(size_t)a * nd + q] * qcg[a];
            Z[q] = g[q] - s;
        }
    }
    return true;
}

}  // namespace sl
