// sl_step1d_static: 1D explicit SL steps (the path of sl_step on a 1D mesh)
// on caller device buffers, for callers that cannot allocate device memory.
//
// Everything the step needs beyond the caller's inputs and outputs -- the
// reference tables of every order, the velocity's Chebyshev coefficients,
// divergence and face speeds, the remapped field, the per-element records,
// the ping-pong field of multi-step calls and the per-block statistics --
// lives in one file-scope device array, `scratch`, of fixed size (sized for
// the largest 1D workload: 65536 elements of order 16).  Each GPU the
// library runs on holds its own copy until the process ends.  Host code
// never passes `scratch` itself to a kernel (in host code the name is a
// host-side stand-in); it uses the device address that hipGetSymbolAddress
// returns, once per device, at the first call on that device.
//
// All calls on one GPU share that GPU's array and it keeps the last call's
// contents: calls that overlap on one GPU (other streams, other host
// threads) race, and must be ordered by the caller.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "sl_internal.h"

namespace sl {
namespace {

constexpr int kStaticMaxK = 65536;
constexpr int kStaticMaxN = kMax1D;  // nodes per element (order 16)
constexpr size_t kStaticMaxDof = (size_t)kStaticMaxK * kStaticMaxN;
constexpr int kStaticMaxBlk = (kStaticMaxK + 13) / 14;  // per-block partials: 14 elements per advect block at n=17
constexpr size_t kAlign = 32;                           // doubles (256 B)
constexpr size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// tables of every order 2..17 of both node families, packed one after
// another (1D layout of tab_offsets: xi, w, l0, l1, Tinv, D, lambda)
constexpr size_t tab_doubles(int n) { return (size_t)5 * n + 2 * (size_t)n * n; }
constexpr size_t tables_total()
{
    size_t t = 0;
    for (int f = 0; f < 2; ++f)
        for (int n = 2; n <= kStaticMaxN; ++n) t += align_up(tab_doubles(n));
    return t;
}

// work region, in doubles: field ping-pong and phihat (2 dof), velocity
// coefficients with the [K][4] copies of velocity and divergence (dof + 8K),
// divergence and its coefficients (2 dof), face speeds (K + 1), records
// (kRec1 K), block statistics (kStatSlots nblk), block flags (2 nblk int32),
// the series degree (one int32)
constexpr size_t kWork = align_up(2 * kStaticMaxDof) + align_up(kStaticMaxDof + 8 * (size_t)kStaticMaxK) +
                         align_up(2 * kStaticMaxDof) + align_up(kStaticMaxK + 1) +
                         align_up((size_t)kRec1 * kStaticMaxK) + align_up((size_t)kStatSlots * kStaticMaxBlk) +
                         align_up(kStaticMaxBlk + 1) + kAlign;
constexpr size_t kScratchDoubles = tables_total() + kWork;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices];  // device address of `scratch` per device, after set-up

__global__ void k_static_zero(double* __restrict__ stat, int nstat, int32_t* __restrict__ flags, int nflag,
                              int32_t* __restrict__ vdeg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nstat) stat[i] = 0.0;
    if (i < nflag) flags[i] = 0;
    if (i == 0) *vdeg = 0;
}

// the step statistics of the block partials: resid_boundary, resid_mass,
// resid_energy, max_picard (maxima), and the flag bits (or)
__global__ void k_static_reduce(const double* __restrict__ stat, const int32_t* __restrict__ flags, int nblk,
                                double* __restrict__ out_stats, int32_t* __restrict__ out_flags)
{
    __shared__ double s_m[4][256];
    __shared__ int32_t s_f[256];
    const int t = threadIdx.x;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    int32_t f = 0;
    for (int b = t; b < nblk; b += 256) {
#pragma unroll
        for (int c = 0; c < 4; ++c) m[c] = fmax(m[c], stat[(size_t)b * kStatSlots + c]);
        f |= flags[b] | flags[nblk + b];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s_m[c][t] = m[c];
    s_f[t] = f;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int c = 0; c < 4; ++c) s_m[c][t] = fmax(s_m[c][t], s_m[c][t + h]);
            s_f[t] |= s_f[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (out_stats)
            for (int c = 0; c < 4; ++c) out_stats[c] = s_m[c][0];
        if (out_flags) *out_flags = s_f[0];
    }
}

// offset of the tables of (family, n) in the table region
size_t table_offset(int family, int n)
{
    size_t t = 0;
    for (int f = 0; f < 2; ++f)
        for (int k = 2; k <= kStaticMaxN; ++k) {
            if (f == family && k == n) return t;
            t += align_up(tab_doubles(k));
        }
    return 0;
}

// Set-up, once per device with that device current: the device address of
// `scratch`, and the tables of every order written to its head.
sl_status setup_device(int dev, double** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev]) {
        *out = g_ptr[dev];
        return SL_OK;
    }
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SL_E_DEVICE;
    std::vector<double> tabs(tables_total(), 0.0);
    for (int f = 0; f < 2; ++f)
        for (int n = 2; n <= kStaticMaxN; ++n) {
            Tables T;
            if (!build_tables(f, n, &T)) return SL_E_DEVICE;
            const TabOff o = tab_offsets(1, n);
            double* d = tabs.data() + table_offset(f, n);
            for (int j = 0; j < n; ++j) {
                d[o.xi + j] = T.xi[j];
                d[o.w + j] = T.w[j];
                d[o.l0 + j] = T.l0[j];
                d[o.l1 + j] = T.l1[j];
                for (int k = 0; k < n; ++k) {
                    d[o.tinv + j * n + k] = T.Tinv[j * n + k];
                    d[o.dmat + j * n + k] = T.D[j * n + k];
                }
            }
        }
    if (hipMemcpy(p, tabs.data(), tabs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return SL_E_DEVICE;
    g_ptr[dev] = (double*)p;
    *out = g_ptr[dev];
    return SL_OK;
}

}  // namespace
}  // namespace sl

using namespace sl;

extern "C" sl_status sl_step1d_static(int32_t K, int32_t order, int32_t nodes, int32_t bc, int32_t form, double x0,
                                      double x1, const double* phi_in, double* phi_out, const double* a,
                                      const double* div_a, double amax, const double* ghost, double dt,
                                      int32_t nsteps, const sl_step_opts* opts, double* stats, int32_t* flags,
                                      void* stream)
{
    // validation before any device call
    sl_step_opts opt = {4, SL_C_BOUNDARY, SL_MODE_HARD, 50, 3, SL_IFACE_INTERP, 1e-8};
    if (opts) opt = *opts;
    const int n = order + 1;
    if (order < 1 || n > kStaticMaxN || K < 1 || K > kStaticMaxK || (size_t)K * n > kStaticMaxDof)
        return SL_E_INVALID;
    if (nodes != SL_NODES_GL && nodes != SL_NODES_CG) return SL_E_INVALID;
    if (bc != SL_BC_PERIODIC && bc != SL_BC_GHOST) return SL_E_INVALID;
    if (form != SL_FORM_ADVECTIVE && form != SL_FORM_CONSERVATIVE) return SL_E_INVALID;
    if (!(x1 > x0) || !std::isfinite(x0) || !std::isfinite(x1)) return SL_E_INVALID;
    if (!phi_in || !phi_out || !a || (bc == SL_BC_GHOST && !ghost)) return SL_E_INVALID;
    if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0 || !(amax >= 0) || !std::isfinite(amax)) return SL_E_INVALID;
    if (!step_opts_valid(opt)) return SL_E_INVALID;
    const int rows = ((opt.constraints & SL_C_BOUNDARY) ? 2 : 0) + ((opt.constraints & SL_C_MASS) ? 1 : 0) +
                     ((opt.constraints & SL_C_ENERGY) ? 1 : 0);
    if (rows > n) return SL_E_INVALID;
    Tables T;
    if (!build_tables(nodes, n, &T)) return SL_E_INVALID;
    const double dx = (x1 - x0) / K;
    if (amax * dt > T.xi[0] * dx * (1.0 + 1e-12)) return SL_E_CFL;

    const ApiHold hold;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SL_E_DEVICE;
    double* base = nullptr;
    const sl_status st = setup_device(dev, &base);
    if (st != SL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t dof = (size_t)K * n;
    if (nsteps == 0) {
        if (phi_out != phi_in &&
            hipMemcpyAsync(phi_out, phi_in, dof * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return SL_E_DEVICE;
        if (stats || flags) hipLaunchKernelGGL(k_static_reduce, dim3(1), dim3(256), 0, s, base, nullptr, 0, stats, flags);
        return hipGetLastError() == hipSuccess ? SL_OK : SL_E_DEVICE;
    }

    // carve the work region (fixed offsets sized for the maximum)
    double* w = base + tables_total();
    double* tmp = w;
    double* phihat = tmp + kStaticMaxDof;
    w += align_up(2 * kStaticMaxDof);
    double* aM = w;  // [K][n], then the [K][4] copies of aM and divM
    w += align_up(kStaticMaxDof + 8 * (size_t)kStaticMaxK);
    double* divN = w;
    double* divM = divN + kStaticMaxDof;
    w += align_up(2 * kStaticMaxDof);
    double* vface = w;
    w += align_up(kStaticMaxK + 1);
    double* rec = w;
    w += align_up((size_t)kRec1 * kStaticMaxK);
    double* stat_part = w;
    w += align_up((size_t)kStatSlots * kStaticMaxBlk);
    int32_t* flag_part = (int32_t*)w;
    int32_t* vdeg_d = flag_part + 2 * kStaticMaxBlk;

    const int nblk = blocks1d(n, K);
    if (nblk < 1 || nblk > kStaticMaxBlk) return SL_E_INVALID;
    const double* tab = base + table_offset(nodes, n);
    const int periodic = bc == SL_BC_PERIODIC, cons = form == SL_FORM_CONSERVATIVE;
    // given divergence: read from the caller's array (prep only reads it then)
    double* div_used = div_a ? const_cast<double*>(div_a) : divN;

    const int nz = std::max(kStatSlots * nblk, 2 * nblk);
    hipLaunchKernelGGL(k_static_zero, dim3((nz + 255) / 256), dim3(256), 0, s, stat_part, kStatSlots * nblk,
                       flag_part, 2 * nblk, vdeg_d);
    if (hipGetLastError() != hipSuccess) return SL_E_DEVICE;
    if (launch_prep1d(n, K, periodic, div_a != nullptr, a, aM, div_used, divM, aM + dof, aM + dof + 4 * (size_t)K,
                      vface, tab, dx, cons, amax, vdeg_d, s))
        return SL_E_DEVICE;

    Step1DArgs A;
    std::memset(&A, 0, sizeof(A));
    if (!step1d_setup(T, n, dx, periodic, cons, opt, amax, &A)) return SL_E_INVALID;
    A.aN = a; A.aM = aM; A.divN = div_used; A.divM = divM; A.vface = vface; A.tab = tab;
    A.aM4 = aM + dof;
    A.divM4 = aM + dof + 4 * (size_t)K;
    A.rec = rec; A.phihat = phihat;
    A.flag_part = flag_part; A.stat_part = stat_part; A.nblk = nblk;
    A.vdeg = n - 1;  // the whole velocity series (its degree is not read back)
    A.K = K;
    A.dt = dt;
    // the last step writes phi_out: step i writes phi_out when nsteps - 1 - i
    // is even, else the scratch field
    const double* src = phi_in;
    for (int i = 0; i < nsteps; ++i) {
        double* dst = ((nsteps - 1 - i) % 2 == 0) ? phi_out : tmp;
        if (bc == SL_BC_GHOST) {
            A.gnow = ghost + 2 * (size_t)i;
            A.gnext = ghost + 2 * (size_t)(i + 1);
        } else {
            A.gnow = A.gnext = vface;  // unused for periodic meshes (valid address)
        }
        A.phi = src;
        A.phi_out = dst;
        if (launch_advect1d(n, A, s) || launch_constrain1d(n, A, s)) return SL_E_DEVICE;
        src = dst;
    }
    if (stats || flags)
        hipLaunchKernelGGL(k_static_reduce, dim3(1), dim3(256), 0, s, stat_part, flag_part, nblk, stats, flags);
    return hipGetLastError() == hipSuccess ? SL_OK : SL_E_DEVICE;
}
