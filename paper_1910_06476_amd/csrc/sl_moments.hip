// Global mass and energy of a field (section 4, mass and energy
// conservation): the quadrature sums of phi and phi^2 over all nodes with the
// node weights w_i (1D) or w_i w_j (2D), on the device.  The element size
// factor is applied by the caller.  Each block sums a fixed set of nodes and
// reduces in a fixed order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sl_internal.h"

namespace sl {
namespace {

constexpr int kMomBlock = 256;
constexpr int kMomMaxBlocks = 2048;

__global__ __launch_bounds__(kMomBlock) void k_moments(const double* __restrict__ phi, int64_t nf, int n, int dim,
                                                       const double* __restrict__ w, double* __restrict__ part)
{
    __shared__ double sm[kMomBlock], se[kMomBlock];
    const int nd = dim == 1 ? n : n * n;
    const int64_t stride = (int64_t)gridDim.x * kMomBlock;
    const int step = (int)(stride % nd);  // the node index advances by this, modulo nd
    int64_t g = (int64_t)blockIdx.x * kMomBlock + threadIdx.x;
    int p = (int)(g % nd);
    double M = 0.0, E = 0.0;
    for (; g < nf; g += stride) {
        const double W = dim == 1 ? w[p] : w[p % n] * w[p / n];
        const double v = phi[g];
        M = fma(W, v, M);
        E = fma(W * v, v, E);
        p += step;
        if (p >= nd) p -= nd;
    }
    sm[threadIdx.x] = M;
    se[threadIdx.x] = E;
    __syncthreads();
    for (int s = kMomBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sm[threadIdx.x] += sm[threadIdx.x + s];
            se[threadIdx.x] += se[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sm[0];
        part[2 * blockIdx.x + 1] = se[0];
    }
}

}  // namespace

int moments_blocks(size_t nf) { return (int)std::min<size_t>(kMomMaxBlocks, (nf + kMomBlock - 1) / kMomBlock); }

int launch_moments(const double* phi, size_t nf, int n, int dim, const double* w, double* part, hipStream_t s)
{
    const int nb = moments_blocks(nf);
    if (nb < 1) return 1;
    hipLaunchKernelGGL(k_moments, dim3(nb), dim3(kMomBlock), 0, s, phi, (int64_t)nf, n, dim, w, part);
    return hipGetLastError() != hipSuccess;
}

}  // namespace sl
