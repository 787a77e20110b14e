// Device side of batched launches: one launch runs the same step kernel for
// several meshes, each block working for one of them.
#pragma once

#include <hip/hip_runtime.h>

namespace sl {

// Request of block b: the last r < nreq with start[r] <= b (start ascending
// from start[0] = 0; request r owns blocks start[r] .. start[r + 1] - 1).
// Uniform over the block: scalar loads only.
__device__ __forceinline__ int batch_request(const int* __restrict__ start, int nreq, int b)
{
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

}  // namespace sl
