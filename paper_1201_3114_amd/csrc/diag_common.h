// Shared by the Section 4 analyses (diag_hist.hip, diag_lags.hip, diag_fft.hip): their
// workgroup size, a workgroup sum, and the ordering of the calls that share the context's
// diagnostics workspace and merge buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace lz {

constexpr int DIAG_WG = 256;

// Block-wide sum over 256 threads (LDS tree, fixed order, so the result is deterministic).
template <typename T>
__device__ T block_sum(T v, T *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = DIAG_WG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const T r = red[0];
    __syncthreads();
    return r;
}

// The context's diagnostics workspace, grown to at least bytes (after the previous call has
// finished) and returned in *ws; a call on another stream than the previous one waits for it.
int diag_begin(lz_ctx *c, hipStream_t s, size_t bytes, char **ws);
// Records the end of a call on stream s, for the next call's diag_begin.
int diag_end(lz_ctx *c, hipStream_t s);

}  // namespace lz
