// Statistical diagnostics of Section 4, as GPU kernels: the byte histogram
// (frequency analysis; Shannon entropy follows from it) and the
// autocorrelation of a byte sequence.  The sums are integers, so the results
// do not depend on the reduction order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace lz {
namespace {

constexpr int DIAG_WG = 256;

// Per-workgroup LDS histogram, merged into the 256 global counters.
__global__ __launch_bounds__(DIAG_WG) void histogram_kernel(const uint8_t *data, uint64_t n,
                                                             unsigned long long *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * DIAG_WG * 4;
    for (uint64_t i = ((uint64_t)blockIdx.x * DIAG_WG + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n && ((uintptr_t)(data + i) & 3) == 0) {
            const uint32_t w = *reinterpret_cast<const uint32_t *>(data + i);
            atomicAdd(&h[w & 0xFF], 1u);
            atomicAdd(&h[(w >> 8) & 0xFF], 1u);
            atomicAdd(&h[(w >> 16) & 0xFF], 1u);
            atomicAdd(&h[w >> 24], 1u);
        } else {
            for (uint64_t j = i; j < n && j < i + 4; ++j) atomicAdd(&h[data[j]], 1u);
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// S_k = sum_{i < n-k} x_i x_{i+k} for k = 0..L.  A workgroup stages TILE + L bytes in LDS;
// each thread owns lags k = threadIdx.x, threadIdx.x + 256, ...
constexpr int AC_TILE = 4096;

__global__ __launch_bounds__(DIAG_WG) void lagsum_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                          unsigned long long *sums) {
    extern __shared__ uint8_t t[];
    const uint64_t i0 = (uint64_t)blockIdx.x * AC_TILE;
    const uint32_t span = AC_TILE + L;
    for (uint32_t j = threadIdx.x; j < span; j += DIAG_WG) t[j] = i0 + j < n ? data[i0 + j] : 0;
    __syncthreads();
    const uint32_t rows = n - i0 < (uint64_t)AC_TILE ? (uint32_t)(n - i0) : (uint32_t)AC_TILE;
    for (uint32_t k = threadIdx.x; k <= L; k += DIAG_WG) {
        // positions i0 + r with r < rows and i0 + r + k < n contribute
        const uint64_t lim = n - i0 > k ? n - i0 - k : 0;
        const uint32_t rk = lim < rows ? (uint32_t)lim : rows;
        uint64_t s = 0;
        for (uint32_t r = 0; r < rk; ++r) s += (uint32_t)t[r] * (uint32_t)t[r + k];
        if (s) atomicAdd(&sums[k], (unsigned long long)s);
    }
}

}  // namespace
}  // namespace lz

using namespace lz;

extern "C" int lz_histogram(lz_ctx *c, const uint8_t *d_data, size_t n, uint64_t *d_hist, void *stream) {
    if (!c || !d_hist || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    LZ_HIP(launch_fill_u64(reinterpret_cast<unsigned long long *>(d_hist), 256, s));
    if (n == 0) return LZ_OK;
    uint64_t blocks = (n + DIAG_WG * 4 * 16 - 1) / (DIAG_WG * 4 * 16);
    if (blocks > (uint64_t)c->dev.cus * 8) blocks = (uint64_t)c->dev.cus * 8;
    hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)blocks), dim3(DIAG_WG), 0, s, d_data, (uint64_t)n,
                       reinterpret_cast<unsigned long long *>(d_hist));
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

extern "C" int lz_lag_sums(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, uint64_t *d_sums,
                           void *stream) {
    if (!c || !d_sums || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    if (max_lag > 16384) return fail(LZ_E_INVAL, "max_lag must be <= 16384");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    LZ_HIP(launch_fill_u64(reinterpret_cast<unsigned long long *>(d_sums), (size_t)max_lag + 1, s));
    if (n == 0) return LZ_OK;
    const uint64_t blocks = (n + AC_TILE - 1) / AC_TILE;
    if (blocks > 0x7FFFFFFFull) return fail(LZ_E_INVAL, "input too long");
    hipLaunchKernelGGL(lagsum_kernel, dim3((unsigned)blocks), dim3(DIAG_WG), (size_t)AC_TILE + max_lag, s, d_data,
                       (uint64_t)n, max_lag, reinterpret_cast<unsigned long long *>(d_sums));
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}
