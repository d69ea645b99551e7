// Batched device-to-device copies: one launch moves many (src, dst, len)
// pieces, where one copy call per piece would queue thousands of small
// launches.  The table of pieces is in device memory, or, for a host table,
// in the kernel arguments (COPY_ARG_PIECES per launch).  A workgroup takes pieces in turn; 16-byte vector moves when the
// two addresses agree modulo 16 (after a short head), bytes otherwise.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace lz {
namespace {

constexpr int COPY_WG = 256;

__device__ __forceinline__ void copy_piece(const CopyPiece &p) {
    const uint8_t *s = p.src;
    uint8_t *d = p.dst;
    const uint64_t len = p.len;
    if ((((uintptr_t)s ^ (uintptr_t)d) & 15) == 0) {
        uint64_t head = (16 - ((uintptr_t)s & 15)) & 15;
        if (head > len) head = len;
        for (uint64_t j = threadIdx.x; j < head; j += COPY_WG) d[j] = s[j];
        const uint64_t nv = (len - head) / 16;
        const uint4 *sv = reinterpret_cast<const uint4 *>(s + head);
        uint4 *dv = reinterpret_cast<uint4 *>(d + head);
        for (uint64_t j = threadIdx.x; j < nv; j += COPY_WG) dv[j] = sv[j];
        for (uint64_t j = head + nv * 16 + threadIdx.x; j < len; j += COPY_WG) d[j] = s[j];
    } else {
        for (uint64_t j = threadIdx.x; j < len; j += COPY_WG) d[j] = s[j];
    }
}

__global__ __launch_bounds__(COPY_WG) void copy_many_kernel(const CopyPiece *pieces, uint32_t n) {
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) copy_piece(pieces[i]);
}

// the pieces in the kernel's arguments: nothing to upload first
struct CopyArgs {
    CopyPiece p[COPY_ARG_PIECES];
    uint32_t n;
};

__global__ __launch_bounds__(COPY_WG) void copy_args_kernel(const CopyArgs a) {
    for (uint32_t i = blockIdx.x; i < a.n; i += gridDim.x) copy_piece(a.p[i]);
}

}  // namespace

hipError_t launch_copy_many(const CopyPiece *pieces, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned grid = n < 4096 ? n : 4096;
    hipLaunchKernelGGL(copy_many_kernel, dim3(grid), dim3(COPY_WG), 0, s, pieces, n);
    return hipGetLastError();
}

hipError_t launch_copy_pieces_host(const CopyPiece *pieces, uint32_t n, hipStream_t s) {
    for (uint32_t i = 0; i < n; i += COPY_ARG_PIECES) {
        CopyArgs a;
        a.n = n - i < COPY_ARG_PIECES ? n - i : COPY_ARG_PIECES;
        for (uint32_t j = 0; j < a.n; ++j) a.p[j] = pieces[i + j];
        hipLaunchKernelGGL(copy_args_kernel, dim3(a.n), dim3(COPY_WG), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lz
