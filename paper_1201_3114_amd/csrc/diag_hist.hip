// Byte histogram (frequency analysis) and Shannon entropy of Section 4 as GPU kernels; the
// counts are exact, so they do not depend on the order of the additions.
#include "diag_common.h"

namespace lz {
namespace {

// Byte histogram.  The workgroup's LDS counters hold HIST_COPIES copies of each
// bin, interleaved (bin * HIST_COPIES + copy, copy = lane mod HIST_COPIES): the
// 32 lanes of a half-wave always add into 32 different banks, whatever their
// bytes, so skewed input (text, constant runs) does not serialise the LDS
// atomics and random input does not collide in banks.  Each lane reads 16 bytes
// per load, HIST_U loads per batch, and issues the next batch's loads before
// counting the current one, so the loads overlap the LDS atomics (non-temporal
// loads: the data is read once; 4% faster per GiB than cached loads).  The copies
// are summed at the end; workgroup b adds its counts to copy b mod DIAG_MERGE of
// the bins in the context's merge buffer (one device atomic per occupied bin:
// eight tables instead of one spread the atomics of hundreds of workgroups over
// more memory channels), and a one-workgroup kernel then writes the sum of the
// copies to the output and clears them for the next call.
// Block 0 also counts the unaligned head and the tail that does not fill 16 bytes.
constexpr int HIST_U = 4;
constexpr int HIST_COPIES = 32;

// 16 bytes of the data, read once: a non-temporal load (the bytes are not kept in the caches)
__device__ __forceinline__ uint4 hist_load(const uint4 *v, uint64_t i, uint64_t nv) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    if (i >= nv) return make_uint4(0, 0, 0, 0);
    const v4u x = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(v + i));
    return make_uint4(x[0], x[1], x[2], x[3]);
}

__device__ __forceinline__ void count_word(uint32_t *h, uint32_t w) {
    atomicAdd(&h[(w & 0xFF) * HIST_COPIES], 1u);
    atomicAdd(&h[((w >> 8) & 0xFF) * HIST_COPIES], 1u);
    atomicAdd(&h[((w >> 16) & 0xFF) * HIST_COPIES], 1u);
    atomicAdd(&h[(w >> 24) * HIST_COPIES], 1u);
}

__global__ __launch_bounds__(DIAG_WG) void histogram_kernel(const uint8_t *data, uint64_t n,
                                                             unsigned long long *merge) {
    __shared__ uint32_t h[256 * HIST_COPIES];
    for (int i = threadIdx.x; i < 256 * HIST_COPIES; i += DIAG_WG) h[i] = 0;
    __syncthreads();
    uint32_t *hc = h + threadIdx.x % HIST_COPIES;  // this lane's copy
    const uint64_t head = ((16 - ((uintptr_t)data & 15)) & 15) < n ? ((16 - ((uintptr_t)data & 15)) & 15) : n;
    const uint64_t nv = (n - head) / 16;
    const uint4 *v = reinterpret_cast<const uint4 *>(data + head);
    if (blockIdx.x == 0) {
        for (uint64_t j = threadIdx.x; j < head; j += DIAG_WG) atomicAdd(&hc[data[j] * HIST_COPIES], 1u);
        for (uint64_t j = head + nv * 16 + threadIdx.x; j < n; j += DIAG_WG) atomicAdd(&hc[data[j] * HIST_COPIES], 1u);
    }
    const uint64_t stride = (uint64_t)gridDim.x * DIAG_WG;
    uint64_t i = (uint64_t)blockIdx.x * DIAG_WG + threadIdx.x;
    uint4 q[HIST_U];
#pragma unroll
    for (int u = 0; u < HIST_U; ++u) q[u] = hist_load(v, i + u * stride, nv);
    for (; i < nv; i += stride * HIST_U) {
        // the next batch's loads are issued before this batch is counted
        const uint64_t j = i + stride * HIST_U;
        uint4 next[HIST_U];
#pragma unroll
        for (int u = 0; u < HIST_U; ++u) next[u] = hist_load(v, j + u * stride, nv);
#pragma unroll
        for (int u = 0; u < HIST_U; ++u) {
            if (i + u * stride >= nv) break;
            count_word(hc, q[u].x);
            count_word(hc, q[u].y);
            count_word(hc, q[u].z);
            count_word(hc, q[u].w);
        }
#pragma unroll
        for (int u = 0; u < HIST_U; ++u) q[u] = next[u];
    }
    __syncthreads();
    unsigned long long c = 0;
    for (int k = 0; k < HIST_COPIES; ++k) c += h[threadIdx.x * HIST_COPIES + k];
    if (c) atomicAdd(&merge[(blockIdx.x % DIAG_MERGE) * 256 + threadIdx.x], c);
}

// Writes the sum of the merge copies to the output and clears them for the next call.
__global__ __launch_bounds__(256) void hist_merge_kernel(unsigned long long *merge, unsigned long long *hist) {
    unsigned long long t = 0;
    for (int k = 0; k < DIAG_MERGE; ++k) {
        t += merge[k * 256 + threadIdx.x];
        merge[k * 256 + threadIdx.x] = 0;
    }
    hist[threadIdx.x] = t;
}

// S = -sum p_i log2 p_i with p_i = h_i / n over the occupied byte values; S = 0 when n = 0.
__global__ __launch_bounds__(DIAG_WG) void entropy_kernel(const unsigned long long *hist, double *out) {
    __shared__ unsigned long long ired[DIAG_WG];
    __shared__ double dred[DIAG_WG];
    const unsigned long long h = hist[threadIdx.x];
    const unsigned long long n = block_sum<unsigned long long>(h, ired);
    double term = 0.0;
    if (h != 0) {
        const double p = (double)h / (double)n;
        term = -p * log2(p);
    }
    const double S = block_sum<double>(term, dred);
    if (threadIdx.x == 0) out[0] = S;
}

}  // namespace

// The context's diagnostics workspace: grown on demand, and calls on different
// streams are ordered through one event so that they never share it at once.
int diag_begin(lz_ctx *c, hipStream_t s, size_t bytes, char **ws) {
    if (c->diag_has_last && c->diag_last != s) LZ_HIP(hipStreamWaitEvent(s, c->diag_event, 0));
    if (bytes > c->diag_ws_bytes) {
        if (c->diag_has_last) LZ_HIP(hipEventSynchronize(c->diag_event));
        if (c->diag_ws) LZ_HIP(hipFree(c->diag_ws));
        c->diag_ws = nullptr;
        c->diag_ws_bytes = 0;
        const hipError_t e = hipMalloc(&c->diag_ws, bytes);
        if (e != hipSuccess) {
            c->diag_ws = nullptr;
            return e == hipErrorOutOfMemory ? fail(LZ_E_NOMEM, "diagnostics workspace does not fit")
                                            : hip_fail(e, "diagnostics workspace");
        }
        c->diag_ws_bytes = bytes;
    }
    *ws = static_cast<char *>(c->diag_ws);
    return LZ_OK;
}

int diag_end(lz_ctx *c, hipStream_t s) {
    LZ_HIP(hipEventRecord(c->diag_event, s));
    c->diag_last = s;
    c->diag_has_last = true;
    return LZ_OK;
}

}  // namespace lz

using namespace lz;

extern "C" int lz_histogram(lz_ctx *c, const uint8_t *d_data, size_t n, uint64_t *d_hist, void *stream) {
    if (!c || !d_hist || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    if (n == 0) {
        LZ_HIP(launch_fill_u64(reinterpret_cast<unsigned long long *>(d_hist), 256, s));
        return LZ_OK;
    }
    // about 16 KiB per workgroup at least, at most 2 workgroups per CU; the 32-bit LDS counters
    // stay below 2^32 while each workgroup covers fewer than 2^32 bytes
    uint64_t blocks = (n + 16383) / 16384;
    if (blocks > (uint64_t)c->dev.cus * 2) blocks = (uint64_t)c->dev.cus * 2;
    if (n / blocks >= (1ull << 32) - 1024) blocks = (n >> 31) + 1;
    if (blocks > 0x7FFFFFFFull) return fail(LZ_E_INVAL, "input too long");
    char *ws;  // the merge buffer is the context's: calls on different streams are ordered
    if (int rc = diag_begin(c, s, 0, &ws)) return rc;
    hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)blocks), dim3(DIAG_WG), 0, s, d_data, (uint64_t)n,
                       c->diag_merge);
    hipLaunchKernelGGL(hist_merge_kernel, dim3(1), dim3(256), 0, s, c->diag_merge,
                       reinterpret_cast<unsigned long long *>(d_hist));
    LZ_HIP(hipGetLastError());
    return diag_end(c, s);
}

extern "C" int lz_entropy(lz_ctx *c, const uint64_t *d_hist, double *d_S, void *stream) {
    if (!c || !d_hist || !d_S) return fail(LZ_E_INVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    hipLaunchKernelGGL(entropy_kernel, dim3(1), dim3(DIAG_WG), 0, s,
                       reinterpret_cast<const unsigned long long *>(d_hist), d_S);
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}
