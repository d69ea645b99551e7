// Statistical analyses of Section 4 as GPU kernels: the byte histogram
// (frequency analysis) and Shannon entropy, the autocorrelation of a byte
// sequence, and, for a byte matrix (a text or an image laid out row by row),
// the circular autocorrelation matrix and the 2-D Fourier power spectrum.
// Integer sums are exact (the results do not depend on the reduction order);
// the floating-point results are binary64.  The lag sums are int8 matrix
// products on the matrix cores (up to lag 256 in one launch, beyond that in
// windows of at most 4096 lags); the 2-D transforms run
// as FFTs for sides with no prime factor above 5 and as binary64 matrix products
// on the matrix cores otherwise.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "internal.h"

namespace lz {
namespace {

constexpr int DIAG_WG = 256;

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

// ---- the lag sums on the matrix cores ----------------------------------------------------
//
// With the bytes laid out as rows of 32, S_k is a sum along the diagonals of the integer matrix
// products G_t[c][j] = sum_r x[32 r + c] x[32 (r + t) + j] (c, j < 32; lag k = 32 t + j - c), with
// the rows as their inner dimension, which run on v_mfma_i32_32x32x32_i8.  The matrix cores take
// signed bytes, so the kernels work with x' = x - 128 (byte XOR 0x80; 0 past n) and
//   S_k = S'_k + 256 T - 128 (P_k + Q_k) - 16384 max(n - k, 0),
// T the byte total, P_k and Q_k the sums of the first and the last min(k, n) bytes: each workgroup
// adds its sums plus 256 times its bytes' total, one atomic per lag, into one of several copies
// of the context's merge buffer (the copies spread the device atomics of hundreds of
// workgroups), and a correction kernel adds up the copies, clears them and applies the rest.
//
typedef int v4i __attribute__((ext_vector_type(4)));

// ---- the lag sums for lags up to 256: 32-byte rows, 32 x 32 x 32 int8 products ----------------
//
// Tiles t = 0 .. NT - 1 with NT = (L + 31) / 32 + 1 cover lags 0..L with no tile to spare (nine
// for L = 256).  One v_mfma_i32_32x32x32_i8 takes 32
// rows: lane l supplies column l % 32 of rows 16 (l / 32) .. + 15 as its 16 operand bytes, A
// unshifted and B shifted by t rows, so the same LDS column serves both and B comes from one
// 24-byte read by alignbyte.  The result's register i in lane l is G[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
//
// Wave w of the four takes tiles w, w + 4, ... (F = NT / 4 of them, all the task's rows: every
// such tile of the wave has the same shift w mod 4 within a word) and the S = NT mod 4 last tiles
// over its quarter of the rows, so each wave does the same number of products and holds only
// F + S accumulators.  A task is LS_ROWS rows of 32 bytes, staged column by column (a thread
// transposes pieces of 4 rows x LS_CB bytes with byte permutes) with the LS_HALO rows after it
// that the shifted operands reach.  The next task's loads are issued before the current task's
// products, and the accumulators stay in registers over LS_FLUSH tasks of the workgroup (each
// accumulator then sums at most LS_FLUSH x LS_ROWS products of at most 2^14, below 2^31) before
// the diagonals are added into the LDS lag counters.  Each workgroup adds its sums plus 256 times
// its bytes' total into copy b mod LS_COPIES of the merge buffer (the lags' adds of hundreds of
// workgroups, spread over more copies than the kernel above uses).
constexpr uint32_t LS_ROWS = 512;
// staging: a thread takes LS_EV pieces of 4 rows x LS_CB bytes (LS_CB = 32: whole rows)
constexpr uint32_t LS_CB = LS_ROWS >= 1024 ? 32 : LS_ROWS * 32 / 1024;
constexpr uint32_t LS_EV = LS_ROWS * 32 / (4 * LS_CB) / DIAG_WG;
static_assert(LS_CB == 32 || LS_CB == 16 || LS_CB == 8, "piece width");
static_assert(LS_EV * DIAG_WG * 4 * LS_CB == LS_ROWS * 32, "every thread stages whole pieces");
constexpr uint32_t LS_HALO = 8;                 // rows past a task read by the shifted operands
constexpr uint32_t LS_STRIDE = LS_ROWS + 16;    // LDS bytes per column, an odd multiple of 16
constexpr uint32_t LS_FLUSH = 64;               // tasks between flushes: 64 x 512 x 2^14 = 2^29
constexpr uint32_t LS_MAX_NT = 9;               // lags up to 256
// merge copies: workgroup b adds into copy b mod LS_COPIES (hundreds of workgroups add to each lag)
constexpr uint32_t LS_COPIES = 32;
static_assert((size_t)LS_COPIES * (32 * (LS_MAX_NT - 1) + 2) <= DIAG_MERGE_WORDS, "merge buffer too small");
static_assert(LS_ROWS % 128 == 0 && LS_ROWS >= 128, "whole 32-row blocks for each of the four waves");
static_assert((uint64_t)LS_FLUSH * LS_ROWS * 16384 < (1ull << 31), "32-bit accumulators");

typedef int v16i __attribute__((ext_vector_type(16)));

// Raw bytes i0 .. i0 + nb - 1 loaded one by one, 0x80 for bytes at or past n (the XOR with 0x80
// that turns the others into x - 128 then makes them 0).
__device__ inline uint4 ls_bytes(const uint8_t *data, uint64_t n, uint64_t i0, uint32_t nb) {
    uint32_t w[4] = {0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
    for (uint32_t b = 0; b < nb; ++b)
        if (i0 + b < n) w[b / 4] = (w[b / 4] & ~(0xFFu << (8 * (b % 4)))) | ((uint32_t)data[i0 + b] << (8 * (b % 4)));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ inline uint4 ls_load16(const uint8_t *data, uint64_t n, uint64_t i0, bool aligned16, uint32_t nb) {
    // bytes i0 .. i0 + nb - 1 (nb = 8 or 16, i0 a multiple of nb) as x - 128 (XOR 0x80), 0 past n
    if (aligned16 && i0 + nb <= n) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (nb == 16) {
            v = *reinterpret_cast<const uint4 *>(data + i0);
        } else {
            const uint2 u = *reinterpret_cast<const uint2 *>(data + i0);
            v.x = u.x, v.y = u.y;
        }
        v.x ^= 0x80808080u, v.y ^= 0x80808080u, v.z ^= 0x80808080u, v.w ^= 0x80808080u;
        return v;
    }
    uint32_t w[4] = {0, 0, 0, 0};
    for (uint32_t b = 0; b < nb; ++b)
        if (i0 + b < n) w[b / 4] |= ((uint32_t)data[i0 + b] ^ 0x80u) << (8 * (b % 4));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int NT>
__global__ __launch_bounds__(DIAG_WG) __attribute__((amdgpu_waves_per_eu(2))) void lagsum_small_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                                unsigned long long *merge) {
    static_assert(NT >= 1 && NT <= (int)LS_MAX_NT, "tiles");
    constexpr int F = NT / 4, S = NT % 4;  // tiles per wave over all rows; tiles shared out by rows
    __shared__ __align__(16) uint8_t lt[32 * LS_STRIDE];
    // lag counters for k = -32 .. 32 NT - 1: the diagonals of every tile land in range, so the
    // flush adds without a test (the counters outside 0..L are never read)
    __shared__ unsigned long long acc_all[32 * NT + 32];
    __shared__ long long wred[DIAG_WG / 64];
    unsigned long long *acc = acc_all + 32;
    for (uint32_t k = threadIdx.x; k < 32 * NT + 32; k += DIAG_WG) acc_all[k] = 0;
    const uint32_t t = threadIdx.x, lane = t % 64, col = lane % 32, h = lane / 32;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t / 64);
    const bool aligned16 = (reinterpret_cast<uintptr_t>(data) & 15) == 0;
    const uint64_t nrows = (n + 31) / 32, tasks = (nrows + LS_ROWS - 1) / LS_ROWS;
    v16i d[F + S];
#pragma unroll
    for (int q = 0; q < F + S; ++q) d[q] = (v16i){};
    // piece p = t + DIAG_WG v: rows 4 (p / PQ) .. + 3, bytes LS_CB (p % PQ) .. + LS_CB - 1 of each
    // (PQ = 32 / LS_CB pieces per 4 rows), as LS_CB / 4 raw words per row: pw[v][row][word]; every
    // thread also one half row of the halo (thread t mod 2 LS_HALO's).  Each load is issued
    // unconditionally, from offset 0 when its bytes are not all inside aligned data (bit set in
    // redo); those are fetched again byte by byte when the task is staged, where the thread waits
    // for its loads anyway.
    constexpr uint32_t PQ = 32 / LS_CB, PW = LS_CB / 4, NL = 4 * LS_EV * ((PW + 3) / 4);  // loads per task
    static_assert(NL < 32, "one redo bit per load and the halo");
    const bool vec = aligned16 && n >= 16;
    uint32_t pw[LS_EV][4][PW];
    uint4 ph = make_uint4(0, 0, 0, 0);
    uint32_t redo = 0;
    auto piece_at = [&](uint64_t b0, uint32_t v, int r, uint32_t hw) -> uint64_t {
        const uint32_t pc = t + DIAG_WG * v;
        return b0 + (4 * (uint64_t)(pc / PQ) + r) * 32 + LS_CB * (pc % PQ) + 4 * hw;
    };
    auto halo_at = [&](uint64_t b0) -> uint64_t {
        return b0 + (uint64_t)(LS_ROWS + (t % (2 * LS_HALO)) / 2) * 32 + 16 * (t % 2);
    };
    auto put = [&](uint32_t v, int r, uint32_t hw, const uint4 &x) {
        pw[v][r][hw] = x.x;
        if (PW > 1) pw[v][r][hw + 1] = x.y;
        if (PW > 2) pw[v][r][hw + 2] = x.z;
        if (PW > 3) pw[v][r][hw + 3] = x.w;
    };
    auto load = [&](uint64_t task) {
        const uint64_t b0 = task * LS_ROWS * 32;
        if (!vec) {  // misaligned data or under 16 bytes: every load byte by byte (no offset-0 load)
            redo = (2u << NL) - 1;
            return;
        }
        redo = 0;
        uint32_t k = 0;
#pragma unroll
        for (uint32_t v = 0; v < LS_EV; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (uint32_t hw = 0; hw < PW; hw += 4, ++k) {
                    const uint64_t i0 = piece_at(b0, v, r, hw);
                    const bool in = i0 + 4 * (PW >= 4 ? 4 : PW) <= n;
                    redo |= in ? 0u : 1u << k;
                    const uint8_t *src = data + (in ? i0 : 0);
                    if (PW >= 4) {
                        put(v, r, hw, *reinterpret_cast<const uint4 *>(src));
                    } else {
                        const uint2 u = *reinterpret_cast<const uint2 *>(src);
                        put(v, r, hw, make_uint4(u.x, u.y, 0u, 0u));
                    }
                }
        const uint64_t hb = halo_at(b0);
        const bool in = hb + 16 <= n;
        redo |= in ? 0u : 1u << NL;
        ph = *reinterpret_cast<const uint4 *>(data + (in ? hb : 0));
    };
    // the loads that were not all inside aligned data, byte by byte (tail and misaligned data only)
    auto fixup = [&](uint64_t task) {
        if (!redo) return;
        const uint64_t b0 = task * LS_ROWS * 32;
        uint32_t k = 0;
#pragma unroll
        for (uint32_t v = 0; v < LS_EV; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (uint32_t hw = 0; hw < PW; hw += 4, ++k)
                    if (redo >> k & 1) put(v, r, hw, ls_bytes(data, n, piece_at(b0, v, r, hw), PW >= 4 ? 16 : 4 * PW));
        if (redo >> NL & 1) ph = ls_bytes(data, n, halo_at(b0), 16);
    };
    int tsum = 0;  // this thread's share of sum (x - 128) over the tasks' own rows
    // lag of d[q][i]: 32 tile + col - (8 (i / 4) + 4 h + i % 4), tile = wave + 4 q (q < F) or 4 F + q - F
    unsigned long long *diag = acc + (int)col - 4 * (int)h;
    auto flush = [&]() {
#pragma unroll
        for (int q = 0; q < F + S; ++q)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int tile_off = q < F ? 32 * 4 * q : 32 * (4 * F + q - F);
                unsigned long long *p = (q < F ? diag + 32 * (int)wave : diag) + (tile_off - 8 * (i / 4) - i % 4);
                atomicAdd(p, (unsigned long long)(long long)d[q][i]);
                d[q][i] = 0;
            }
    };
    if (blockIdx.x < tasks) load(blockIdx.x);
    for (uint64_t first = blockIdx.x; first < tasks; first += (uint64_t)LS_FLUSH * gridDim.x) {
        const uint64_t stop =
            tasks - first < (uint64_t)LS_FLUSH * gridDim.x ? tasks : first + (uint64_t)LS_FLUSH * gridDim.x;
        for (uint64_t task = first; task < stop; task += gridDim.x) {
            fixup(task);
            __syncthreads();  // the previous task's operand reads are done
            uint32_t *lt32 = reinterpret_cast<uint32_t *>(lt);
#pragma unroll
            for (uint32_t v = 0; v < LS_EV; ++v) {
                const uint32_t pc = t + DIAG_WG * v, e = pc / PQ, cb = LS_CB * (pc % PQ);
#pragma unroll
                for (uint32_t w = 0; w < PW; ++w) {
                    uint32_t r[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        r[q] = pw[v][q][w] ^ 0x80808080u;
                        tsum = __builtin_amdgcn_sdot4((int)r[q], 0x01010101, tsum, false);
                    }
                    // 4 x 4 byte transpose: column cb + 4 w + b gets bytes b of rows 0..3
                    const uint32_t lo01 = __byte_perm(r[0], r[1], 0x5140), hi01 = __byte_perm(r[0], r[1], 0x7362);
                    const uint32_t lo23 = __byte_perm(r[2], r[3], 0x5140), hi23 = __byte_perm(r[2], r[3], 0x7362);
                    const uint32_t c0 = cb + 4 * w;
                    lt32[(c0 + 0) * (LS_STRIDE / 4) + e] = __byte_perm(lo01, lo23, 0x5410);
                    lt32[(c0 + 1) * (LS_STRIDE / 4) + e] = __byte_perm(lo01, lo23, 0x7632);
                    lt32[(c0 + 2) * (LS_STRIDE / 4) + e] = __byte_perm(hi01, hi23, 0x5410);
                    lt32[(c0 + 3) * (LS_STRIDE / 4) + e] = __byte_perm(hi01, hi23, 0x7632);
                }
            }
            if (t < 2 * LS_HALO) {
                const uint32_t w4[4] = {ph.x ^ 0x80808080u, ph.y ^ 0x80808080u, ph.z ^ 0x80808080u, ph.w ^ 0x80808080u};
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    lt[(16 * (t % 2) + b) * LS_STRIDE + LS_ROWS + t / 2] = (uint8_t)(w4[b / 4] >> (8 * (b % 4)));
            }
            __syncthreads();
            if (task + gridDim.x < tasks) load(task + gridDim.x);  // in flight during the products
            const uint8_t *cp = lt + col * LS_STRIDE + 16 * h;
            if (F > 0) {
                // all row blocks, tiles wave + 4 q: B words q .. q + 4 shifted by wave bytes; the next
                // block's words are read before this one's products
                uint4 av = *reinterpret_cast<const uint4 *>(cp);
                uint2 ex = *reinterpret_cast<const uint2 *>(cp + 16);
                for (uint32_t rb = 0; rb < LS_ROWS; rb += 32) {
                    const uint32_t w[6] = {av.x, av.y, av.z, av.w, ex.x, ex.y};
                    if (rb + 32 < LS_ROWS) {
                        av = *reinterpret_cast<const uint4 *>(cp + rb + 32);
                        ex = *reinterpret_cast<const uint2 *>(cp + rb + 48);
                    }
                    const v4i a = (v4i){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
#pragma unroll
                    for (int q = 0; q < F; ++q) {
                        v4i b;
#pragma unroll
                        for (int j = 0; j < 4; ++j) b[j] = (int)__builtin_amdgcn_alignbyte(w[q + j + 1], w[q + j], wave);
                        d[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, d[q], 0, 0, 0);
                    }
                }
            }
            if (S > 0) {
                // this wave's quarter of the row blocks, the last S tiles 4 F + j: B words F .. F + 4
                for (uint32_t rb = wave * (LS_ROWS / 4); rb < (wave + 1) * (LS_ROWS / 4); rb += 32) {
                    const uint4 av = *reinterpret_cast<const uint4 *>(cp + rb);
                    const uint4 bw = *reinterpret_cast<const uint4 *>(cp + rb + 4 * F);
                    const uint32_t b4 = *reinterpret_cast<const uint32_t *>(cp + rb + 4 * F + 16);
                    const uint32_t w[5] = {bw.x, bw.y, bw.z, bw.w, b4};
                    const v4i a = (v4i){(int)av.x, (int)av.y, (int)av.z, (int)av.w};
#pragma unroll
                    for (int j = 0; j < S; ++j) {
                        v4i b;
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            b[u] = j == 0 ? (int)w[u] : (int)__builtin_amdgcn_alignbyte(w[u + 1], w[u], j);
                        d[F + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, d[F + j], 0, 0, 0);
                    }
                }
            }
        }
        flush();
    }
    // the bytes' total: sum (x - 128) over the own rows plus 128 per own byte
    unsigned long long nb = 0;
    for (uint64_t tk = blockIdx.x; tk < tasks; tk += gridDim.x) {
        const uint64_t b0 = tk * LS_ROWS * 32, b1 = b0 + LS_ROWS * 32;
        nb += (b1 < n ? b1 : n) - b0;
    }
    long long ws = tsum;
    for (int o = 32; o > 0; o >>= 1) ws += __shfl_down(ws, o, 64);
    if (lane == 0) wred[wave] = ws;
    __syncthreads();  // also: every wave's flush is done
    const unsigned long long tot =
        (unsigned long long)(wred[0] + wred[1] + wred[2] + wred[3]) + 128ull * nb;
    unsigned long long *copy = merge + (size_t)(blockIdx.x % LS_COPIES) * (L + 2);
    for (uint32_t k = t; k <= L; k += DIAG_WG) {
        const unsigned long long v = acc[k] + 256ull * tot;
        if (v) atomicAdd(&copy[k], v);
    }
    if (t == 0 && tot) atomicAdd(&copy[L + 1], tot);
}

// ---- the lag sums past lag 256: windows of lags on 32-byte rows ---------------------------------
//
// One launch per window of lags k_lo .. k_lo + Lw (k_lo a multiple of 32, Lw < LW_WINDOW): the
// products of the kernel above, B taken from the rows k_lo / 32 further on.  A task stages its own
// LW_ROWS rows (region A) and, apart, the rows from k_lo / 32 on that its shifted operands read
// (region B, LW_ROWS + LW_BHALO rows), so a window's LDS does not grow with k_lo.  A window has up
// to 129 tiles: the two waves w and w + 4 take the tiles t = s + 4 f (s = w mod 4: one shift within
// a word for all of them), split near the middle of f, each in items of up to LW_IT consecutive f
// over all the task's rows; at the end of an item its accumulators are added into the LDS lag
// counters (unconditionally: counters for relative lags -32 .. 32 NT - 1).  Each workgroup adds
// its sums plus 256 times its bytes' total into copy b mod DIAG_MERGE of the merge buffer (the
// first window also the total), and lagsum_fix_kernel applies the correction.
constexpr uint32_t LW_ROWS = 1024;
constexpr int LW_WG = 512;
constexpr uint32_t LW_IT = 4;                                 // tiles per item
constexpr uint32_t LW_WINDOW = 4096;                          // lags per window at most
constexpr uint32_t LW_MAX_NT = LW_WINDOW / 32 + 1;            // 129 tiles
constexpr uint32_t LW_MAX_F = (LW_MAX_NT + 3) / 4;            // tiles of one residue mod 4
// B bytes read by an item at f0 (a multiple of 4): 4 f0 + 16 h + up to 32 past the row block
constexpr uint32_t LW_BHALO = 4 * LW_IT * ((LW_MAX_F - 1) / LW_IT) + 48;
// LDS bytes per column: the next odd multiple of 16 above the rows (no bank conflicts between columns)
constexpr uint32_t lw_stride(uint32_t rows) { return (rows / 16 + 1) % 2 ? (rows / 16 + 1) * 16 : (rows / 16 + 2) * 16; }
constexpr uint32_t LW_ASTRIDE = lw_stride(LW_ROWS), LW_BSTRIDE = lw_stride(LW_ROWS + LW_BHALO);
constexpr uint32_t LW_APIECES = LW_ROWS / 4, LW_BPIECES = (LW_ROWS + LW_BHALO) / 4;  // 4 rows x 32 bytes
constexpr uint32_t LW_PV = (LW_APIECES + LW_BPIECES + LW_WG - 1) / LW_WG;  // pieces per thread
static_assert(LW_ROWS % 32 == 0 && (uint64_t)LW_ROWS * 16384 < (1ull << 31), "32-bit accumulators per item");
static_assert((size_t)DIAG_MERGE * (16384 + 2) <= DIAG_MERGE_WORDS, "merge buffer too small");

// bytes of rows 4e .. 4e + 3 (w[r][word], 8 words a row) written transposed: column c of the
// region gets the word of rows 4e..4e+3 at word index e
__device__ inline void ls_put_rows4(uint32_t *region32, uint32_t stride_words, uint32_t e, const uint32_t (&w)[4][8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t lo01 = __byte_perm(w[0][q], w[1][q], 0x5140), hi01 = __byte_perm(w[0][q], w[1][q], 0x7362);
        const uint32_t lo23 = __byte_perm(w[2][q], w[3][q], 0x5140), hi23 = __byte_perm(w[2][q], w[3][q], 0x7362);
        region32[(4 * q + 0) * stride_words + e] = __byte_perm(lo01, lo23, 0x5410);
        region32[(4 * q + 1) * stride_words + e] = __byte_perm(lo01, lo23, 0x7632);
        region32[(4 * q + 2) * stride_words + e] = __byte_perm(hi01, hi23, 0x5410);
        region32[(4 * q + 3) * stride_words + e] = __byte_perm(hi01, hi23, 0x7632);
    }
}

// One item: tiles sh + 4 (f0 + q), q < NV, over all LW_ROWS rows of the staged task (ap: the
// lane's A column at its 16-row half, bp: its B column from byte 4 f0 on, so tile q's B operand is
// the words q .. q + 4 shifted by sh bytes), then its accumulators added into the lag counters
// (diag: the lag counter of d[0][0] for this lane).
template <int NV>
__device__ __forceinline__ void lw_item(const uint8_t *ap, const uint8_t *bp, uint32_t sh, unsigned long long *diag) {
    constexpr int NB = (NV + 7) / 4;  // 16-byte B reads per row block: words 0 .. NV + 3
    v16i d[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) d[q] = (v16i){};
    // row blocks of 32; the next block's words are read before this one's products
    uint4 av = *reinterpret_cast<const uint4 *>(ap);
    uint4 bw[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) bw[u] = *reinterpret_cast<const uint4 *>(bp + 16 * u);
#pragma unroll 2
    for (uint32_t rb = 0; rb < LW_ROWS; rb += 32) {
        uint32_t w[4 * NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) w[4 * u] = bw[u].x, w[4 * u + 1] = bw[u].y, w[4 * u + 2] = bw[u].z, w[4 * u + 3] = bw[u].w;
        const v4i a = (v4i){(int)av.x, (int)av.y, (int)av.z, (int)av.w};
        if (rb + 32 < LW_ROWS) {
            av = *reinterpret_cast<const uint4 *>(ap + rb + 32);
#pragma unroll
            for (int u = 0; u < NB; ++u) bw[u] = *reinterpret_cast<const uint4 *>(bp + rb + 32 + 16 * u);
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            v4i b;
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = (int)__builtin_amdgcn_alignbyte(w[q + j + 1], w[q + j], sh);
            d[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, d[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i) atomicAdd(diag + (128 * q - 8 * (i / 4) - i % 4), (unsigned long long)(long long)d[q][i]);
}

__global__ __launch_bounds__(LW_WG) void lagsum_wide_kernel(const uint8_t *data, uint64_t n, uint32_t Lw,
                                                              uint32_t k_lo, uint32_t L_all,
                                                              unsigned long long *merge) {
    __shared__ __align__(16) uint8_t la[32 * LW_ASTRIDE];
    __shared__ __align__(16) uint8_t lb[32 * LW_BSTRIDE];
    __shared__ unsigned long long cnt_all[32 * LW_MAX_NT + 32];
    __shared__ long long wred[LW_WG / 64];
    const uint32_t NT = (Lw + 31) / 32 + 1;
    unsigned long long *cnt = cnt_all + 32;
    const uint32_t t = threadIdx.x, lane = t % 64, col = lane % 32, h = lane / 32;
    for (uint32_t k = t; k < 32 * NT + 32; k += LW_WG) cnt_all[k] = 0;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(t / 64), sh = wave % 4, half = wave / 4;
    const uint32_t F = NT > sh ? (NT - sh + 3) / 4 : 0;  // tiles sh, sh + 4, ... below NT
    const bool aligned16 = (reinterpret_cast<uintptr_t>(data) & 15) == 0;
    const uint64_t nrows = (n + 31) / 32, tasks = (nrows + LW_ROWS - 1) / LW_ROWS, bshift = k_lo / 32;
    // piece p = t + LW_WG v: rows 4p .. 4p + 3 of region A (p < LW_APIECES), else rows
    // 4 (p - LW_APIECES) .. + 3 of region B; pw[v][row][word]
    uint32_t pw[LW_PV][4][8];
    auto load = [&](uint64_t task) {
#pragma unroll
        for (uint32_t v = 0; v < LW_PV; ++v) {
            const uint32_t p = t + LW_WG * v;
            const uint64_t r0 = p < LW_APIECES ? task * LW_ROWS + 4 * (uint64_t)p
                                               : task * LW_ROWS + bshift + 4 * (uint64_t)(p - LW_APIECES);
            const bool live = p < LW_APIECES + LW_BPIECES;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint4 x = live ? ls_load16(data, n, (r0 + r) * 32 + 16 * q, aligned16, 16) : make_uint4(0, 0, 0, 0);
                    pw[v][r][4 * q + 0] = x.x, pw[v][r][4 * q + 1] = x.y, pw[v][r][4 * q + 2] = x.z, pw[v][r][4 * q + 3] = x.w;
                }
        }
    };
    int tsum = 0;  // this thread's share of sum (x - 128) over the tasks' own rows
    if (blockIdx.x < tasks) load(blockIdx.x);
    for (uint64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
        __syncthreads();  // the previous task's operand reads are done
#pragma unroll
        for (uint32_t v = 0; v < LW_PV; ++v) {
            const uint32_t p = t + LW_WG * v;
            if (p < LW_APIECES) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < 8; ++q) tsum = __builtin_amdgcn_sdot4((int)pw[v][r][q], 0x01010101, tsum, false);
                ls_put_rows4(reinterpret_cast<uint32_t *>(la), LW_ASTRIDE / 4, p, pw[v]);
            } else if (p < LW_APIECES + LW_BPIECES) {
                ls_put_rows4(reinterpret_cast<uint32_t *>(lb), LW_BSTRIDE / 4, p - LW_APIECES, pw[v]);
            }
        }
        __syncthreads();
        if (task + gridDim.x < tasks) load(task + gridDim.x);  // in flight during the products
        // this wave's tiles sh + 4 f for f in [fs, fe): the two waves of a shift split its F tiles near
        // the middle, at a multiple of 4 (16-byte aligned B reads), in items of up to LW_IT
        const uint8_t *ap = la + col * LW_ASTRIDE + 16 * h;
        const uint32_t fsplit = 4 * ((F + 4) / 8), fs = half ? fsplit : 0, fe = half ? F : fsplit;
        for (uint32_t f0 = fs; f0 < fe; f0 += LW_IT) {
            const uint32_t nv = fe - f0 < LW_IT ? fe - f0 : LW_IT;
            const uint8_t *bp = lb + col * LW_BSTRIDE + 16 * h + 16 * (f0 / 4);  // 16-byte aligned
            unsigned long long *diag = cnt + 32 * (sh + 4 * f0) + (int)col - 4 * (int)h;
            static_assert(LW_IT == 4, "one instantiation per item width");
            switch (nv) {
                case 4: lw_item<4>(ap, bp, sh, diag); break;
                case 3: lw_item<3>(ap, bp, sh, diag); break;
                case 2: lw_item<2>(ap, bp, sh, diag); break;
                default: lw_item<1>(ap, bp, sh, diag); break;
            }
        }
    }
    // the bytes' total: sum (x - 128) over the own rows plus 128 per own byte
    unsigned long long nb = 0;
    for (uint64_t tk = blockIdx.x; tk < tasks; tk += gridDim.x) {
        const uint64_t b0 = tk * LW_ROWS * 32, b1 = b0 + LW_ROWS * 32;
        nb += (b1 < n ? b1 : n) - b0;
    }
    long long ws = tsum;
    for (int o = 32; o > 0; o >>= 1) ws += __shfl_down(ws, o, 64);
    if (lane == 0) wred[wave] = ws;
    __syncthreads();  // also: every wave's counter adds are done
    long long all = 0;
#pragma unroll
    for (int w = 0; w < LW_WG / 64; ++w) all += wred[w];
    const unsigned long long tot = (unsigned long long)all + 128ull * nb;
    // copy layout: lags 0..L_all, then the byte total (added by the first window only)
    unsigned long long *copy = merge + (size_t)(blockIdx.x % DIAG_MERGE) * (L_all + 2);
    for (uint32_t r = t; r <= Lw; r += LW_WG) {
        const unsigned long long v = cnt[r] + 256ull * tot;
        if (v) atomicAdd(&copy[k_lo + r], v);
    }
    if (k_lo == 0 && t == 0 && tot) atomicAdd(&copy[L_all + 1], tot);
}

// The correction for L <= 256 (one window, one workgroup of LS_FIX_WG threads): thread k takes
// lag k, sums its LS_COPIES merge copies (all loads issued before the first is used) and clears
// them; the first and last L bytes are loaded at the same time, and P_k + Q_k comes from one scan
// of x_j + x_{n-1-j} (a wave scan by shuffles, then the wave totals through LDS).
constexpr int LS_FIX_WG = 512;
static_assert(LS_FIX_WG > 32 * (LS_MAX_NT - 1) && LS_FIX_WG >= (int)LS_COPIES, "a thread per lag and per copy");
__global__ __launch_bounds__(LS_FIX_WG) void lagsum_fix_small_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                                     unsigned long long *merge,
                                                                     unsigned long long *sums,
                                                                     unsigned long long *total) {
    __shared__ uint32_t wsum[LS_FIX_WG / 64];
    __shared__ unsigned long long tsum[LS_FIX_WG / 64];
    const uint32_t k = threadIdx.x, lane = k % 64, wave = k / 64;
    const size_t cs = (size_t)L + 2;  // copy stride: lags 0..L, then the byte total
    unsigned long long part[LS_COPIES];
#pragma unroll
    for (uint32_t c = 0; c < LS_COPIES; ++c) part[c] = k <= L ? merge[c * cs + k] : 0ull;
    unsigned long long tc = k < LS_COPIES ? merge[k * cs + L + 1] : 0ull;
    const uint32_t x = k < L && k < n ? (uint32_t)data[k] + data[n - 1 - k] : 0u;  // j = k < L <= 256
    // inclusive scan of x over the block
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if ((int)lane >= o) inc += y;
    }
    for (int o = 32; o > 0; o >>= 1) tc += __shfl_down(tc, o, 64);
    if (lane == 63) wsum[wave] = inc;
    if (lane == 0) tsum[wave] = tc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (uint32_t w = 0; w < LS_FIX_WG / 64; ++w) before += w < wave ? wsum[w] : 0u;
    if (k <= L) {
        // P_k + Q_k: the bytes j < k of both ends
        const unsigned long long pq = before + inc - x;
        unsigned long long raw = 0;
#pragma unroll
        for (uint32_t c = 0; c < LS_COPIES; ++c) {
            raw += part[c];
            merge[c * cs + k] = 0;
        }
        const unsigned long long m = k < n ? n - k : 0;
        sums[k] = raw - 128ull * pq - 16384ull * m;
    }
    if (k < LS_COPIES) merge[k * cs + L + 1] = 0;
    if (k == 0 && total) {
        unsigned long long tt = 0;
        for (uint32_t w = 0; w < LS_FIX_WG / 64; ++w) tt += tsum[w];
        *total = tt;
    }
}

// S_k = raw_k - 128 (P_k + Q_k) - 16384 max(n - k, 0) for k <= L, raw_k the sum of the merge
// copies (cleared here for the next call), P_k and Q_k the sums of the first and the last min(k, n)
// bytes.  Workgroup b takes lags kb = FIX_LAGS b .. kb + FIX_LAGS - 1, a lag per thread: it adds
// up the first and the last min(kb, n) bytes (16-byte loads where aligned), then scans
// x_j + x_{n-1-j} over its own lags (a wave scan by shuffles, the wave totals through LDS); every
// load of a thread is issued before the first is used.  The first workgroup also writes the
// byte total when asked for.
constexpr int FIX_LAGS = DIAG_WG;

// sum of data[lo, hi) over the block: each thread adds its 16-byte chunks and the unaligned ends
__device__ inline unsigned long long fix_range_part(const uint8_t *data, uint64_t lo, uint64_t hi) {
    if (lo >= hi) return 0;
    const uintptr_t base = reinterpret_cast<uintptr_t>(data);
    uint64_t a = ((base + lo + 15) & ~(uintptr_t)15) - base;  // first 16-byte aligned index >= lo
    if (a > hi) a = hi;
    uint64_t z = ((base + hi) & ~(uintptr_t)15) - base;        // last aligned index <= hi
    if (z < a) z = a;
    unsigned long long s = 0;
    const uint32_t t = threadIdx.x;
    if (t < a - lo) s += data[lo + t];   // head, under 16 bytes
    if (t < hi - z) s += data[z + t];    // tail, under 16 bytes
    constexpr int U = 4;                 // chunks in flight per thread
    for (uint64_t c0 = a + 16 * (uint64_t)t; c0 < z; c0 += (uint64_t)16 * DIAG_WG * U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t c = c0 + (uint64_t)16 * DIAG_WG * u;
            v[u] = c < z ? *reinterpret_cast<const uint4 *>(data + c) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            s += __builtin_amdgcn_udot4(v[u].x, 0x01010101u, 0u, false) + __builtin_amdgcn_udot4(v[u].y, 0x01010101u, 0u, false) +
                 __builtin_amdgcn_udot4(v[u].z, 0x01010101u, 0u, false) + __builtin_amdgcn_udot4(v[u].w, 0x01010101u, 0u, false);
    }
    return s;
}

__global__ __launch_bounds__(DIAG_WG) void lagsum_fix_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                             unsigned long long *merge, unsigned long long *sums,
                                                             unsigned long long *total) {
    __shared__ unsigned long long wtot[DIAG_WG / 64];
    __shared__ uint32_t wscan[DIAG_WG / 64];
    const uint32_t t = threadIdx.x, lane = t % 64, wave = t / 64;
    const uint32_t kb = blockIdx.x * FIX_LAGS, k = kb + t;
    const size_t cs = (size_t)L + 2;  // copy stride: lags 0..L, then the byte total
    unsigned long long part[DIAG_MERGE], tc = 0;
#pragma unroll
    for (int c = 0; c < DIAG_MERGE; ++c) part[c] = k <= L ? merge[c * cs + k] : 0ull;
    if (blockIdx.x == 0 && t < DIAG_MERGE) tc = merge[t * cs + L + 1];
    const uint32_t x = k < L && k < n ? (uint32_t)data[k] + data[n - 1 - k] : 0u;  // j = k, for the lags above k
    const uint64_t m = kb < n ? kb : n;
    unsigned long long base = fix_range_part(data, 0, m) + fix_range_part(data, n - m, n);
    // the block's sums: base over all threads, wave scans of x
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if ((int)lane >= o) inc += y;
    }
    for (int o = 32; o > 0; o >>= 1) base += __shfl_down(base, o, 64);
    for (int o = 32; o > 0; o >>= 1) tc += __shfl_down(tc, o, 64);
    if (lane == 63) wscan[wave] = inc;
    if (lane == 0) wtot[wave] = base;
    __syncthreads();
    unsigned long long pq = 0;  // P_k + Q_k: the bytes j < k of both ends
#pragma unroll
    for (uint32_t w = 0; w < DIAG_WG / 64; ++w) pq += wtot[w] + (w < wave ? wscan[w] : 0u);
    pq += inc - x;
    if (k <= L) {
        unsigned long long raw = 0;
#pragma unroll
        for (int c = 0; c < DIAG_MERGE; ++c) {
            raw += part[c];
            merge[c * cs + k] = 0;
        }
        const unsigned long long mk = k < n ? n - k : 0;
        sums[k] = raw - 128ull * pq - 16384ull * mk;
    }
    if (blockIdx.x == 0) {
        if (t < DIAG_MERGE) merge[t * cs + L + 1] = 0;
        if (t == 0 && total) *total = tc;
    }
}

// ---- entropy and the normalised 1-D autocorrelation -------------------------------------


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

// r_k for k = 0..L of a byte sequence x_0..x_{n-1} with mean m:
//   r_k = sum_{i<n-k} (x_i - m)(x_{i+k} - m) / sum_i (x_i - m)^2
//       = (S_k - m (A_k + B_k) + (n-k) m^2) / (S_0 - n m^2),
// A_k = sum_{i<n-k} x_i = T - (sum of the last k bytes), B_k = sum_{i>=k} x_i = T - (sum of the first k bytes).
// One workgroup scans the first and last L bytes in chunks of 256.
__global__ __launch_bounds__(DIAG_WG) void autocorr_norm_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                                 const unsigned long long *sums,
                                                                 const unsigned long long *total, double *r) {
    __shared__ unsigned long long sh[DIAG_WG], st[DIAG_WG];
    const unsigned long long T = *total;
    const double m = (double)T / (double)n;
    const double den = (double)sums[0] - (double)n * m * m;
    // no coefficient when every byte is equal (or there are none): n S_0 = T^2 exactly then, and
    // only then (the equality case of Cauchy-Schwarz), compared in 128-bit integers
    const bool constant = n == 0 || (unsigned __int128)n * sums[0] == (unsigned __int128)T * T;
    unsigned long long carry_h = 0, carry_t = 0;
    if (threadIdx.x == 0) r[0] = constant ? __builtin_nan("") : 1.0;
    for (uint32_t c = 0; c < L; c += DIAG_WG) {
        const uint64_t i = (uint64_t)c + threadIdx.x;  // k = i + 1 includes byte i of the head / tail
        sh[threadIdx.x] = i < n ? data[i] : 0;
        st[threadIdx.x] = i < n ? data[n - 1 - i] : 0;
        __syncthreads();
        for (int s = 1; s < DIAG_WG; s <<= 1) {  // inclusive scans
            const unsigned long long a = threadIdx.x >= (unsigned)s ? sh[threadIdx.x - s] : 0;
            const unsigned long long b = threadIdx.x >= (unsigned)s ? st[threadIdx.x - s] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            st[threadIdx.x] += b;
            __syncthreads();
        }
        const uint64_t k = i + 1;
        if (k <= L) {
            double v;
            if (constant) {
                v = __builtin_nan("");
            } else if (k >= n) {
                v = 0.0;
            } else {
                const double Ak = (double)(T - (carry_t + st[threadIdx.x]));
                const double Bk = (double)(T - (carry_h + sh[threadIdx.x]));
                v = ((double)sums[k] - m * (Ak + Bk) + (double)(n - k) * m * m) / den;
            }
            r[k] = v;
        }
        carry_h += sh[DIAG_WG - 1];
        carry_t += st[DIAG_WG - 1];
        __syncthreads();
    }
}

// ---- 2-D discrete Fourier transform as two passes ----------------------------------------
//
// One pass applies the N-point DFT along the rows index of an N x M matrix and
// writes the result transposed:  dst[c][r] = sum_k e^{sign 2 pi i r k / N} src[k][c].
// Two passes (first along the H rows of the H x W image, then along its W
// columns) give the 2-D DFT in natural layout.  Every size is allowed (no
// power-of-two restriction); the twiddle index r k mod N is kept exact in
// integers, so every twiddle is one table entry.

constexpr int DFT_T = 64;  // output tile edge (r and c)
constexpr int DFT_K = 16;  // k values per LDS stage

// tw[j] = (cos 2 pi j / N, sin 2 pi j / N)
__global__ void twiddle_kernel(double2 *tw, uint32_t N) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s, c;
    sincospi(2.0 * (double)j / (double)N, &s, &c);
    tw[j] = make_double2(c, s);
}

__device__ __forceinline__ double2 dft_value(uint8_t v) { return make_double2((double)v, 0.0); }
__device__ __forceinline__ double2 dft_value(double v) { return make_double2(v, 0.0); }
__device__ __forceinline__ double2 dft_value(double2 v) { return v; }

// The pass runs on the matrix cores: binary64 MFMA 16x16x4 (v_mfma_f64_16x16x4f64), operand
// layout: lane i holds A[i % 16][i / 16] and B[i / 16][i % 16] of the 16x4 and 4x16 operands,
// and D[4 j + i / 16][i % 16] in its j-th accumulator.  A complex product takes four real
// products: re += wr xr - wi xi, im += wr xi + wi xr.  The inputs and twiddles of the next
// 16-deep k stage are loaded into registers while the current stage computes; the loads are
// unconditional, from valid addresses, so nothing waits for them before the stage's products,
// and out-of-range entries are zeroed when stored to LDS.
typedef double v4d __attribute__((ext_vector_type(4)));

// What a pass writes for output (column c, index r) of its transforms, row-major in its
// M x nout output: the complex value, |Z|^2, |Z|^2 with the zero frequency (c = r = 0 of the
// second pass) set to 0, or Re Z / den (the normalised autocorrelation; NaN when den is).
// A real matrix (h rows) has a Hermitian 2-D transform, Z[h - k1][w - k2] = conj Z[k1][k2]
// (indices mod h and w), so a first pass over real columns keeps only indices r < nout =
// h/2 + 1 of each column's transform, the second pass transforms those h/2 + 1 columns, and
// its real results (|Z|^2, or Re Z of an even real matrix's transform) are written twice:
// row c, and, as row h - c with k2 -> w - k2, each row the pass does not compute itself
// (mirror = h; 0 writes no mirror rows).
enum : int { EPI_COMPLEX = 0, EPI_POWER = 1, EPI_POWER_NODC = 2, EPI_ACF = 3 };
struct PassOut {
    double2 *z;
    double *p;
    const double *den;
    uint32_t nout;
    uint32_t mirror;
};

template <int E>
__device__ __forceinline__ void pass_store(const PassOut &o, uint32_t c, uint32_t r, uint32_t N, uint32_t M,
                                           double re, double im) {
    if (r >= o.nout) return;
    const size_t i = (size_t)c * o.nout + r;
    if constexpr (E == EPI_COMPLEX) {
        o.z[i] = make_double2(re, im);
    } else {
        double v;
        if constexpr (E == EPI_ACF) {
            const double d = o.den[0];
            v = d != d ? d : re / d;
        } else {
            v = (E == EPI_POWER_NODC && c == 0 && r == 0) ? 0.0 : re * re + im * im;
        }
        o.p[i] = v;
        // the real outputs keep whole rows (nout = N)
        if (o.mirror && c != 0 && o.mirror - c >= M) o.p[(size_t)(o.mirror - c) * N + (r ? N - r : 0)] = v;
    }
}

template <typename In, int E, int TR>
__global__ __launch_bounds__(DIAG_WG) void dft_pass_kernel(const In *src, uint32_t N, uint32_t M, const double2 *tw,
                                                            double sign, PassOut dst) {
    // TR x 64 outputs per workgroup: with TR = 64 each wave takes a 32 x 32 block as 2 x 2 tiles of
    // 16 x 16, with TR = 32 (grids that would not fill the chip) a 32 x 16 block as 2 x 1 tiles.
    // A real input (bytes or doubles) has no imaginary part: two of the four products are skipped.
    static_assert(TR == 64 || TR == 32, "tile height");
    constexpr int WC = TR == 64 ? 2 : 4;             // waves across the tile's columns
    constexpr int TB = 4 / WC;                       // column tiles per wave
    constexpr bool REAL = !std::is_same_v<In, double2>;
    constexpr int TWQ = TR * DFT_K / DIAG_WG;        // twiddles each thread stages per k stage
    __shared__ double2 s_src[DFT_K][DFT_T];  // [k][c]
    __shared__ double2 s_tw[DFT_K][TR];      // [k][r]
    const uint32_t r0 = blockIdx.x * TR, c0 = blockIdx.y * DFT_T;
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const uint32_t wr = (wave / WC) * 32, wc = (wave % WC) * (16 * TB);
    const uint32_t li = lane % 16, lk = lane / 16;
    // staging: column cc of the input tile for k rows kq + 4q; twiddle row tr_s for k rows kt + (DFT_K/TWQ) q
    const uint32_t cc = threadIdx.x % DFT_T, kq = threadIdx.x / DFT_T;
    const uint32_t tr_s = threadIdx.x % TR, kt = threadIdx.x / TR;
    const uint32_t rs = r0 + tr_s;
    const uint32_t rmod = rs < N ? rs : 0;
    const uint32_t cs = c0 + cc < M ? c0 + cc : M - 1;
    uint32_t off[TWQ];
    for (int q = 0; q < TWQ; ++q) off[q] = (uint32_t)(((uint64_t)rmod * (kt + (DFT_K / TWQ) * q)) % N);
    const uint32_t step = (uint32_t)(((uint64_t)rmod * DFT_K) % N);
    uint32_t base = 0;
    In nx[4];
    double2 nw[TWQ];
    auto fetch = [&](uint32_t k0) {
        for (int q = 0; q < 4; ++q) {
            const uint32_t k = k0 + kq + 4 * q;
            nx[q] = src[(size_t)(k < N ? k : N - 1) * M + cs];
        }
        for (int q = 0; q < TWQ; ++q) {
            uint32_t j = base + off[q];
            if (j >= N) j -= N;
            nw[q] = tw[j];
        }
        base += step;
        if (base >= N) base -= N;
    };
    v4d re[2][TB], im[2][TB];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < TB; ++b) re[a][b] = im[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (uint32_t k0 = 0; k0 < N; k0 += DFT_K) {
        for (int q = 0; q < 4; ++q) {
            const uint32_t k = k0 + kq + 4 * q;
            s_src[kq + 4 * q][cc] = (k < N && c0 + cc < M) ? dft_value(nx[q]) : make_double2(0.0, 0.0);
        }
        for (int q = 0; q < TWQ; ++q) {
            const uint32_t kk = kt + (DFT_K / TWQ) * q, k = k0 + kk;
            s_tw[kk][tr_s] = (k < N && rs < N) ? make_double2(nw[q].x, sign * nw[q].y) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (k0 + DFT_K < N) fetch(k0 + DFT_K);
#pragma unroll
        for (int k4 = 0; k4 < DFT_K / 4; ++k4) {
            const int k = 4 * k4 + (int)lk;
            double2 w[2], x[TB];
            for (int t = 0; t < 2; ++t) w[t] = s_tw[k][wr + 16 * t + li];
            for (int t = 0; t < TB; ++t) x[t] = s_src[k][wc + 16 * t + li];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < TB; ++b) {
                    re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[a].x, x[b].x, re[a][b], 0, 0, 0);
                    if constexpr (!REAL) {
                        re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-w[a].y, x[b].y, re[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[a].x, x[b].y, im[a][b], 0, 0, 0);
                    }
                    im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[a].y, x[b].x, im[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < TB; ++b)
            for (int j = 0; j < 4; ++j) {
                const uint32_t r = r0 + wr + 16 * a + 4 * j + lk, c = c0 + wc + 16 * b + li;
                if (r < N && c < M) pass_store<E>(dst, c, r, N, M, re[a][b][j], im[a][b][j]);
            }
}

// ---- the same pass by FFT, for power-of-two lengths -------------------------------------
//
// For N = 2^p <= FFT_MAX the pass uses Stockham autosort stages (the self-sorting
// FFT): with stride s and n = N / s, a radix-r stage reads the r values
// x[q + s (j + l n / r)], l < r, takes their r-point DFT, multiplies output k by
// W_n^{j k} and writes it to x[q + s (r j + k)], so the result ends in natural
// order.  Radix-4 stages, after one radix-2 stage when p is odd.  A workgroup
// transforms C adjacent columns in LDS: each input row is read as C contiguous
// elements and each output row (one column's transform) is written contiguously.
// Each workgroup computes W^b, b < N/4 (W = e^{sign 2 pi i / N}), into LDS while its
// input loads are in flight; the stages' other twiddles follow exactly, as
// W^{a N/4 + b} = (sign i)^a W^b.  About 2.1 p flops per value instead of the
// direct pass's 8 N.
constexpr uint32_t FFT_MAX = 4096;
constexpr uint32_t FFT_PP_MAX = 1024;             // two LDS copies of the columns up to this length (36 KB)
constexpr uint32_t FFT_WG_ELEMS = 1024;           // complex values per workgroup when N <= 1024 (16 KB of LDS)
constexpr int FFT_EPT = FFT_MAX / DIAG_WG;        // values per thread, at most
constexpr int FFT_B2 = FFT_MAX / 2 / DIAG_WG;     // radix-2 butterflies per thread, at most
constexpr int FFT_B4 = FFT_MAX / 4 / DIAG_WG;     // radix-4 butterflies per thread per stage, at most

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

__host__ __device__ constexpr uint32_t fft_twiddles(uint32_t N) { return N < 4 ? 1 : N / 4; }

// W^j for j < 3N/4 from the quarter table q[b] = W^b: multiplying by W^{N/4} = sign i is exact.
__device__ __forceinline__ double2 fft_twiddle(const double2 *q, uint32_t j, uint32_t logN, double sign) {
    if (logN < 2) return make_double2(1.0, 0.0);  // N <= 2 uses j = 0 only
    const double2 w = q[j & ((1u << (logN - 2)) - 1)];
    switch (j >> (logN - 2)) {
        case 0: return w;
        case 1: return make_double2(-sign * w.y, sign * w.x);
        default: return make_double2(-w.x, -w.y);
    }
}

template <typename In, int E>
__global__ __launch_bounds__(DIAG_WG) void fft_pass_kernel(const In *src, uint32_t N, uint32_t M, uint32_t logN,
                                                            uint32_t C, double sign, PassOut dst) {
    // C columns of N values (twice when N <= FFT_PP_MAX: each stage reads one copy and writes the
    // other, so it needs one barrier instead of two), then the twiddles
    extern __shared__ double2 fbuf[];
    const bool pp = N <= FFT_PP_MAX;
    double2 *cur = fbuf, *nxt = fbuf + (pp ? (size_t)C * N : 0);
    double2 *ftw = fbuf + (size_t)(pp ? 2 : 1) * C * N;
    // consecutive column groups on the same XCD (workgroups are dealt to the 8 XCDs in turn),
    // so the partly shared cache lines of neighbouring groups meet in one L2
    uint32_t g = blockIdx.x;
    if (gridDim.x % 8 == 0) g = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t c0 = g * C;
    const uint32_t cols = M - c0 < C ? M - c0 : C;
    const uint32_t total = cols * N;
    {
        // all of a thread's loads are issued before the first is stored, and the twiddles
        // (the values the table kernel computes: sincospi of 2j / N) are made meanwhile
        In v[FFT_EPT];
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                v[i] = src[(size_t)k * M + c0 + cl];
            }
        }
        for (uint32_t j = threadIdx.x; j < fft_twiddles(N); j += DIAG_WG) {
            double sn, cs;
            sincospi(2.0 * (double)j / (double)N, &sn, &cs);
            ftw[j] = make_double2(cs, sign * sn);
        }
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                cur[cl * N + k] = dft_value(v[i]);
            }
        }
    }
    __syncthreads();
    uint32_t st = 0;  // log2 of the stride s
    if (logN & 1) {
        // radix-2 stage, s = 1: x[j], x[j + N/2] -> x[2j], x[2j + 1]
        const uint32_t half = N >> 1, nb = cols * half;
        double2 a[FFT_B2], b[FFT_B2];
#pragma unroll
        for (int i = 0; i < FFT_B2; ++i) {
            const uint32_t u = threadIdx.x + i * DIAG_WG;
            if (u < nb) {
                const double2 *x = cur + (u >> (logN - 1)) * N;
                const uint32_t j = u & (half - 1);
                a[i] = x[j];
                b[i] = x[j + half];
            }
        }
        if (!pp) __syncthreads();
#pragma unroll
        for (int i = 0; i < FFT_B2; ++i) {
            const uint32_t u = threadIdx.x + i * DIAG_WG;
            if (u < nb) {
                double2 *x = nxt + (u >> (logN - 1)) * N;
                const uint32_t j = u & (half - 1);
                x[2 * j] = cadd(a[i], b[i]);
                x[2 * j + 1] = cmul(csub(a[i], b[i]), fft_twiddle(ftw, j, logN, sign));
            }
        }
        __syncthreads();
        double2 *t = cur;
        cur = nxt;
        nxt = t;
        st = 1;
    }
    const uint32_t quarter = N >> 2, nb4 = cols * quarter;
    for (; st < logN; st += 2) {
        const uint32_t s = 1u << st, m = N >> (st + 2);
        double2 a[FFT_B4][4];
#pragma unroll
        for (int i = 0; i < FFT_B4; ++i) {
            const uint32_t u = threadIdx.x + i * DIAG_WG;
            if (u < nb4) {
                const double2 *x = cur + (u >> (logN - 2)) * N;
                const uint32_t t = u & (quarter - 1), q = t & (s - 1), j = t >> st;
#pragma unroll
                for (int l = 0; l < 4; ++l) a[i][l] = x[q + s * (j + l * m)];
            }
        }
        if (!pp) __syncthreads();
#pragma unroll
        for (int i = 0; i < FFT_B4; ++i) {
            const uint32_t u = threadIdx.x + i * DIAG_WG;
            if (u < nb4) {
                double2 *x = nxt + (u >> (logN - 2)) * N;
                const uint32_t t = u & (quarter - 1), q = t & (s - 1), j = t >> st;
                const double2 t0 = cadd(a[i][0], a[i][2]), t1 = csub(a[i][0], a[i][2]);
                const double2 t2 = cadd(a[i][1], a[i][3]), t3 = csub(a[i][1], a[i][3]);
                const double2 rt3 = make_double2(-sign * t3.y, sign * t3.x);  // W_4 t3, W_4 = sign i
                const uint32_t w = t - q;                                    // j s: W_n^{j k} = table[j s k]
                x[q + s * (4 * j)] = cadd(t0, t2);
                x[q + s * (4 * j + 1)] = cmul(cadd(t1, rt3), fft_twiddle(ftw, w, logN, sign));
                x[q + s * (4 * j + 2)] = cmul(csub(t0, t2), fft_twiddle(ftw, 2 * w, logN, sign));
                x[q + s * (4 * j + 3)] = cmul(csub(t1, rt3), fft_twiddle(ftw, 3 * w, logN, sign));
            }
        }
        __syncthreads();
        double2 *t = cur;
        cur = nxt;
        nxt = t;
    }
    for (uint32_t e = threadIdx.x; e < total; e += DIAG_WG) {
        const double2 v = cur[e];
        pass_store<E>(dst, c0 + (e >> logN), e & (N - 1), N, M, v.x, v.y);
    }
}

// ---- the same pass by mixed-radix FFT, for lengths 2^a 3^b 5^c --------------------------
//
// ---- 1024-point pass: one wave per column, three register stages -----------------------
//
// With n = t + 64 j and k = k1 + 16 k2 (t, k2 < 64; j, k1 < 16),
//   X[k1 + 16 k2] = sum_t W_64^{t k2} [W_1024^{t k1} sum_j x[t + 64 j] W_16^{j k1}],
// and the 64-point DFTs over t split again as t = a + 4 b, k2 = c + 16 d (a, d < 4; b, c < 16):
//   Y[c + 16 d] = sum_a W_4^{a d} [W_64^{a c} sum_b y[a + 4 b] W_16^{b c}].
// Lane t of a column's wave loads x[t + 64 j] (16 values), takes their 16-point DFT in registers
// and the twiddles W_1024^{t k1}; through LDS, lane (k1, a) = (t / 4, t % 4) takes the 16 values
// y[a + 4 b] of its k1, their 16-point DFT and the twiddles W_64^{a c}; through LDS again, each
// lane takes four 4-point DFTs over a and stores X[k1 + 16 c + 256 d], 64 consecutive outputs per
// store.  The LDS row strides (68 and 258 entries of 16 bytes) put the 8 lanes of each 128-byte
// LDS cycle on distinct banks in every exchange.  The workgroup makes the quarter twiddle table
// W^b, b < 256, while its loads are in flight.  A 16-point DFT is 4 x 4: 4-point DFTs, the
// twiddles W_16^{n2 k1}, 4-point DFTs.
constexpr uint32_t FFT1K = 1024;
constexpr int FFT1K_COLS = DIAG_WG / 64;  // columns per workgroup, one per wave
constexpr int FFT1K_S1 = 68;              // LDS row stride of the stage-1 output (rows k1)
constexpr int FFT1K_S2 = 258;             // LDS row stride of the stage-2 output (rows a)
constexpr int FFT1K_WAVE = 16 * FFT1K_S1; // LDS entries per wave (the stage-2 output fits in them)

static_assert(DIAG_WG == FFT1K / 4, "one quarter-table entry per thread");

// Orders a wave's LDS accesses before and after this point for the compiler; the wave's own
// LDS operations complete in order, so its lanes then see each other's stores.
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr size_t fft1k_lds() { return ((size_t)FFT1K_COLS * FFT1K_WAVE + FFT1K / 4) * 16; }

// z (sign i)^q
__device__ __forceinline__ double2 rot_q(double2 z, uint32_t q, double sign) {
    switch (q & 3) {
        case 0: return z;
        case 1: return make_double2(-sign * z.y, sign * z.x);
        case 2: return make_double2(-z.x, -z.y);
        default: return make_double2(sign * z.y, -sign * z.x);
    }
}

// W^j, j < 1024, from the quarter table q[b] = W^b (b < 256)
__device__ __forceinline__ double2 tw1k(const double2 *q, uint32_t j, double sign) {
    return rot_q(q[j & 255], j >> 8, sign);
}

__device__ __forceinline__ void dft4(double2 &a0, double2 &a1, double2 &a2, double2 &a3, double sign) {
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot_q(csub(a1, a3), 1, sign);
    a0 = cadd(t0, t2);
    a1 = cadd(t1, t3);
    a2 = csub(t0, t2);
    a3 = csub(t1, t3);
}

// v[k] <- sum_n v[n] W_16^{n k}, W_16 = e^{sign 2 pi i / 16}
__device__ __forceinline__ void dft16(double2 (&v)[16], double sign) {
    constexpr double C1 = 0.92387953251128674;  // cos(pi / 8)
    constexpr double S1 = 0.38268343236508977;  // sin(pi / 8)
    constexpr double R2 = 0.70710678118654752;  // cos(pi / 4)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2], sign);
    // v[4 k1 + n2] now holds A[n2][k1]; twiddles W_16^{n2 k1}
    v[5] = cmul(v[5], make_double2(C1, sign * S1));     // n2 = 1, k1 = 1
    v[9] = cmul(v[9], make_double2(R2, sign * R2));     // 1, 2
    v[13] = cmul(v[13], make_double2(S1, sign * C1));   // 1, 3
    v[6] = cmul(v[6], make_double2(R2, sign * R2));     // 2, 1
    v[10] = rot_q(v[10], 1, sign);                      // 2, 2
    v[14] = cmul(v[14], make_double2(-R2, sign * R2));  // 2, 3
    v[7] = cmul(v[7], make_double2(S1, sign * C1));     // 3, 1
    v[11] = cmul(v[11], make_double2(-R2, sign * R2));  // 3, 2
    v[15] = cmul(v[15], make_double2(-C1, -sign * S1)); // 3, 3
    double2 u[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        double2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
        dft4(a0, a1, a2, a3, sign);
        u[k1] = a0;
        u[k1 + 4] = a1;
        u[k1 + 8] = a2;
        u[k1 + 12] = a3;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = u[k];
}

template <typename In, int E>
__global__ __launch_bounds__(DIAG_WG) void fft1k_pass_kernel(const In *src, uint32_t M, double sign, PassOut dst) {
    extern __shared__ double2 fbuf[];
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    double2 *L = fbuf + (size_t)wave * FFT1K_WAVE;
    double2 *q = fbuf + (size_t)FFT1K_COLS * FFT1K_WAVE;
    // consecutive column groups on the same XCD (workgroups are dealt to the 8 XCDs in turn)
    uint32_t g = blockIdx.x;
    if (gridDim.x % 8 == 0) g = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t col = g * FFT1K_COLS + wave;
    const bool live = col < M;
    In x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j)
        if (live) x[j] = src[(size_t)(lane + 64 * j) * M + col];
    {
        double sn, cs;
        sincospi(2.0 * (double)threadIdx.x / (double)FFT1K, &sn, &cs);
        q[threadIdx.x] = make_double2(cs, sign * sn);
    }
    __syncthreads();
    if (!live) return;
    double2 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = dft_value(x[j]);
    // stage 1: 16-point DFT over j, twiddles W^{t k1}
    dft16(v, sign);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) L[k1 * FFT1K_S1 + lane] = k1 ? cmul(v[k1], tw1k(q, lane * k1, sign)) : v[0];
    wave_fence();
    // stage 2: lane (k1, a) takes y[a + 4 b][k1], a 16-point DFT over b, twiddles W_64^{a c}
    const uint32_t k1 = lane >> 2, a = lane & 3;
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = L[k1 * FFT1K_S1 + a + 4 * b];
    wave_fence();
    dft16(v, sign);
#pragma unroll
    for (int c = 0; c < 16; ++c)
        L[a * FFT1K_S2 + c * 16 + k1] = (a && c) ? cmul(v[c], tw1k(q, 16 * a * c, sign)) : v[c];
    wave_fence();
    // stage 3: 4-point DFTs over a of pairs p = 16 c + k1 = 64 i + lane; X[p + 256 d]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t p = 64 * i + lane;
        double2 a0 = L[p], a1 = L[FFT1K_S2 + p], a2 = L[2 * FFT1K_S2 + p], a3 = L[3 * FFT1K_S2 + p];
        dft4(a0, a1, a2, a3, sign);
        pass_store<E>(dst, col, p, FFT1K, M, a0.x, a0.y);
        pass_store<E>(dst, col, p + 256, FFT1K, M, a1.x, a1.y);
        pass_store<E>(dst, col, p + 512, FFT1K, M, a2.x, a2.y);
        pass_store<E>(dst, col, p + 768, FFT1K, M, a3.x, a3.y);
    }
}

// Lengths N <= FFT_MAX whose only prime factors are 2, 3 and 5 (and that are not
// powers of two) run as Stockham stages of radix 5, 3, 4 and 2 in turn (the radix
// of each stage in FftPlan).  A radix-R stage with stride s, n = N / s, reads
// x[q + s (j + l n/R)] for l < R, takes their R-point DFT (radix 2 and 4 in
// their exact +-1, +-i form, radix 3 and 5 with W_R^p = W_N^{p N/R} from the
// table), multiplies output k by W_n^{jk} = W_N^{j s k} and writes it to
// x[q + s (R j + k)].  The N-entry table (the twiddle kernel's, sign applied) is
// copied into LDS beside the data; the rest is as in fft_pass_kernel.
struct FftPlan {
    uint32_t nst;
    uint8_t rad[16];
};

template <int R>
__device__ __forceinline__ void mixed_stage(double2 *fbuf, const double2 *ftw, uint32_t N, uint32_t cols,
                                            uint32_t s, double sign) {
    constexpr int BPT = (int)((FFT_MAX / R + DIAG_WG - 1) / DIAG_WG);
    const uint32_t nr = N / R, m = nr / s, nb = cols * nr, step = N / R;
    double2 a[BPT][R];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const uint32_t u = threadIdx.x + i * DIAG_WG;
        if (u < nb) {
            const uint32_t cl = u / nr, t = u - cl * nr, j = t / s, q = t - j * s;
            const double2 *x = fbuf + (size_t)cl * N;
#pragma unroll
            for (int l = 0; l < R; ++l) a[i][l] = x[q + s * (j + l * m)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const uint32_t u = threadIdx.x + i * DIAG_WG;
        if (u < nb) {
            const uint32_t cl = u / nr, t = u - cl * nr, j = t / s, q = t - j * s;
            double2 y[R];
            if constexpr (R == 2) {
                y[0] = cadd(a[i][0], a[i][1]);
                y[1] = csub(a[i][0], a[i][1]);
            } else if constexpr (R == 4) {
                const double2 t0 = cadd(a[i][0], a[i][2]), t1 = csub(a[i][0], a[i][2]);
                const double2 t2 = cadd(a[i][1], a[i][3]), t3 = csub(a[i][1], a[i][3]);
                const double2 rt3 = make_double2(-sign * t3.y, sign * t3.x);  // W_4 t3, W_4 = sign i
                y[0] = cadd(t0, t2);
                y[1] = cadd(t1, rt3);
                y[2] = csub(t0, t2);
                y[3] = csub(t1, rt3);
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    double2 acc = a[i][0];
#pragma unroll
                    for (int l = 1; l < R; ++l)
                        acc = k == 0 ? cadd(acc, a[i][l]) : cadd(acc, cmul(a[i][l], ftw[((l * k) % R) * step]));
                    y[k] = acc;
                }
            }
            double2 *x = fbuf + (size_t)cl * N;
            x[q + s * (R * j)] = y[0];
#pragma unroll
            for (int k = 1; k < R; ++k) x[q + s * (R * j + k)] = cmul(y[k], ftw[j * s * k]);
        }
    }
    __syncthreads();
}

template <typename In, int E>
__global__ __launch_bounds__(DIAG_WG) void fft_mixed_pass_kernel(const In *src, uint32_t N, uint32_t M, uint32_t C,
                                                                  FftPlan plan, const double2 *tw, double sign,
                                                                  PassOut dst) {
    extern __shared__ double2 fbuf[];  // C columns of N values, then the N twiddles
    double2 *ftw = fbuf + (size_t)C * N;
    uint32_t g = blockIdx.x;
    if (gridDim.x % 8 == 0) g = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t c0 = g * C;
    const uint32_t cols = M - c0 < C ? M - c0 : C;
    const uint32_t total = cols * N;
    {
        In v[FFT_EPT];
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                v[i] = src[(size_t)k * M + c0 + cl];
            }
        }
        for (uint32_t j = threadIdx.x; j < N; j += DIAG_WG) {
            const double2 w = tw[j];
            ftw[j] = make_double2(w.x, sign * w.y);
        }
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                fbuf[cl * N + k] = dft_value(v[i]);
            }
        }
    }
    __syncthreads();
    uint32_t s = 1;
    for (uint32_t st = 0; st < plan.nst; ++st) {
        const uint32_t R = plan.rad[st];
        if (R == 5) mixed_stage<5>(fbuf, ftw, N, cols, s, sign);
        else if (R == 3) mixed_stage<3>(fbuf, ftw, N, cols, s, sign);
        else if (R == 4) mixed_stage<4>(fbuf, ftw, N, cols, s, sign);
        else mixed_stage<2>(fbuf, ftw, N, cols, s, sign);
        s *= R;
    }
    for (uint32_t e = threadIdx.x; e < total; e += DIAG_WG) {
        const double2 v = fbuf[e];
        const uint32_t cl = e / N;
        pass_store<E>(dst, c0 + cl, e - cl * N, N, M, v.x, v.y);
    }
}

// n S2 - S1^2 from the histogram (exact: n <= 2^24 keeps both products below 2^64),
// the zero-lag sum of the mean-removed image scaled by n.
__global__ __launch_bounds__(DIAG_WG) void acf2_den_kernel(const unsigned long long *hist, uint64_t n,
                                                            double *den) {
    __shared__ unsigned long long ired[DIAG_WG];
    const unsigned long long v = threadIdx.x, h = hist[threadIdx.x];
    const unsigned long long s1 = block_sum<unsigned long long>(h * v, ired);
    const unsigned long long s2 = block_sum<unsigned long long>(h * v * v, ired);
    if (threadIdx.x == 0) {
        const unsigned long long d = (unsigned long long)n * s2 - s1 * s1;
        den[0] = d == 0 ? __builtin_nan("") : (double)d;
    }
}

}  // namespace
}  // namespace lz

using namespace lz;

namespace {
int diag_begin(lz_ctx *c, hipStream_t s, size_t bytes, char **ws);
int diag_end(lz_ctx *c, hipStream_t s);
}  // namespace

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

namespace {

// The lag sums into sums[0..max_lag]; with total non-null, also the byte total into *total.
// ordered: the caller has already ordered this stream after the context's other diagnostics
// (diag_begin) and records the event afterwards itself.
int lag_sums(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, unsigned long long *sums,
             unsigned long long *total, hipStream_t s, bool ordered = false) {
    if (n > 0) {
        // the workgroups' sums meet in the context's merge copies, which the correction kernel adds
        // up, writes to d_sums and clears: calls on different streams are ordered
        char *ws;
        if (!ordered)
            if (int rc = diag_begin(c, s, 0, &ws)) return rc;
        // resident workgroups only, as many tasks each (rounds = tasks / slots, rounded up)
        auto grid = [&](const void *kern, int wg, uint64_t tasks, unsigned *blocks) -> int {
            int per_cu = 0;
            LZ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, wg, 0));
            if (per_cu < 1) return fail(LZ_E_INVAL, "lag sums need more LDS or registers than the device has");
            const uint64_t slots = (uint64_t)c->dev.cus * (uint64_t)per_cu;
            const uint64_t rounds = (tasks + slots - 1) / slots;
            *blocks = (unsigned)((tasks + rounds - 1) / rounds);
            return LZ_OK;
        };
        unsigned blocks = 0;
        if (max_lag <= 32 * (LS_MAX_NT - 1)) {  // up to 256 lags: one launch
            const uint32_t nt = (max_lag + 31) / 32 + 1;
            void (*kern)(const uint8_t *, uint64_t, uint32_t, unsigned long long *) =
                nt == 1 ? lagsum_small_kernel<1> : nt == 2 ? lagsum_small_kernel<2> : nt == 3 ? lagsum_small_kernel<3>
                : nt == 4 ? lagsum_small_kernel<4> : nt == 5 ? lagsum_small_kernel<5> : nt == 6 ? lagsum_small_kernel<6>
                : nt == 7 ? lagsum_small_kernel<7> : nt == 8 ? lagsum_small_kernel<8> : lagsum_small_kernel<9>;
            if (int rc = grid(reinterpret_cast<const void *>(kern), DIAG_WG, ((n + 31) / 32 + LS_ROWS - 1) / LS_ROWS, &blocks))
                return rc;
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(DIAG_WG), 0, s, d_data, (uint64_t)n, max_lag, c->diag_merge);
            hipLaunchKernelGGL(lagsum_fix_small_kernel, dim3(1), dim3(LS_FIX_WG), 0, s, d_data, (uint64_t)n, max_lag,
                               c->diag_merge, sums, total);
            LZ_HIP(hipGetLastError());
            return ordered ? LZ_OK : diag_end(c, s);
        }
        // windows of at most LW_WINDOW lags, as even as 32-lag steps allow, one launch each
        const uint64_t lags = (uint64_t)max_lag + 1, nwin = (lags + LW_WINDOW - 1) / LW_WINDOW;
        const uint32_t W = (uint32_t)(((lags + nwin - 1) / nwin + 31) / 32 * 32);
        if (int rc = grid(reinterpret_cast<const void *>(&lagsum_wide_kernel), LW_WG,
                          ((n + 31) / 32 + LW_ROWS - 1) / LW_ROWS, &blocks))
            return rc;
        for (uint32_t k_lo = 0; k_lo <= max_lag; k_lo += W) {
            const uint32_t Lw = max_lag - k_lo < W - 1 ? max_lag - k_lo : W - 1;
            hipLaunchKernelGGL(lagsum_wide_kernel, dim3(blocks), dim3(LW_WG), 0, s, d_data, (uint64_t)n, Lw, k_lo,
                               max_lag, c->diag_merge);
        }
        hipLaunchKernelGGL(lagsum_fix_kernel, dim3(max_lag / FIX_LAGS + 1), dim3(DIAG_WG), 0, s, d_data,
                           (uint64_t)n, max_lag, c->diag_merge, sums, total);
        LZ_HIP(hipGetLastError());
        return ordered ? LZ_OK : diag_end(c, s);
    }
    LZ_HIP(launch_fill_u64(sums, (size_t)max_lag + 1, s));  // n == 0: every sum is 0
    if (total) LZ_HIP(launch_fill_u64(total, 1, s));
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

}  // namespace

extern "C" int lz_lag_sums(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, uint64_t *d_sums,
                           void *stream) {
    if (!c || !d_sums || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    if (max_lag > 16384) return fail(LZ_E_INVAL, "max_lag must be <= 16384");
    LZ_HIP(hipSetDevice(c->device));
    return lag_sums(c, d_data, n, max_lag, reinterpret_cast<unsigned long long *>(d_sums), nullptr,
                    (hipStream_t)stream);
}

namespace {

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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_matrix(const lz_ctx *c, const uint8_t *img, uint32_t h, uint32_t w, const void *out) {
    if (!c || !img || !out) return fail(LZ_E_INVAL, "NULL argument");
    if (h == 0 || w == 0) return fail(LZ_E_INVAL, "empty matrix");
    if (h > 65536 || w > 65536 || (uint64_t)h * w > (1ull << 24))
        return fail(LZ_E_INVAL, "matrix too large: h, w <= 65536 and h * w <= 2^24");
    return LZ_OK;
}

struct Dft2 {
    double2 *tw_h, *tw_w, *a, *b;
};

// Workspace: twiddles for h and w, then two h*w complex buffers; extra bytes go first.
Dft2 dft2_layout(char *ws, uint32_t h, uint32_t w, size_t extra) {
    Dft2 d;
    size_t off = align256(extra);
    d.tw_h = reinterpret_cast<double2 *>(ws + off);
    off += align256((size_t)h * sizeof(double2));
    d.tw_w = reinterpret_cast<double2 *>(ws + off);
    off += align256((size_t)w * sizeof(double2));
    d.a = reinterpret_cast<double2 *>(ws + off);
    off += align256((size_t)h * w * sizeof(double2));
    d.b = reinterpret_cast<double2 *>(ws + off);
    return d;
}

size_t dft2_bytes(uint32_t h, uint32_t w, size_t extra) {
    return align256(extra) + align256((size_t)h * sizeof(double2)) + align256((size_t)w * sizeof(double2)) +
           2 * align256((size_t)h * w * sizeof(double2));
}

bool fft_ok(const lz_ctx *c, uint32_t N);

// The twiddle tables of the lengths that are not powers of two (the power-of-two FFT makes its own).
int launch_twiddles(const lz_ctx *c, const Dft2 &d, uint32_t h, uint32_t w, hipStream_t s) {
    if (!fft_ok(c, h)) hipLaunchKernelGGL(twiddle_kernel, dim3((h + 255) / 256), dim3(256), 0, s, d.tw_h, h);
    if (!fft_ok(c, w)) hipLaunchKernelGGL(twiddle_kernel, dim3((w + 255) / 256), dim3(256), 0, s, d.tw_w, w);
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

// The radices of N for the mixed-radix pass (5s, 3s, 4s, then a 2), or nst = 0 if N has
// another prime factor.
FftPlan mixed_plan(uint32_t N) {
    FftPlan p{};
    uint32_t n = N;
    for (uint32_t r : {5u, 3u}) {
        while (n % r == 0 && p.nst < 16) {
            p.rad[p.nst++] = (uint8_t)r;
            n /= r;
        }
    }
    while (n % 4 == 0 && p.nst < 16) {
        p.rad[p.nst++] = 4;
        n /= 4;
    }
    if (n == 2 && p.nst < 16) {
        p.rad[p.nst++] = 2;
        n = 1;
    }
    if (n != 1) p.nst = 0;
    return p;
}

size_t mixed_lds(uint32_t N) {
    const uint32_t per_wg = N > FFT_WG_ELEMS ? N : FFT_WG_ELEMS;
    return ((size_t)(per_wg / N) * N + N) * sizeof(double2);
}

bool mixed_ok(const lz_ctx *c, uint32_t N) {
    return N <= FFT_MAX && N > 1 && mixed_plan(N).nst > 0 && mixed_lds(N) <= (size_t)c->dev.lds_per_wg_max;
}

size_t fft_lds(uint32_t N) {
    const uint32_t per_wg = N > FFT_WG_ELEMS ? N : FFT_WG_ELEMS;
    return ((size_t)(N <= FFT_PP_MAX ? 2 : 1) * per_wg + fft_twiddles(N)) * sizeof(double2);
}

bool fft_ok(const lz_ctx *c, uint32_t N) {
    const size_t lds = fft_lds(N);
    return (N & (N - 1)) == 0 && N <= FFT_MAX && lds <= (size_t)c->dev.lds_per_wg_max;
}

// Output (M x out.nout) = transpose of (DFT_N along the rows of src (N x M)), its first out.nout
// rows, stored by epilogue E: by FFT when N is a power of two up to FFT_MAX, by mixed-radix FFT
// when N <= FFT_MAX has no prime factor above 5, otherwise directly on the matrix cores (tw: the
// N-entry table, needed by the last two).
template <typename In, int E>
int launch_dft_pass(const lz_ctx *c, const In *src, uint32_t N, uint32_t M, const double2 *tw, double sign,
                    PassOut out, hipStream_t s) {
    if (N == FFT1K && fft1k_lds() <= (size_t)c->dev.lds_per_wg_max) {
        const size_t lds = fft1k_lds();
        if (lds > 65536)
            LZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fft1k_pass_kernel<In, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        // a multiple of 8 workgroups, so that neighbouring column groups share an XCD (the
        // workgroups past the last column only help make the twiddle table and leave)
        const uint32_t groups = ((M + FFT1K_COLS - 1) / FFT1K_COLS + 7) / 8 * 8;
        hipLaunchKernelGGL((fft1k_pass_kernel<In, E>), dim3(groups), dim3(DIAG_WG), lds, s, src, M, sign, out);
    } else if (fft_ok(c, N)) {
        uint32_t logN = 0;
        while ((1u << logN) < N) ++logN;
        const uint32_t per_wg = N > FFT_WG_ELEMS ? N : FFT_WG_ELEMS;
        const uint32_t C = per_wg / N;
        const uint32_t groups = (M + C - 1) / C;
        const size_t lds = fft_lds(N);
        if (lds > 65536)
            LZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fft_pass_kernel<In, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((fft_pass_kernel<In, E>), dim3(groups), dim3(DIAG_WG), lds, s, src, N, M, logN, C, sign,
                           out);
    } else if (mixed_ok(c, N)) {
        const uint32_t per_wg = N > FFT_WG_ELEMS ? N : FFT_WG_ELEMS;
        const uint32_t C = per_wg / N;
        const uint32_t groups = (M + C - 1) / C;
        const size_t lds = mixed_lds(N);
        if (lds > 65536)
            LZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fft_mixed_pass_kernel<In, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((fft_mixed_pass_kernel<In, E>), dim3(groups), dim3(DIAG_WG), lds, s, src, N, M, C,
                           mixed_plan(N), tw, sign, out);
    } else {
        // 64 x 64 tiles, or 32 x 64 where those would leave compute units idle
        const uint32_t gy = (M + DFT_T - 1) / DFT_T;
        if ((uint64_t)((out.nout + DFT_T - 1) / DFT_T) * gy < (uint64_t)c->dev.cus) {
            const dim3 grid((out.nout + 31) / 32, gy);
            hipLaunchKernelGGL((dft_pass_kernel<In, E, 32>), grid, dim3(DIAG_WG), 0, s, src, N, M, tw, sign, out);
        } else {
            const dim3 grid((out.nout + DFT_T - 1) / DFT_T, gy);
            hipLaunchKernelGGL((dft_pass_kernel<In, E, 64>), grid, dim3(DIAG_WG), 0, s, src, N, M, tw, sign, out);
        }
    }
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

// complex results, indices r < nout of each transform; real results, whole rows of n, with the
// mirror rows of an h-row matrix (0: none)
PassOut complex_out(double2 *z, uint32_t nout) { return PassOut{z, nullptr, nullptr, nout, 0}; }
PassOut real_out(double *p, uint32_t n, uint32_t h, const double *den = nullptr) {
    return PassOut{nullptr, p, den, n, h};
}

}  // namespace

extern "C" int lz_entropy(lz_ctx *c, const uint64_t *d_hist, double *d_S, void *stream) {
    if (!c || !d_hist || !d_S) return fail(LZ_E_INVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    hipLaunchKernelGGL(entropy_kernel, dim3(1), dim3(DIAG_WG), 0, s,
                       reinterpret_cast<const unsigned long long *>(d_hist), d_S);
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

extern "C" int lz_autocorrelation(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, double *d_r,
                                  void *stream) {
    if (!c || !d_r || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    if (max_lag > 16384) return fail(LZ_E_INVAL, "max_lag must be <= 16384");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    char *ws;
    if (int rc = diag_begin(c, s, 8 + ((size_t)max_lag + 1) * 8, &ws)) return rc;
    unsigned long long *total = reinterpret_cast<unsigned long long *>(ws);
    unsigned long long *sums = total + 1;
    if (int rc = lag_sums(c, d_data, n, max_lag, sums, total, s, true)) return rc;
    hipLaunchKernelGGL(autocorr_norm_kernel, dim3(1), dim3(DIAG_WG), 0, s, d_data, (uint64_t)n, max_lag, sums,
                       total, d_r);
    LZ_HIP(hipGetLastError());
    return diag_end(c, s);
}

extern "C" int lz_power_spectrum_2d(lz_ctx *c, const uint8_t *d_img, uint32_t h, uint32_t w, double *d_power,
                                    void *stream) {
    if (int rc = check_matrix(c, d_img, h, w, d_power)) return rc;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    char *ws;
    if (int rc = diag_begin(c, s, dft2_bytes(h, w, 0), &ws)) return rc;
    const Dft2 d = dft2_layout(ws, h, w, 0);
    if (int rc = launch_twiddles(c, d, h, w, s)) return rc;
    // a: w x (h/2 + 1), the columns' transforms up to index h/2 (the rest is their mirror image);
    // then |Z|^2 of the second pass, rows 0..h/2 and their mirror rows, straight into the output
    const uint32_t hh = h / 2 + 1;
    if (int rc = launch_dft_pass<uint8_t, EPI_COMPLEX>(c, d_img, h, w, d.tw_h, -1.0, complex_out(d.a, hh), s))
        return rc;
    if (int rc = launch_dft_pass<double2, EPI_POWER>(c, d.a, w, hh, d.tw_w, -1.0, real_out(d_power, w, h), s))
        return rc;
    return diag_end(c, s);
}

extern "C" int lz_autocorrelation_2d(lz_ctx *c, const uint8_t *d_img, uint32_t h, uint32_t w, double *d_acf,
                                     void *stream) {
    if (int rc = check_matrix(c, d_img, h, w, d_acf)) return rc;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    char *ws;
    const size_t extra = 256 * 8 + 8;  // histogram, then the denominator
    if (int rc = diag_begin(c, s, dft2_bytes(h, w, extra), &ws)) return rc;
    uint64_t *hist = reinterpret_cast<uint64_t *>(ws);
    double *den = reinterpret_cast<double *>(hist + 256);
    const Dft2 d = dft2_layout(ws, h, w, extra);
    const size_t n = (size_t)h * w;
    if (int rc = lz_histogram(c, d_img, n, hist, stream)) return rc;
    hipLaunchKernelGGL(acf2_den_kernel, dim3(1), dim3(DIAG_WG), 0, s,
                       reinterpret_cast<const unsigned long long *>(hist), (uint64_t)n, den);
    LZ_HIP(hipGetLastError());
    if (int rc = launch_twiddles(c, d, h, w, s)) return rc;
    // a: w x (h/2 + 1); b: |Z|^2 with the zero frequency removed (h x w, real and even);
    // a: w x (h/2 + 1) again; then Re G / den, rows 0..h/2 and their mirror rows (G is even too)
    const uint32_t hh = h / 2 + 1;
    double *pm = reinterpret_cast<double *>(d.b);
    if (int rc = launch_dft_pass<uint8_t, EPI_COMPLEX>(c, d_img, h, w, d.tw_h, -1.0, complex_out(d.a, hh), s))
        return rc;
    if (int rc = launch_dft_pass<double2, EPI_POWER_NODC>(c, d.a, w, hh, d.tw_w, -1.0, real_out(pm, w, h), s))
        return rc;
    if (int rc = launch_dft_pass<double, EPI_COMPLEX>(c, pm, h, w, d.tw_h, 1.0, complex_out(d.a, hh), s))
        return rc;
    if (int rc = launch_dft_pass<double2, EPI_ACF>(c, d.a, w, hh, d.tw_w, 1.0, real_out(d_acf, w, h, den), s))
        return rc;
    return diag_end(c, s);
}
