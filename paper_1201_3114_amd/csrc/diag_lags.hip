// The autocorrelation of a byte sequence (Section 4) as GPU kernels: the lag sums
// S_k = sum_i x_i x_{i+k} are int8 matrix products on the matrix cores (up to lag 256 in one
// launch, beyond that in windows of at most 4096 lags), exact in 64-bit integers, so they do not
// depend on the order of the additions; the normalised coefficients are binary64 from them.
#include "diag_common.h"

namespace lz {
namespace {

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
// of x_j + x_{n-1-j} (a wave scan by shuffles, then the wave totals through LDS).  With r
// non-null (n > 0) it also writes the normalised coefficients r_k, as autocorr_norm_kernel does
// and in the same binary64 operations: A_k + B_k = 2T - (P_k + Q_k) is an exact integer below
// 2^53, as is each of A_k and B_k there.
constexpr int LS_FIX_WG = 512;
static_assert(LS_FIX_WG > 32 * (LS_MAX_NT - 1) && LS_FIX_WG >= (int)LS_COPIES, "a thread per lag and per copy");
__global__ __launch_bounds__(LS_FIX_WG) void lagsum_fix_small_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                                     unsigned long long *merge,
                                                                     unsigned long long *sums,
                                                                     unsigned long long *total, double *r) {
    __shared__ uint32_t wsum[LS_FIX_WG / 64];
    __shared__ unsigned long long tsum[LS_FIX_WG / 64];
    __shared__ unsigned long long s0;
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
    // P_k + Q_k: the bytes j < k of both ends
    const unsigned long long pq = before + inc - x;
    unsigned long long sk = 0;
    if (k <= L) {
        unsigned long long raw = 0;
#pragma unroll
        for (uint32_t c = 0; c < LS_COPIES; ++c) {
            raw += part[c];
            merge[c * cs + k] = 0;
        }
        const unsigned long long m = k < n ? n - k : 0;
        sk = raw - 128ull * pq - 16384ull * m;
        sums[k] = sk;
        if (k == 0) s0 = sk;
    }
    if (k < LS_COPIES) merge[k * cs + L + 1] = 0;
    unsigned long long T = 0;
    for (uint32_t w = 0; w < LS_FIX_WG / 64; ++w) T += tsum[w];
    if (k == 0 && total) *total = T;
    if (!r) return;
    __syncthreads();  // S_0
    if (k > L) return;
    const unsigned long long S0 = s0;
    const double mean = (double)T / (double)n;
    const double den = (double)S0 - (double)n * mean * mean;
    // no coefficient when every byte is equal: n S_0 = T^2 exactly then, and only then
    const bool constant = (unsigned __int128)n * S0 == (unsigned __int128)T * T;
    double v;
    if (constant) v = __builtin_nan("");
    else if (k == 0) v = 1.0;
    else if (k >= n) v = 0.0;
    else v = ((double)sk - mean * (double)(2 * T - pq) + (double)(n - k) * mean * mean) / den;
    r[k] = v;
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

// ---- the normalised 1-D autocorrelation ---------------------------------------------------

// r_k for k = 0..L of a byte sequence x_0..x_{n-1} with mean m:
//   r_k = sum_{i<n-k} (x_i - m)(x_{i+k} - m) / sum_i (x_i - m)^2
//       = (S_k - m (A_k + B_k) + (n-k) m^2) / (S_0 - n m^2),
// A_k = sum_{i<n-k} x_i = T - (sum of the last k bytes), B_k = sum_{i>=k} x_i = T - (sum of the first k bytes),
// so A_k + B_k = 2T - (P_k + Q_k) with P_k + Q_k = sum_{j<k} (x_j + x_{n-1-j}), an exact integer below 2^53.
// One workgroup per 256 lags: workgroup b takes k = 256 b + 1 .. 256 b + 256 (and workgroup 0 also r_0):
// the sum of x_j + x_{n-1-j} over j < 256 b (16-byte loads where aligned, a workgroup sum), then a
// wave scan over its own 256 values of j.  NaN for no bytes or one repeated byte (n S_0 = T^2 exactly,
// compared in 128-bit integers), 0 for k >= n.
__global__ __launch_bounds__(DIAG_WG) void autocorr_norm_kernel(const uint8_t *data, uint64_t n, uint32_t L,
                                                                 const unsigned long long *sums,
                                                                 const unsigned long long *total, double *r) {
    __shared__ unsigned long long red[DIAG_WG];
    __shared__ uint32_t wsum[DIAG_WG / 64];
    const uint32_t t = threadIdx.x, lane = t % 64, wave = t / 64;
    const uint64_t kb = (uint64_t)blockIdx.x * DIAG_WG;
    const unsigned long long T = *total;
    const bool constant = n == 0 || (unsigned __int128)n * sums[0] == (unsigned __int128)T * T;
    const uint64_t mb = kb < n ? kb : n;
    const unsigned long long base =
        block_sum<unsigned long long>(fix_range_part(data, 0, mb) + fix_range_part(data, n - mb, n), red);
    const uint64_t j = kb + t;  // lag k = j + 1 includes byte j of both ends
    const uint32_t x = j < n ? (uint32_t)data[j] + data[n - 1 - j] : 0u;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if ((int)lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before += wsum[w];
    if (blockIdx.x == 0 && t == 0) r[0] = constant ? __builtin_nan("") : 1.0;
    const uint64_t k = j + 1;
    if (k > L) return;
    double v;
    if (constant) {
        v = __builtin_nan("");
    } else if (k >= n) {
        v = 0.0;
    } else {
        const unsigned long long pq = base + before + inc;  // P_k + Q_k
        const double mean = (double)T / (double)n;
        const double den = (double)sums[0] - (double)n * mean * mean;
        v = ((double)sums[k] - mean * (double)(2 * T - pq) + (double)(n - k) * mean * mean) / den;
    }
    r[k] = v;
}

// The lag sums into sums[0..max_lag]; with total non-null, also the byte total into *total.
// ordered: the caller has already ordered this stream after the context's other diagnostics
// (diag_begin) and records the event afterwards itself.
// r: when the lags fit one launch (and n > 0), the normalised coefficients are written too and
// *normalised is set.
int lag_sums(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, unsigned long long *sums,
             unsigned long long *total, hipStream_t s, bool ordered = false, double *r = nullptr,
             bool *normalised = nullptr) {
    if (normalised) *normalised = false;
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
                               c->diag_merge, sums, total, r);
            LZ_HIP(hipGetLastError());
            if (normalised) *normalised = r != nullptr;
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
}  // namespace lz

using namespace lz;

extern "C" int lz_lag_sums(lz_ctx *c, const uint8_t *d_data, size_t n, uint32_t max_lag, uint64_t *d_sums,
                           void *stream) {
    if (!c || !d_sums || (!d_data && n)) return fail(LZ_E_INVAL, "NULL argument");
    if (max_lag > 16384) return fail(LZ_E_INVAL, "max_lag must be <= 16384");
    LZ_HIP(hipSetDevice(c->device));
    return lag_sums(c, d_data, n, max_lag, reinterpret_cast<unsigned long long *>(d_sums), nullptr,
                    (hipStream_t)stream);
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
    bool normalised = false;
    if (int rc = lag_sums(c, d_data, n, max_lag, sums, total, s, true, d_r, &normalised)) return rc;
    if (!normalised)
        hipLaunchKernelGGL(autocorr_norm_kernel, dim3(max_lag > 0 ? (max_lag + DIAG_WG - 1) / DIAG_WG : 1),
                           dim3(DIAG_WG), 0, s, d_data, (uint64_t)n, max_lag, sums, total, d_r);
    LZ_HIP(hipGetLastError());
    return diag_end(c, s);
}
