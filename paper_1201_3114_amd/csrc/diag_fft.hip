// The 2-D analyses of Section 4 for a byte matrix (a text or an image laid out row by row) as
// GPU kernels: the Fourier power spectrum and the circular autocorrelation matrix, in binary64.
// The 2-D transforms run as FFTs for sides with no prime factor above 5 and as binary64 matrix
// products on the matrix cores otherwise.
#include "diag_common.h"

#include <type_traits>

namespace lz {
namespace {

// ---- 2-D discrete Fourier transform as two passes ----------------------------------------
//
// One pass applies the N-point DFT along the rows index of an N x M matrix and
// writes the result transposed:  dst[c][r] = sum_k e^{sign 2 pi i r k / N} src[k][c].
// Two passes (first along the H rows of the H x W image, then along its W
// columns) give the 2-D DFT in natural layout.  Every size is allowed (no
// power-of-two restriction); the twiddle index r k mod N is kept exact in
// integers, so every twiddle is one table entry.

constexpr int DFT_T = 64;  // output tile edge (r and c)
constexpr int DFT_KS32 = 32, DFT_KS64 = 16;  // terms per LDS stage for 32- and 64-row tiles

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
// k stage (16 or 32 terms) are loaded into registers while the current stage computes; the loads are
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
// The autocorrelation matrix's denominator n S2 - S1^2 comes from the moment sums mom: a first
// pass over bytes adds each workgroup's S1 = sum x and S2 = sum x^2 into copy (slot mod
// MOM_COPIES), mom[MOM_STRIDE copy] and the word after it, a cache line per copy so that the
// device atomics of different copies do not wait for each other (exact: S1 < 2^32 and S2 < 2^40
// for at most 2^24 bytes); in the last pass one thread per workgroup adds up the copies (den,
// NaN when n S2 = S1^2, that is when every byte is equal).
constexpr uint32_t MOM_COPIES = 32, MOM_STRIDE = 16;  // 16 words: 128 bytes
enum : int { EPI_COMPLEX = 0, EPI_POWER = 1, EPI_POWER_NODC = 2, EPI_ACF = 3 };
struct PassOut {
    double2 *z;
    double *p;
    uint32_t nout;
    uint32_t mirror;
    unsigned long long *mom;  // first pass over bytes: add the moment sums here (or nullptr)
    uint64_t n;               // EPI_ACF: the matrix's n = h w, with mom holding its moment sums
    double den;               // EPI_ACF: set by the kernel from mom and n
};

// The workgroup's moment sums (per-thread s1, s2) into copy slot mod MOM_COPIES of o.mom; every
// thread of the workgroup (DIAG_WG threads) calls it: it holds a barrier.
__device__ __forceinline__ void add_moments(const PassOut &o, unsigned long long s1, unsigned long long s2,
                                            uint32_t slot) {
    __shared__ unsigned long long mred[2][DIAG_WG / 64];
    for (int k = 32; k > 0; k >>= 1) {
        s1 += __shfl_xor(s1, k, 64);
        s2 += __shfl_xor(s2, k, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        mred[0][threadIdx.x / 64] = s1;
        mred[1][threadIdx.x / 64] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t1 = 0, t2 = 0;
        for (int w = 0; w < DIAG_WG / 64; ++w) {
            t1 += mred[0][w];
            t2 += mred[1][w];
        }
        unsigned long long *m = o.mom + MOM_STRIDE * (slot % MOM_COPIES);
        if (t1) atomicAdd(&m[0], t1);
        if (t2) atomicAdd(&m[1], t2);
    }
}

// n S2 - S1^2 from the moment copies, exactly (n <= 2^24 keeps both products below 2^64): thread 0
// adds up the copies and the workgroup (DIAG_WG threads, all of which call it) shares the result.
__device__ __forceinline__ double acf_den(const PassOut &o) {
    __shared__ double den_s;
    if (threadIdx.x == 0) {
        unsigned long long s1 = 0, s2 = 0;
        for (uint32_t c = 0; c < MOM_COPIES; ++c) {
            s1 += o.mom[MOM_STRIDE * c];
            s2 += o.mom[MOM_STRIDE * c + 1];
        }
        const unsigned long long d = o.n * s2 - s1 * s1;
        den_s = d == 0 ? __builtin_nan("") : (double)d;
    }
    __syncthreads();
    return den_s;
}

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
            const double d = o.den;
            v = d != d ? d : re / d;
        } else {
            v = (E == EPI_POWER_NODC && c == 0 && r == 0) ? 0.0 : re * re + im * im;
        }
        o.p[i] = v;
        // the real outputs keep whole rows (nout = N)
        if (o.mirror && c != 0 && o.mirror - c >= M) o.p[(size_t)(o.mirror - c) * N + (r ? N - r : 0)] = v;
    }
}

template <typename In, int E, int TR, int KS>
__global__ __launch_bounds__(DIAG_WG) void dft_pass_kernel(const In *src, uint32_t N, uint32_t M, const double2 *tw,
                                                            double sign, PassOut dst) {
    if constexpr (E == EPI_ACF) dst.den = acf_den(dst);
    // Workgroups are dealt to the 8 XCDs in turn: when the tiles divide evenly, those sharing an
    // input column tile go to one XCD, whose L2 then reads those columns from HBM once.
    const uint32_t nt = gridDim.x * gridDim.y, lin = blockIdx.x + gridDim.x * blockIdx.y;
    const uint32_t tix = nt % 8 == 0 ? (lin % 8) * (nt / 8) + lin / 8 : lin;
    const uint32_t rt = tix % gridDim.x, ct = tix / gridDim.x;  // row tile, column tile
    // the workgroups of the first row tile see every input once: they add the moment sums
    const bool moments = std::is_same_v<In, uint8_t> && dst.mom && rt == 0;
    unsigned long long m1 = 0, m2 = 0;
    // TR x 64 outputs per workgroup: with TR = 64 each wave takes a 32 x 32 block as 2 x 2 tiles of
    // 16 x 16, with TR = 32 (grids that would not fill the chip) a 32 x 16 block as 2 x 1 tiles.
    // A real input (bytes or doubles) has no imaginary part: two of the four products are skipped.
    // KS terms per LDS stage: the loads of the next stage are in flight during this one's products.
    static_assert(TR == 64 || TR == 32, "tile height");
    static_assert(KS % 4 == 0 && (TR * KS) % DIAG_WG == 0, "whole rows of the stage per thread");
    constexpr int QX = KS / 4;                       // input rows each thread stages per k stage
    constexpr int WC = TR == 64 ? 2 : 4;             // waves across the tile's columns
    constexpr int TB = 4 / WC;                       // column tiles per wave
    constexpr bool REAL = !std::is_same_v<In, double2>;
    constexpr int TWQ = TR * KS / DIAG_WG;           // twiddles each thread stages per k stage
    __shared__ double2 s_src[KS][DFT_T];  // [k][c]
    __shared__ double2 s_tw[KS][TR];      // [k][r]
    const uint32_t r0 = rt * TR, c0 = ct * DFT_T;
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const uint32_t wr = (wave / WC) * 32, wc = (wave % WC) * (16 * TB);
    const uint32_t li = lane % 16, lk = lane / 16;
    // staging: column cc of the input tile for k rows kq + 4q; twiddle row tr_s for k rows kt + (KS/TWQ) q
    const uint32_t cc = threadIdx.x % DFT_T, kq = threadIdx.x / DFT_T;
    const uint32_t tr_s = threadIdx.x % TR, kt = threadIdx.x / TR;
    const uint32_t rs = r0 + tr_s;
    const uint32_t rmod = rs < N ? rs : 0;
    const uint32_t cs = c0 + cc < M ? c0 + cc : M - 1;
    uint32_t off[TWQ];
    for (int q = 0; q < TWQ; ++q) off[q] = (uint32_t)(((uint64_t)rmod * (kt + (KS / TWQ) * q)) % N);
    const uint32_t step = (uint32_t)(((uint64_t)rmod * KS) % N);
    uint32_t base = 0;
    In nx[QX];
    double2 nw[TWQ];
    auto fetch = [&](uint32_t k0) {
        for (int q = 0; q < QX; ++q) {
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
    for (uint32_t k0 = 0; k0 < N; k0 += KS) {
        for (int q = 0; q < QX; ++q) {
            const uint32_t k = k0 + kq + 4 * q;
            const bool in = k < N && c0 + cc < M;
            s_src[kq + 4 * q][cc] = in ? dft_value(nx[q]) : make_double2(0.0, 0.0);
            if constexpr (std::is_same_v<In, uint8_t>) {
                const unsigned long long xv = in ? nx[q] : 0;
                m1 += xv;
                m2 += xv * xv;
            }
        }
        for (int q = 0; q < TWQ; ++q) {
            const uint32_t kk = kt + (KS / TWQ) * q, k = k0 + kk;
            s_tw[kk][tr_s] = (k < N && rs < N) ? make_double2(nw[q].x, sign * nw[q].y) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (k0 + KS < N) fetch(k0 + KS);
#pragma unroll
        for (int k4 = 0; k4 < KS / 4; ++k4) {
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
    if (moments) add_moments(dst, m1, m2, ct);
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
    if constexpr (E == EPI_ACF) dst.den = acf_den(dst);
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
    if (c0 >= M) return;  // a workgroup of the padding (the grid is a multiple of 8)
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
        unsigned long long m1 = 0, m2 = 0;
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                cur[cl * N + k] = dft_value(v[i]);
                if constexpr (std::is_same_v<In, uint8_t>) {
                    m1 += v[i];
                    m2 += (unsigned long long)v[i] * v[i];
                }
            }
        }
        if (std::is_same_v<In, uint8_t> && dst.mom) add_moments(dst, m1, m2, blockIdx.x);
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
    if constexpr (E == EPI_ACF) dst.den = acf_den(dst);
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
    if constexpr (std::is_same_v<In, uint8_t>) {
        if (dst.mom) {  // every thread: the waves past the last column add nothing
            unsigned long long m1 = 0, m2 = 0;
            if (live)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    m1 += x[j];
                    m2 += (unsigned long long)x[j] * x[j];
                }
            add_moments(dst, m1, m2, blockIdx.x);
        }
    }
    if (!live) return;  // the whole wave
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
    if constexpr (E == EPI_ACF) dst.den = acf_den(dst);
    extern __shared__ double2 fbuf[];  // C columns of N values, then the N twiddles
    double2 *ftw = fbuf + (size_t)C * N;
    uint32_t g = blockIdx.x;
    if (gridDim.x % 8 == 0) g = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t c0 = g * C;
    if (c0 >= M) return;  // a workgroup of the padding (the grid is a multiple of 8)
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
        unsigned long long m1 = 0, m2 = 0;
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const uint32_t e = threadIdx.x + i * DIAG_WG;
            if (e < total) {
                const uint32_t k = e / cols, cl = e - k * cols;
                fbuf[cl * N + k] = dft_value(v[i]);
                if constexpr (std::is_same_v<In, uint8_t>) {
                    m1 += v[i];
                    m2 += (unsigned long long)v[i] * v[i];
                }
            }
        }
        if (std::is_same_v<In, uint8_t> && dst.mom) add_moments(dst, m1, m2, blockIdx.x);
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
        const uint32_t groups = ((M + C - 1) / C + 7) / 8 * 8;  // a multiple of 8: the XCD-aware order
        const size_t lds = fft_lds(N);
        if (lds > 65536)
            LZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fft_pass_kernel<In, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((fft_pass_kernel<In, E>), dim3(groups), dim3(DIAG_WG), lds, s, src, N, M, logN, C, sign,
                           out);
    } else if (mixed_ok(c, N)) {
        const uint32_t per_wg = N > FFT_WG_ELEMS ? N : FFT_WG_ELEMS;
        const uint32_t C = per_wg / N;
        const uint32_t groups = ((M + C - 1) / C + 7) / 8 * 8;  // a multiple of 8: the XCD-aware order
        const size_t lds = mixed_lds(N);
        if (lds > 65536)
            LZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&fft_mixed_pass_kernel<In, E>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL((fft_mixed_pass_kernel<In, E>), dim3(groups), dim3(DIAG_WG), lds, s, src, N, M, C,
                           mixed_plan(N), tw, sign, out);
    } else {
        // 64 x 64 tiles, or 32 x 64 where those would leave compute units idle; DFT_KS32 and
        // DFT_KS64 terms per LDS stage (the smaller tiles do half the products per term)
        const uint32_t gy = (M + DFT_T - 1) / DFT_T;
        if ((uint64_t)((out.nout + DFT_T - 1) / DFT_T) * gy < (uint64_t)c->dev.cus) {
            const dim3 grid((out.nout + 31) / 32, gy);
            hipLaunchKernelGGL((dft_pass_kernel<In, E, 32, DFT_KS32>), grid, dim3(DIAG_WG), 0, s, src, N, M, tw,
                               sign, out);
        } else {
            const dim3 grid((out.nout + DFT_T - 1) / DFT_T, gy);
            hipLaunchKernelGGL((dft_pass_kernel<In, E, 64, DFT_KS64>), grid, dim3(DIAG_WG), 0, s, src, N, M, tw,
                               sign, out);
        }
    }
    LZ_HIP(hipGetLastError());
    return LZ_OK;
}

// complex results, indices r < nout of each transform; real results, whole rows of n, with the
// mirror rows of an h-row matrix (0: none)
PassOut complex_out(double2 *z, uint32_t nout, unsigned long long *mom = nullptr) {
    return PassOut{z, nullptr, nout, 0, mom, 0, 0.0};
}
PassOut real_out(double *p, uint32_t n, uint32_t h, unsigned long long *mom = nullptr, uint64_t count = 0) {
    return PassOut{nullptr, p, n, h, mom, count, 0.0};
}

}  // namespace
}  // namespace lz

using namespace lz;

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
    const size_t extra = (size_t)MOM_STRIDE * MOM_COPIES * 8;  // the moment sums S1, S2 (a pair per copy)
    if (int rc = diag_begin(c, s, dft2_bytes(h, w, extra), &ws)) return rc;
    unsigned long long *mom = reinterpret_cast<unsigned long long *>(ws);
    const Dft2 d = dft2_layout(ws, h, w, extra);
    const uint64_t n = (uint64_t)h * w;
    LZ_HIP(launch_fill_u64(mom, (size_t)MOM_STRIDE * MOM_COPIES, s));
    if (int rc = launch_twiddles(c, d, h, w, s)) return rc;
    // a: w x (h/2 + 1), adding the moment sums; b: |Z|^2 with the zero frequency removed (h x w,
    // real and even); a: w x (h/2 + 1) again; then Re G / den, den = n S2 - S1^2 from the moment
    // sums, rows 0..h/2 and their mirror rows (G is even too)
    const uint32_t hh = h / 2 + 1;
    double *pm = reinterpret_cast<double *>(d.b);
    if (int rc = launch_dft_pass<uint8_t, EPI_COMPLEX>(c, d_img, h, w, d.tw_h, -1.0, complex_out(d.a, hh, mom), s))
        return rc;
    if (int rc = launch_dft_pass<double2, EPI_POWER_NODC>(c, d.a, w, hh, d.tw_w, -1.0, real_out(pm, w, h), s))
        return rc;
    if (int rc = launch_dft_pass<double, EPI_COMPLEX>(c, pm, h, w, d.tw_h, 1.0, complex_out(d.a, hh), s))
        return rc;
    if (int rc = launch_dft_pass<double2, EPI_ACF>(c, d.a, w, hh, d.tw_w, 1.0, real_out(d_acf, w, h, mom, n), s))
        return rc;
    return diag_end(c, s);
}
