// gfx950 kernels of the Lorenz chaotic cipher (arXiv:1201.3114, Sections 3
// and 5).  One lane carries M independent chains (blocks of the parallel
// version); the per-byte work is Steps 1-3 of Section 3.2, dominated by
// n_it forward-Euler steps of the Lorenz system in binary64 (14 roundings per
// step, no contraction: the file is built with -ffp-contract=off and nothing
// here may be fused, so results equal the exact IEEE sequence of the method).
//
// Byte streams: a wave stages `tile` bytes of each of its 64*M chains into
// LDS with lane-contiguous (coalesced) global loads, the lanes consume their
// own chain's bytes from LDS, write the output bytes back in place, and the
// wave stores the tile with lane-contiguous global stores.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "internal.h"

namespace lz {
namespace {

constexpr double SIGMA = 10.0;
constexpr double RHO = 28.0;
constexpr double BETA = 8.0 / 3.0;
constexpr double SCALE_NU = 1e13;  // 10^nu, nu = floor(log10 2^(52-6)) = 13
constexpr int WAVE = 64;

// ---- scalar pieces of the method ------------------------------------------------

__device__ __forceinline__ double sel3(uint32_t m, double x, double y, double z) {
    return m == 0 ? x : (m == 1 ? y : z);
}

// Eq. R_nu: byte Omega (0..3) of floor(alpha 10^13) in two's complement.  The
// integer N has |N| < 2^53; N mod 2^32 is formed exactly in binary64.
__device__ __forceinline__ uint32_t r_nu(double alpha, uint32_t om) {
    const double N = floor(alpha * SCALE_NU);
    const double hi = floor(N * 0x1p-32);
    const double lo = N - hi * 0x1p32;
    return ((uint32_t)lo >> (8u * om)) & 0xFFu;
}

// Step 2: Theta = P / 10^(3 + Omega_3), one correctly rounded division.
__device__ __forceinline__ double theta_of(uint32_t p, uint32_t o3) {
    const double p10 = o3 == 0 ? 1e3 : (o3 == 1 ? 1e4 : (o3 == 2 ? 1e5 : 1e6));
    return (double)p / p10;
}

// Integrity word N(v) = floor(v 10^13) as a two's complement 64-bit pattern.
__device__ __forceinline__ unsigned long long digest_word(double v) {
    const double N = floor(v * SCALE_NU);
    const double hi = floor(N * 0x1p-32);
    const double lo = N - hi * 0x1p32;
    return ((unsigned long long)(uint32_t)(int32_t)hi << 32) | (unsigned long long)(uint32_t)lo;
}

// Section 3.1: one forward Euler step of the Lorenz system, fixed order.
__device__ __forceinline__ void euler_step(double &x, double &y, double &z, double dt) {
    const double dx = SIGMA * (y - x);
    const double dy = (x * (RHO - z)) - y;
    const double dz = (x * y) - (BETA * z);
    x = x + dt * dx;
    y = y + dt * dy;
    z = z + dt * dz;
}

// Format variant: the Euler step with each update fused into one rounding (9 roundings).
__device__ __forceinline__ void euler_fma_step(double &x, double &y, double &z, double dt) {
    const double dx = SIGMA * (y - x);
    const double dy = __builtin_fma(x, RHO - z, -y);
    const double dz = __builtin_fma(x, y, -(BETA * z));
    x = __builtin_fma(dt, dx, x);
    y = __builtin_fma(dt, dy, y);
    z = __builtin_fma(dt, dz, z);
}

// Lorenz vector field in the Euler step's evaluation order.
__device__ __forceinline__ void lorenz_field(double x, double y, double z, double &fx, double &fy, double &fz) {
    fx = SIGMA * (y - x);
    fy = (x * (RHO - z)) - y;
    fz = (x * y) - (BETA * z);
}

// Format variant: classical Runge-Kutta 4, r += dt/6 ((k1 + k4) + 2 (k2 + k3)).
__device__ __forceinline__ void rk4_step(double &x, double &y, double &z, double dt, double h2, double h6) {
    double ax, ay, az, bx, by, bz, cx, cy, cz, dx, dy, dz;
    lorenz_field(x, y, z, ax, ay, az);
    lorenz_field(x + h2 * ax, y + h2 * ay, z + h2 * az, bx, by, bz);
    lorenz_field(x + h2 * bx, y + h2 * by, z + h2 * bz, cx, cy, cz);
    lorenz_field(x + dt * cx, y + dt * cy, z + dt * cz, dx, dy, dz);
    x = x + h6 * ((ax + dx) + 2.0 * (bx + cx));
    y = y + h6 * ((ay + dy) + 2.0 * (by + cy));
    z = z + h6 * ((az + dz) + 2.0 * (bz + cz));
}

template <int I>
__device__ __forceinline__ void step(double &x, double &y, double &z, double dt, double h2, double h6) {
    if constexpr (I == LZ_INTEGRATOR_EULER_FMA) euler_fma_step(x, y, z, dt);
    else if constexpr (I == LZ_INTEGRATOR_RK4) rk4_step(x, y, z, dt, h2, h6);
    else euler_step(x, y, z, dt);
}

// Step 2's F^(n_it) for the M chains of a lane, interleaved step by step.
template <int M, int I>
__device__ __forceinline__ void lorenz_steps(double (&x)[M], double (&y)[M], double (&z)[M], double dt,
                                             uint32_t n_it) {
    const double h2 = dt * 0.5, h6 = I == LZ_INTEGRATOR_RK4 ? dt / 6.0 : 0.0;
    // Steps per loop iteration: 60 Euler steps for one chain (a divisor of the default 3000, about 6.7 KB
    // of code), fewer per iteration with more chains; RK4's 68-operation step gains nothing from more.
    constexpr int U = I == LZ_INTEGRATOR_RK4 ? 2 : 60 / M;
    const uint32_t q = n_it / U;
    for (uint32_t i = 0; i < q; ++i) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int m = 0; m < M; ++m) step<I>(x[m], y[m], z[m], dt, h2, h6);
        }
    }
    for (uint32_t i = q * U; i < n_it; ++i) {
#pragma unroll
        for (int m = 0; m < M; ++m) step<I>(x[m], y[m], z[m], dt, h2, h6);
    }
}

// State of the M chains of one lane.
template <int M>
struct Chains {
    double x[M], y[M], z[M];     // r
    double a0[M], a1[M], a2[M];  // alpha
    uint32_t mu0[M], mu1[M], mu2[M];
    uint32_t om0[M], om1[M], om2[M];
    double ap0[M], ap1[M], ap2[M];  // a'
    uint32_t k0[M], k1[M], k2[M];
    uint32_t dec[M];                // 1 = decrypt
};

// Block b starts at r0 + b 2^-24 (every coordinate); alpha_i = r[mu_i] (Eq. alpha, n = 0).
template <int M>
__device__ __forceinline__ void init_chain(Chains<M> &c, int m, const double (&r0)[3], const double (&ap)[3],
                                           const uint8_t (&mu)[3], const uint8_t (&om)[3], const uint8_t (&k)[3],
                                           uint64_t b, uint32_t dec) {
    const double off = (double)b * 0x1p-24;
    c.x[m] = r0[0] + off;
    c.y[m] = r0[1] + off;
    c.z[m] = r0[2] + off;
    c.mu0[m] = mu[0]; c.mu1[m] = mu[1]; c.mu2[m] = mu[2];
    c.om0[m] = om[0]; c.om1[m] = om[1]; c.om2[m] = om[2];
    c.a0[m] = sel3(c.mu0[m], c.x[m], c.y[m], c.z[m]);
    c.a1[m] = sel3(c.mu1[m], c.x[m], c.y[m], c.z[m]);
    c.a2[m] = sel3(c.mu2[m], c.x[m], c.y[m], c.z[m]);
    c.ap0[m] = ap[0]; c.ap1[m] = ap[1]; c.ap2[m] = ap[2];
    c.k0[m] = k[0]; c.k1[m] = k[1]; c.k2[m] = k[2];
    c.dec[m] = dec;
}

__device__ __forceinline__ uint32_t mod_k(uint32_t v, uint32_t k) { return k == 4 ? (v & 3u) : v % 3u; }

// Steps 1-3 of Section 3.2 for one byte of each of the M chains.
template <int M, int I>
__device__ __forceinline__ void crypt_byte(Chains<M> &c, const uint32_t (&bin)[M], uint32_t (&bout)[M], double dt,
                                           uint32_t n_it) {
    uint32_t R1[M], R2[M], p[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        // Step 1: y = (x + R1 + R2) mod 2^8 (encode) or x = (y - R1 - R2) mod 2^8 (decode)
        R1[m] = r_nu(c.a0[m], c.om0[m]);
        R2[m] = r_nu(c.a1[m], c.om1[m]);
        const uint32_t ks = R1[m] + R2[m];
        if (c.dec[m]) {
            p[m] = (bin[m] - ks) & 0xFFu;
            bout[m] = p[m];
        } else {
            p[m] = bin[m];
            bout[m] = (bin[m] + ks) & 0xFFu;
        }
        // Step 2: Theta = P_i / 10^(3 + Omega_3) added to the coordinate mu_3
        const double th = theta_of(p[m], c.om2[m]);
        // r[mu_3] += Theta, written as value selects: a select of the coordinate's address
        // would force the chain state out of registers
        const uint32_t s = c.mu2[m];
        const double moved = sel3(s, c.x[m], c.y[m], c.z[m]) + th;
        c.x[m] = s == 0 ? moved : c.x[m];
        c.y[m] = s == 1 ? moved : c.y[m];
        c.z[m] = s == 2 ? moved : c.z[m];
    }
    // Step 2 (cont.): r <- F^(n_it)(r)
    lorenz_steps<M, I>(c.x, c.y, c.z, dt, n_it);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        // Step 3: mu_i <- (mu_i + R_i) mod 3 with R_i from the old alpha_i, Omega_i
        const uint32_t R3 = r_nu(c.a2[m], c.om2[m]);
        c.mu0[m] = (c.mu0[m] + R1[m]) % 3u;
        c.mu1[m] = (c.mu1[m] + R2[m]) % 3u;
        c.mu2[m] = (c.mu2[m] + R3) % 3u;
        // alpha_i = r[mu_i] (Eq. alpha), then Omega_i <- (Omega_i + R(alpha_i, Omega_i)) mod k_i
        // (the index [(i+2) mod 3]+1 evaluated 1-based is i itself)
        c.a0[m] = sel3(c.mu0[m], c.x[m], c.y[m], c.z[m]);
        c.a1[m] = sel3(c.mu1[m], c.x[m], c.y[m], c.z[m]);
        c.a2[m] = sel3(c.mu2[m], c.x[m], c.y[m], c.z[m]);
        c.om0[m] = mod_k(c.om0[m] + r_nu(c.a0[m], c.om0[m]), c.k0[m]);
        c.om1[m] = mod_k(c.om1[m] + r_nu(c.a1[m], c.om1[m]), c.k1[m]);
        c.om2[m] = mod_k(c.om2[m] + r_nu(c.a2[m], c.om2[m]), c.k2[m]);
        // r <- r + a'
        c.x[m] = c.x[m] + c.ap0[m];
        c.y[m] = c.y[m] + c.ap1[m];
        c.z[m] = c.z[m] + c.ap2[m];
    }
}

// ---- wave-level helpers -------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_xor_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off, WAVE);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off, WAVE);
        v ^= ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

// Per-wave LDS layout: tile rows (64*M x stride), then the chain table.
struct WaveLds {
    uint8_t *tile;
    const uint8_t **in;
    uint8_t **out;
    uint32_t *cnt;
};

// Row stride of the LDS tile: an odd number of 4-byte words past a multiple of 64 banks
// (tile is a multiple of 16), so the 64 lanes reading their own rows hit distinct banks.
__host__ __device__ constexpr size_t tile_stride(int tile) { return (size_t)tile + 4; }
__host__ __device__ constexpr size_t wave_lds_bytes(int m, int tile) {
    return (size_t)WAVE * m * (tile_stride(tile) + 2 * sizeof(void *) + sizeof(uint32_t));
}

template <int M>
__device__ __forceinline__ WaveLds wave_lds(char *base, int tile) {
    WaveLds w;
    w.tile = reinterpret_cast<uint8_t *>(base);
    char *p = base + (size_t)WAVE * M * tile_stride(tile);
    w.in = reinterpret_cast<const uint8_t **>(p);
    p += (size_t)WAVE * M * sizeof(void *);
    w.out = reinterpret_cast<uint8_t **>(p);
    p += (size_t)WAVE * M * sizeof(void *);
    w.cnt = reinterpret_cast<uint32_t *>(p);
    return w;
}

// Runs cnt[m] bytes of every chain of the wave through crypt_byte, staging
// input and output through LDS.  on_stop(m) is called right after chain m's
// last byte (or before the loop when cnt[m] == 0), with c holding that chain's
// state; chains past their end keep running on zero bytes but their results
// are neither stored nor used.
template <int M, int I, typename OnStop>
__device__ __forceinline__ void wave_run(Chains<M> &c, const WaveLds &w, int tile, const uint8_t *const (&in)[M],
                                         uint8_t *const (&out)[M], const uint32_t (&cnt)[M], double dt,
                                         uint32_t n_it, int lane, OnStop on_stop) {
    uint32_t mx = 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        w.in[m * WAVE + lane] = in[m];
        w.out[m * WAVE + lane] = out[m];
        w.cnt[m * WAVE + lane] = cnt[m];
        mx = cnt[m] > mx ? cnt[m] : mx;
        if (cnt[m] == 0) on_stop(m);
    }
    mx = wave_max_u32(mx);
    wave_sync();
    const size_t stride = tile_stride(tile);
    const int rows = WAVE * M;
    for (uint32_t t0 = 0; t0 < mx; t0 += (uint32_t)tile) {
        // stage in: byte u of the wave tile -> row u / tile, column u % tile
        for (int u = lane; u < rows * tile; u += WAVE) {
            const int row = u / tile, col = u % tile;
            const uint32_t j = t0 + (uint32_t)col;
            if (j < w.cnt[row]) w.tile[row * stride + col] = w.in[row][j];
        }
        wave_sync();
        const uint32_t nk = mx - t0 < (uint32_t)tile ? mx - t0 : (uint32_t)tile;
        for (uint32_t kk = 0; kk < nk; ++kk) {
            const uint32_t j = t0 + kk;
            uint32_t bin[M], bout[M];
#pragma unroll
            for (int m = 0; m < M; ++m) bin[m] = j < cnt[m] ? w.tile[(m * WAVE + lane) * stride + kk] : 0u;
            crypt_byte<M, I>(c, bin, bout, dt, n_it);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (j < cnt[m]) w.tile[(m * WAVE + lane) * stride + kk] = (uint8_t)bout[m];
                if (j + 1 == cnt[m]) on_stop(m);
            }
        }
        wave_sync();
        // stage out
        for (int u = lane; u < rows * tile; u += WAVE) {
            const int row = u / tile, col = u % tile;
            const uint32_t j = t0 + (uint32_t)col;
            if (j < w.cnt[row]) w.out[row][j] = w.tile[row * stride + col];
        }
        wave_sync();
    }
}

// ---- plain path: one message ---------------------------------------------------------

struct PlainArgs {
    double ap[3], r0[3];
    uint8_t mu[3], om[3], k[3];
    uint32_t decrypt;
    double dt;
    uint32_t n_it, block_len, tile;
    const uint8_t *in;
    uint8_t *out;
    uint64_t n, nb;
    uint64_t block_base;  // index of the first block (0 for a whole message)
    unsigned long long *tag_acc;
    StreamExtra x;        // read only by the stream instance (X = true)
};

__device__ __forceinline__ void load_slot(Chains<1> &c, const ChainSlot &s, const double (&ap)[3],
                                          const uint8_t (&k)[3], uint32_t dec) {
    c.x[0] = s.r[0]; c.y[0] = s.r[1]; c.z[0] = s.r[2];
    c.a0[0] = s.al[0]; c.a1[0] = s.al[1]; c.a2[0] = s.al[2];
    c.mu0[0] = s.mu[0]; c.mu1[0] = s.mu[1]; c.mu2[0] = s.mu[2];
    c.om0[0] = s.om[0]; c.om1[0] = s.om[1]; c.om2[0] = s.om[2];
    c.ap0[0] = ap[0]; c.ap1[0] = ap[1]; c.ap2[0] = ap[2];
    c.k0[0] = k[0]; c.k1[0] = k[1]; c.k2[0] = k[2];
    c.dec[0] = dec;
}

__device__ __forceinline__ void save_slot(ChainSlot &s, const Chains<1> &c) {
    s.r[0] = c.x[0]; s.r[1] = c.y[0]; s.r[2] = c.z[0];
    s.al[0] = c.a0[0]; s.al[1] = c.a1[0]; s.al[2] = c.a2[0];
    s.mu[0] = (uint8_t)c.mu0[0]; s.mu[1] = (uint8_t)c.mu1[0]; s.mu[2] = (uint8_t)c.mu2[0];
    s.om[0] = (uint8_t)c.om0[0]; s.om[1] = (uint8_t)c.om1[0]; s.om[2] = (uint8_t)c.om2[0];
}

// X: the stream instance (M = 1), whose lanes nb and nb + 1 may carry a.x's head and tail.
template <int M, int I, bool X>
__global__ __launch_bounds__(256) void plain_kernel(PlainArgs a) {
    static_assert(!X || M == 1, "the stream instance runs one chain per lane");
    extern __shared__ char lds[];
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const int wpw = blockDim.x / WAVE;
    const WaveLds w = wave_lds<M>(lds + (size_t)wid * wave_lds_bytes(M, a.tile), a.tile);
    const uint64_t base = ((uint64_t)blockIdx.x * wpw + wid) * WAVE * M;

    Chains<M> c;
    const uint8_t *in[M];
    uint8_t *out[M];
    uint32_t cnt[M];
    bool valid[M];
    unsigned long long d0[M], d1[M], d2[M];
    double r0[3] = {a.r0[0], a.r0[1], a.r0[2]}, ap[3] = {a.ap[0], a.ap[1], a.ap[2]};
    uint8_t mu[3] = {a.mu[0], a.mu[1], a.mu[2]}, om[3] = {a.om[0], a.om[1], a.om[2]},
            k[3] = {a.k[0], a.k[1], a.k[2]};
    // stream instance: 1 = this lane is the head chain, 2 = the tail chain
    const uint32_t n_head = X && a.x.head_slot ? 1u : 0u;
    const uint64_t g0 = base + lane;
    const uint32_t role = !X || g0 < a.nb ? 0u : (g0 == a.nb && n_head ? 1u : (g0 == a.nb + n_head && a.x.tail_slot ? 2u : 0u));
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const uint64_t g = base + (uint64_t)m * WAVE + lane;
        valid[m] = g < a.nb;
        const uint64_t off = g * a.block_len;
        cnt[m] = (valid[m] && off < a.n) ? (uint32_t)(a.n - off < a.block_len ? a.n - off : a.block_len) : 0u;
        in[m] = a.in + (valid[m] && off < a.n ? off : 0);
        out[m] = a.out + (valid[m] && off < a.n ? off : 0);
        init_chain<M>(c, m, r0, ap, mu, om, k, a.block_base + (valid[m] ? g : 0), a.decrypt);
        d0[m] = d1[m] = d2[m] = 0;
    }
    if constexpr (X) {
        if (role == 1) {
            load_slot(c, *a.x.head_slot, ap, k, a.decrypt);
            valid[0] = a.x.head_complete != 0;
            cnt[0] = a.x.head_cnt;
            in[0] = a.x.head_in;
            out[0] = a.x.head_out;
        } else if (role == 2) {
            init_chain<1>(c, 0, r0, ap, mu, om, k, a.x.tail_block, a.decrypt);
            cnt[0] = a.x.tail_cnt;
            in[0] = a.x.tail_in;
            out[0] = a.x.tail_out;
        }
    }
    wave_run<M, I>(c, w, (int)a.tile, in, out, cnt, a.dt, a.n_it, lane, [&](int m) __attribute__((always_inline)) {
        if constexpr (X) {
            if (role == 2 || (role == 1 && !a.x.head_complete)) {
                save_slot(role == 2 ? *a.x.tail_slot : *a.x.head_slot, c);
                return;
            }
        }
        d0[m] = digest_word(c.x[m]);
        d1[m] = digest_word(c.y[m]);
        d2[m] = digest_word(c.z[m]);
    });
    unsigned long long t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
    for (int m = 0; m < M; ++m)
        if (valid[m]) { t0 ^= d0[m]; t1 ^= d1[m]; t2 ^= d2[m]; }
    t0 = wave_xor_u64(t0);
    t1 = wave_xor_u64(t1);
    t2 = wave_xor_u64(t2);
    if (lane == 0 && base < a.nb + (X ? 2 : 0)) {
        atomicXor(&a.tag_acc[0], t0);
        atomicXor(&a.tag_acc[1], t1);
        atomicXor(&a.tag_acc[2], t2);
    }
}

// Encrypt: tag bytes to out_tag.  Decrypt: compare with stored tag, status,
// and zero the body on failure (grid-stride over the body).
__global__ void plain_finalize_kernel(int decrypt, const unsigned long long *tag_acc, const uint8_t *stored,
                                      uint8_t *tag_out, int32_t *status, uint8_t *body, uint64_t n) {
    const unsigned long long t[3] = {tag_acc[0], tag_acc[1], tag_acc[2]};
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!decrypt) {
        if (tid < LZ_TAG_BYTES) tag_out[tid] = (uint8_t)(t[tid / 8] >> (8 * (tid % 8)));
        return;
    }
    bool ok = true;
    for (int q = 0; q < LZ_TAG_BYTES; ++q) ok = ok && stored[q] == (uint8_t)(t[q / 8] >> (8 * (q % 8)));
    if (tid == 0 && status) *status = ok ? LZ_OK : LZ_E_INTEGRITY;
    if (!ok)
        for (uint64_t i = tid; i < n; i += (uint64_t)gridDim.x * blockDim.x) body[i] = 0;
}

// Stores the address of a batch's status array in its slot (read by batch_finalize_kernel).
__global__ void set_status_ref_kernel(int32_t **slot, int32_t *status) { *slot = status; }

__global__ void fill_u64_kernel(unsigned long long *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---- batched path: persistent kernel over a work queue --------------------------------

struct BatchArgs {
    BatchDev b;
    double dt;
    uint32_t n_it, block_len, tile;
};

__device__ __forceinline__ uint32_t find_msg(const uint64_t *prefix, uint32_t n_msg, uint64_t g) {
    // largest i with prefix[i] <= g (prefix is non-decreasing, prefix[0] = 0)
    uint32_t lo = 0, hi = n_msg;  // invariant: prefix[lo] <= g < prefix[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int M, int I>
__global__ __launch_bounds__(256) void batch_kernel(BatchArgs a) {
    extern __shared__ char lds[];
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const WaveLds w = wave_lds<M>(lds + (size_t)wid * wave_lds_bytes(M, a.tile), a.tile);
    const uint64_t per_task = (uint64_t)WAVE * M;
    const uint64_t n_chains = a.b.n_full + a.b.n_tail;

    // No lane-conditional region may sit inside this loop: the compiler is free to merge such
    // regions across the back edge, which leaves lanes re-entering the loop without the others.
    // Every lane therefore takes part in the task grab (lane 0 adds 1, the others 0) and in the
    // tag update (a lane past the end XORs 0).
    for (;;) {
        const unsigned long long grab = atomicAdd(a.b.counter, lane == 0 ? 1ull : 0ull);
        const unsigned long long task =
            ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(grab >> 32)) << 32) |
            __builtin_amdgcn_readfirstlane((uint32_t)grab);
        if (task >= a.b.n_tasks) break;

        Chains<M> c;
        const uint8_t *in[M];
        uint8_t *out[M];
        uint32_t cnt[M], msg[M];
        bool valid[M];
        unsigned long long d0[M], d1[M], d2[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const uint64_t g = task * per_task + (uint64_t)m * WAVE + lane;
            valid[m] = g < n_chains;
            uint32_t i = 0;
            uint64_t b = 0;
            uint32_t len = 0;
            if (valid[m]) {
                if (g < a.b.n_full) {
                    i = find_msg(a.b.full_prefix, a.b.n_msg, g);
                    b = g - a.b.full_prefix[i];
                    len = a.block_len;
                } else {
                    i = a.b.tail_msg[g - a.b.n_full];
                    b = a.b.msgs[i].nb - 1;
                    len = (uint32_t)(a.b.msgs[i].n - b * a.block_len);
                }
            }
            const MsgDesc &md = a.b.msgs[i];
            msg[m] = i;
            cnt[m] = valid[m] ? len : 0u;
            in[m] = md.in + b * a.block_len;
            out[m] = md.out + b * a.block_len;
            const double r0[3] = {md.r0[0], md.r0[1], md.r0[2]}, ap[3] = {md.ap[0], md.ap[1], md.ap[2]};
            const uint8_t mu[3] = {md.mu[0], md.mu[1], md.mu[2]}, om[3] = {md.om[0], md.om[1], md.om[2]},
                          k[3] = {md.k[0], md.k[1], md.k[2]};
            init_chain<M>(c, m, r0, ap, mu, om, k, b, md.decrypt);
            d0[m] = d1[m] = d2[m] = 0;
        }
        wave_run<M, I>(c, w, (int)a.tile, in, out, cnt, a.dt, a.n_it, lane, [&](int m) __attribute__((always_inline)) {
            d0[m] = digest_word(c.x[m]);
            d1[m] = digest_word(c.y[m]);
            d2[m] = digest_word(c.z[m]);
        });
        // tag: XOR of block digests per message, one atomic per lane and word
#pragma unroll
        for (int m = 0; m < M; ++m) {
            unsigned long long *t = &a.b.tag_acc[3 * (size_t)msg[m]];
            atomicXor(t + 0, valid[m] ? d0[m] : 0ull);
            atomicXor(t + 1, valid[m] ? d1[m] : 0ull);
            atomicXor(t + 2, valid[m] ? d2[m] : 0ull);
        }
    }
}

// One workgroup per message: tag out (encrypt) or tag check, status and zeroing (decrypt).
__global__ void batch_finalize_kernel(BatchDev b, int decrypt) {
    const uint32_t i = blockIdx.x;
    if (i >= b.n_msg) return;
    const MsgDesc &md = b.msgs[i];
    const unsigned long long t[3] = {b.tag_acc[3 * (size_t)i], b.tag_acc[3 * (size_t)i + 1],
                                     b.tag_acc[3 * (size_t)i + 2]};
    if (!decrypt) {
        if (threadIdx.x < LZ_TAG_BYTES) {
            const int q = threadIdx.x;
            md.out[md.n + q] = (uint8_t)(t[q / 8] >> (8 * (q % 8)));
        }
        return;
    }
    const uint8_t *stored = md.in + md.n;
    bool ok = true;
    for (int q = 0; q < LZ_TAG_BYTES; ++q) ok = ok && stored[q] == (uint8_t)(t[q / 8] >> (8 * (q % 8)));
    if (threadIdx.x == 0) (*b.status_ref)[i] = ok ? LZ_OK : LZ_E_INTEGRITY;
    if (!ok)
        for (uint64_t j = threadIdx.x; j < md.n; j += blockDim.x) md.out[j] = 0;
}

// ---- served path: resumable chains ------------------------------------------------------

struct TickArgs {
    TickDev t;
    double dt;
    uint32_t n_it, block_len, tile;
};

template <int M, int I>
__global__ __launch_bounds__(256) void tick_kernel(TickArgs a) {
    extern __shared__ char lds[];
    const int lane = threadIdx.x % WAVE;
    const int wid = threadIdx.x / WAVE;
    const int wpw = blockDim.x / WAVE;
    const WaveLds w = wave_lds<M>(lds + (size_t)wid * wave_lds_bytes(M, a.tile), a.tile);
    const uint64_t base = ((uint64_t)blockIdx.x * wpw + wid) * WAVE * M;

    Chains<M> c;
    const uint8_t *in[M];
    uint8_t *out[M];
    uint32_t cnt[M], slot[M];
    bool valid[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const uint64_t e = base + (uint64_t)m * WAVE + lane;
        valid[m] = e < a.t.n_list;
        slot[m] = valid[m] ? a.t.list[e] : 0u;
        cnt[m] = 0;
        in[m] = nullptr;
        out[m] = nullptr;
        if (!valid[m]) {  // past the end of the list: idle lane, touches no memory
            const double z3[3] = {0.0, 0.0, 0.0};
            const uint8_t u3[3] = {0, 0, 0}, k3[3] = {4, 4, 4};
            init_chain<M>(c, m, z3, z3, u3, u3, k3, 0, 0);
            continue;
        }
        const ChainSlot &s = a.t.slots[slot[m]];
        const MsgDesc &md = a.t.reqs[s.req].m;
        const double ap[3] = {md.ap[0], md.ap[1], md.ap[2]};
        const uint8_t k[3] = {md.k[0], md.k[1], md.k[2]};
        if (s.fresh) {
            const double r0[3] = {md.r0[0], md.r0[1], md.r0[2]};
            const uint8_t mu[3] = {md.mu[0], md.mu[1], md.mu[2]}, om[3] = {md.om[0], md.om[1], md.om[2]};
            init_chain<M>(c, m, r0, ap, mu, om, k, s.blk, md.decrypt);
        } else {
            c.x[m] = s.r[0]; c.y[m] = s.r[1]; c.z[m] = s.r[2];
            c.a0[m] = s.al[0]; c.a1[m] = s.al[1]; c.a2[m] = s.al[2];
            c.mu0[m] = s.mu[0]; c.mu1[m] = s.mu[1]; c.mu2[m] = s.mu[2];
            c.om0[m] = s.om[0]; c.om1[m] = s.om[1]; c.om2[m] = s.om[2];
            c.ap0[m] = ap[0]; c.ap1[m] = ap[1]; c.ap2[m] = ap[2];
            c.k0[m] = k[0]; c.k1[m] = k[1]; c.k2[m] = k[2];
            c.dec[m] = md.decrypt;
        }
        const uint32_t left = s.len - s.pos;
        cnt[m] = left < a.t.tick_bytes ? left : a.t.tick_bytes;
        const uint64_t off = (uint64_t)s.blk * a.block_len + s.pos;
        in[m] = md.in + off;
        out[m] = md.out + off;
    }
    wave_run<M, I>(c, w, (int)a.tile, in, out, cnt, a.dt, a.n_it, lane, [&](int m) __attribute__((always_inline)) {
        if (!valid[m]) return;
        ChainSlot &s = a.t.slots[slot[m]];
        s.r[0] = c.x[m]; s.r[1] = c.y[m]; s.r[2] = c.z[m];
        s.al[0] = c.a0[m]; s.al[1] = c.a1[m]; s.al[2] = c.a2[m];
        s.mu[0] = (uint8_t)c.mu0[m]; s.mu[1] = (uint8_t)c.mu1[m]; s.mu[2] = (uint8_t)c.mu2[m];
        s.om[0] = (uint8_t)c.om0[m]; s.om[1] = (uint8_t)c.om1[m]; s.om[2] = (uint8_t)c.om2[m];
    });
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (!valid[m]) continue;
        ChainSlot &s = a.t.slots[slot[m]];
        s.fresh = 0;
        s.pos += cnt[m];
        if (s.pos != s.len) continue;
        ReqDesc &rq = a.t.reqs[s.req];
        atomicXor(&rq.tag[0], digest_word(s.r[0]));
        atomicXor(&rq.tag[1], digest_word(s.r[1]));
        atomicXor(&rq.tag[2], digest_word(s.r[2]));
        __threadfence();
        if (atomicSub(&rq.remaining, 1u) != 1u) continue;
        // last chain of the request: every other chain's tag XOR is visible
        __threadfence();
        const unsigned long long t[3] = {atomicXor(&rq.tag[0], 0ull), atomicXor(&rq.tag[1], 0ull),
                                         atomicXor(&rq.tag[2], 0ull)};
        int32_t st = LZ_OK;
        if (!rq.m.decrypt) {
            for (int q = 0; q < LZ_TAG_BYTES; ++q) rq.m.out[rq.m.n + q] = (uint8_t)(t[q / 8] >> (8 * (q % 8)));
        } else {
            for (int q = 0; q < LZ_TAG_BYTES; ++q)
                if (rq.stored_tag[q] != (uint8_t)(t[q / 8] >> (8 * (q % 8)))) st = LZ_E_INTEGRITY;
        }
        rq.status = st;
        const uint32_t at = atomicAdd(a.t.done_count, 1u);
        a.t.done_queue[at] = (s.req << 1) | (st != LZ_OK ? 1u : 0u);
    }
}

// ---- streaming ----------------------------------------------------------------------------

// End of a stream: fold in the pending partial block (or, for an empty message, block 0's
// initial state), then write the tag (encrypt) or compare it (decrypt).
__global__ void stream_finish_kernel(const ChainSlot *slot, int pending, int empty, double r00, double r01, double r02,
                                     unsigned long long *tag_acc, int decrypt, uint8_t *tag, int32_t *status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long t[3] = {tag_acc[0], tag_acc[1], tag_acc[2]};
    if (pending) {
        t[0] ^= digest_word(slot->r[0]);
        t[1] ^= digest_word(slot->r[1]);
        t[2] ^= digest_word(slot->r[2]);
    } else if (empty) {
        t[0] ^= digest_word(r00);
        t[1] ^= digest_word(r01);
        t[2] ^= digest_word(r02);
    }
    if (!decrypt) {
        for (int q = 0; q < LZ_TAG_BYTES; ++q) tag[q] = (uint8_t)(t[q / 8] >> (8 * (q % 8)));
        return;
    }
    bool ok = true;
    for (int q = 0; q < LZ_TAG_BYTES; ++q) ok = ok && tag[q] == (uint8_t)(t[q / 8] >> (8 * (q % 8)));
    *status = ok ? LZ_OK : LZ_E_INTEGRITY;
}

// ---- the method's scalar pieces over arrays, for checking them one by one -----------

__global__ void unit_r_kernel(const double *alpha, const uint8_t *om, size_t n, uint8_t *out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (uint8_t)r_nu(alpha[i], om[i] & 3u);
}

__global__ void unit_theta_kernel(const uint8_t *p, const uint8_t *o3, size_t n, double *out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = theta_of(p[i], o3[i] & 3u);
}

// F^steps of Step 2 (the cipher kernels' loop) on each state (x, y, z).
template <int I>
__global__ void unit_lorenz_kernel(double *r, size_t n, double dt, uint32_t steps) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[1] = {r[3 * i]}, y[1] = {r[3 * i + 1]}, z[1] = {r[3 * i + 2]};
    lorenz_steps<1, I>(x, y, z, dt, steps);
    r[3 * i] = x[0];
    r[3 * i + 1] = y[0];
    r[3 * i + 2] = z[0];
}

// Zeroes the body of each listed request (failed decryptions), one workgroup each.
__global__ void req_zero_kernel(const ReqDesc *reqs, const uint32_t *ids, uint32_t n) {
    if (blockIdx.x >= n) return;
    const MsgDesc &md = reqs[ids[blockIdx.x]].m;
    for (uint64_t j = threadIdx.x; j < md.n; j += blockDim.x) md.out[j] = 0;
}

// Installs newly admitted requests: record i goes to reqs[meta[3i]], and its
// meta[3i+1] chains (slot indices idx[meta[3i+2] ..]) start fresh at byte 0.
__global__ void install_kernel(ReqDesc *reqs, ChainSlot *slots, const ReqDesc *staged, const uint32_t *meta,
                               const uint32_t *idx, uint32_t n_new, uint32_t block_len) {
    const uint32_t i = blockIdx.x;
    if (i >= n_new) return;
    const uint32_t rs = meta[3 * i], nb = meta[3 * i + 1], first = meta[3 * i + 2];
    if (threadIdx.x == 0) reqs[rs] = staged[i];
    const uint64_t n = staged[i].m.n;
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        ChainSlot &c = slots[idx[first + b]];
        const uint64_t off = (uint64_t)b * block_len;
        c.fresh = 1;
        c.pos = 0;
        c.len = n == 0 ? 0u : (uint32_t)(n - off < block_len ? n - off : block_len);
        c.req = rs;
        c.blk = b;
    }
}

template <int M, typename F>
hipError_t dispatch_i(uint32_t integ, F f) {
    switch (integ) {
        case LZ_INTEGRATOR_EULER: return f(std::integral_constant<int, M>{}, std::integral_constant<int, 0>{});
        case LZ_INTEGRATOR_EULER_FMA: return f(std::integral_constant<int, M>{}, std::integral_constant<int, 1>{});
        case LZ_INTEGRATOR_RK4: return f(std::integral_constant<int, M>{}, std::integral_constant<int, 2>{});
        default: return hipErrorInvalidValue;
    }
}

// Calls f(M, I) with the compile-time chains-per-lane and integrator of the launch.
template <typename F>
hipError_t dispatch(int m, uint32_t integ, F f) {
    switch (m) {
        case 1: return dispatch_i<1>(integ, f);
        case 2: return dispatch_i<2>(integ, f);
        case 4: return dispatch_i<4>(integ, f);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t lds_bytes(const KernelShape &sh) { return (size_t)(sh.wg / WAVE) * wave_lds_bytes(sh.m, sh.tile); }

bool shape_valid(const KernelShape &sh, const DevInfo &dev) {
    if (sh.m != 1 && sh.m != 2 && sh.m != 4) return false;
    if (sh.wg != 64 && sh.wg != 128 && sh.wg != 256) return false;
    if (sh.tile != 16 && sh.tile != 32 && sh.tile != 64 && sh.tile != 128) return false;
    if (sh.wps < 1 || sh.wps > 8) return false;
    return lds_bytes(sh) <= (size_t)dev.lds_per_wg_max;
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

namespace {

PlainArgs plain_args(const KernelShape &sh, const lz_key &key, const lz_params &prm, int decrypt, const uint8_t *in,
                     uint8_t *out, uint64_t n, uint64_t nb, unsigned long long *tag_acc, uint64_t block_base) {
    PlainArgs a{};
    for (int j = 0; j < 3; ++j) {
        a.ap[j] = key.a_prime[j];
        a.r0[j] = key.r0[j];
        a.mu[j] = key.mu[j];
        a.om[j] = key.omega[j];
        a.k[j] = key.k[j];
    }
    a.decrypt = (uint32_t)decrypt;
    a.dt = prm.dt;
    a.n_it = prm.n_it;
    a.block_len = prm.block_len;
    a.tile = (uint32_t)sh.tile;
    a.in = in;
    a.out = out;
    a.n = n;
    a.nb = nb;
    a.block_base = block_base;
    a.tag_acc = tag_acc;
    return a;
}

}  // namespace

hipError_t launch_plain(const KernelShape &sh, const lz_key &key, const lz_params &prm, int decrypt,
                        const uint8_t *in, uint8_t *out, uint64_t n, unsigned long long *tag_acc, hipStream_t s,
                        uint64_t block_base) {
    const uint64_t nb = n == 0 ? 1 : (n + prm.block_len - 1) / prm.block_len;
    const PlainArgs a = plain_args(sh, key, prm, decrypt, in, out, n, nb, tag_acc, block_base);
    const uint64_t per_wg = (uint64_t)sh.wg * sh.m;
    const uint64_t grid = (a.nb + per_wg - 1) / per_wg;
    const size_t lds = lds_bytes(sh);
    return dispatch(sh.m, prm.integrator, [&](auto mc, auto ic) {
        constexpr int M = decltype(mc)::value;
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((plain_kernel<M, I, false>), dim3((unsigned)grid), dim3(sh.wg), lds, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_stream_step(const KernelShape &shape, const lz_key &key, const lz_params &prm, int decrypt,
                              const uint8_t *in, uint8_t *out, uint64_t full, uint64_t block_base,
                              const StreamExtra &x, unsigned long long *tag_acc, hipStream_t s) {
    const KernelShape sh{1, shape.wg, shape.tile, shape.wps};
    PlainArgs a = plain_args(sh, key, prm, decrypt, in, out, full * prm.block_len, full, tag_acc, block_base);
    a.x = x;
    const uint64_t lanes = full + (x.head_slot ? 1 : 0) + (x.tail_slot ? 1 : 0);
    if (lanes == 0) return hipSuccess;
    const uint64_t grid = (lanes + sh.wg - 1) / sh.wg;
    const size_t lds = lds_bytes(sh);
    return dispatch_i<1>(prm.integrator, [&](auto, auto ic) {
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((plain_kernel<1, I, true>), dim3((unsigned)grid), dim3(sh.wg), lds, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_plain_finalize(int decrypt, const unsigned long long *tag_acc, const uint8_t *stored_tag,
                                 uint8_t *tag_out, int32_t *status, uint8_t *body, uint64_t n, hipStream_t s) {
    unsigned blocks = 1;
    if (decrypt) {
        const uint64_t want = (n + 256 * 16 - 1) / (256 * 16);
        blocks = (unsigned)(want < 1 ? 1 : (want > 2048 ? 2048 : want));
    }
    hipLaunchKernelGGL(plain_finalize_kernel, dim3(blocks), dim3(256), 0, s, decrypt, tag_acc, stored_tag, tag_out,
                       status, body, n);
    return hipGetLastError();
}

hipError_t launch_batch(const KernelShape &sh, const DevInfo &dev, const lz_params &prm, const BatchDev &b,
                        hipStream_t s) {
    BatchArgs a;
    a.b = b;
    a.dt = prm.dt;
    a.n_it = prm.n_it;
    a.block_len = prm.block_len;
    a.tile = (uint32_t)sh.tile;
    // persistent grid: wps waves on each of the 4 SIMDs of every CU, but no more than the tasks
    const uint64_t waves = (uint64_t)dev.cus * 4 * sh.wps;
    const uint64_t wpw = (uint64_t)sh.wg / WAVE;
    uint64_t grid = (waves + wpw - 1) / wpw;
    const uint64_t need = (b.n_tasks + wpw - 1) / wpw;
    if (need < grid) grid = need ? need : 1;
    const size_t lds = lds_bytes(sh);
    return dispatch(sh.m, prm.integrator, [&](auto mc, auto ic) {
        constexpr int M = decltype(mc)::value;
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((batch_kernel<M, I>), dim3((unsigned)grid), dim3(sh.wg), lds, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_set_status_ref(int32_t **slot, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(set_status_ref_kernel, dim3(1), dim3(1), 0, s, slot, status);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchDev &b, int decrypt, hipStream_t s) {
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(b.n_msg ? b.n_msg : 1), dim3(256), 0, s, b, decrypt);
    return hipGetLastError();
}

hipError_t launch_tick(const KernelShape &sh, const lz_params &prm, const TickDev &t, hipStream_t s) {
    if (t.n_list == 0) return hipSuccess;
    TickArgs a;
    a.t = t;
    a.dt = prm.dt;
    a.n_it = prm.n_it;
    a.block_len = prm.block_len;
    a.tile = (uint32_t)sh.tile;
    const uint64_t per_wg = (uint64_t)sh.wg * sh.m;
    const uint64_t grid = (t.n_list + per_wg - 1) / per_wg;
    const size_t lds = lds_bytes(sh);
    return dispatch(sh.m, prm.integrator, [&](auto mc, auto ic) {
        constexpr int M = decltype(mc)::value;
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((tick_kernel<M, I>), dim3((unsigned)grid), dim3(sh.wg), lds, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_unit_r(const double *alpha, const uint8_t *om, size_t n, uint8_t *out, hipStream_t s) {
    const size_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(unit_r_kernel, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s, alpha, om, n, out);
    return hipGetLastError();
}

hipError_t launch_unit_theta(const uint8_t *p, const uint8_t *o3, size_t n, double *out, hipStream_t s) {
    const size_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(unit_theta_kernel, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s, p, o3, n, out);
    return hipGetLastError();
}

hipError_t launch_unit_lorenz(const lz_params &prm, double *r, size_t n, uint32_t steps, hipStream_t s) {
    const size_t blocks = (n + 255) / 256;
    return dispatch_i<1>(prm.integrator, [&](auto, auto ic) {
        constexpr int I = decltype(ic)::value;
        hipLaunchKernelGGL((unit_lorenz_kernel<I>), dim3((unsigned)blocks), dim3(256), 0, s, r, n, prm.dt, steps);
        return hipGetLastError();
    });
}

hipError_t launch_stream_finish(const ChainSlot *slot, int pending, int empty, const lz_key &key,
                                unsigned long long *tag_acc, int decrypt, uint8_t *tag, int32_t *status,
                                hipStream_t s) {
    hipLaunchKernelGGL(stream_finish_kernel, dim3(1), dim3(64), 0, s, slot, pending, empty, key.r0[0], key.r0[1],
                       key.r0[2], tag_acc, decrypt, tag, status);
    return hipGetLastError();
}

hipError_t launch_install(ReqDesc *reqs, ChainSlot *slots, const ReqDesc *staged, const uint32_t *meta,
                          const uint32_t *idx, uint32_t n_new, uint32_t block_len, hipStream_t s) {
    if (n_new == 0) return hipSuccess;
    hipLaunchKernelGGL(install_kernel, dim3(n_new), dim3(256), 0, s, reqs, slots, staged, meta, idx, n_new,
                       block_len);
    return hipGetLastError();
}

hipError_t launch_req_zero(const ReqDesc *reqs, const uint32_t *req_ids, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(req_zero_kernel, dim3(n), dim3(256), 0, s, reqs, req_ids, n);
    return hipGetLastError();
}

}  // namespace lz
