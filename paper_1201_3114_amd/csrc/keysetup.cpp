// Password stage of Section 3.1 on the host: pi -> a = (a1,a2,a3), D, a',
// r0 = a' + lambda, mu, Omega.  Per message, microseconds; the device never
// sees the password, only the 64-byte lz_key.
//
// a_j has at most 8(L+1) <= 176 bits (L = floor(n_pi/3) <= 21), so the
// integers are held in fixed 32-bit-limb naturals.  a' = a_j / 10^D is
// rounded to nearest-even by exact long division (the quotient is taken to
// 53 significant bits plus the exact remainder), SHA-256 follows FIPS 180-4.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "internal.h"

namespace lz {
namespace {

// ---- fixed-width naturals ---------------------------------------------------

constexpr int LIMBS = 16;  // 512 bits: a_i a_j < 2^352, 10^D << 53 < 2^240

struct Nat {
    uint32_t w[LIMBS];
    Nat() { std::memset(w, 0, sizeof w); }
    explicit Nat(uint64_t v) : Nat() {
        w[0] = static_cast<uint32_t>(v);
        w[1] = static_cast<uint32_t>(v >> 32);
    }
    bool is_zero() const {
        for (uint32_t x : w)
            if (x) return false;
        return true;
    }
    int bit_length() const {
        for (int i = LIMBS - 1; i >= 0; --i)
            if (w[i]) return 32 * i + 32 - __builtin_clz(w[i]);
        return 0;
    }
    bool bit(int i) const { return (w[i >> 5] >> (i & 31)) & 1u; }
};

int cmp(const Nat &a, const Nat &b) {
    for (int i = LIMBS - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

Nat add(const Nat &a, const Nat &b) {
    Nat r;
    uint64_t c = 0;
    for (int i = 0; i < LIMBS; ++i) {
        c += static_cast<uint64_t>(a.w[i]) + b.w[i];
        r.w[i] = static_cast<uint32_t>(c);
        c >>= 32;
    }
    return r;
}

Nat sub(const Nat &a, const Nat &b) {  // requires a >= b
    Nat r;
    int64_t br = 0;
    for (int i = 0; i < LIMBS; ++i) {
        int64_t d = static_cast<int64_t>(a.w[i]) - b.w[i] - br;
        br = d < 0;
        r.w[i] = static_cast<uint32_t>(d + (br << 32));
    }
    return r;
}

Nat mul(const Nat &a, const Nat &b) {
    Nat r;
    for (int i = 0; i < LIMBS; ++i) {
        uint64_t c = 0;
        if (!a.w[i]) continue;
        for (int j = 0; i + j < LIMBS; ++j) {
            c += static_cast<uint64_t>(a.w[i]) * b.w[j] + r.w[i + j];
            r.w[i + j] = static_cast<uint32_t>(c);
            c >>= 32;
        }
    }
    return r;
}

Nat shl(const Nat &a, int s) {
    Nat r;
    int q = s >> 5, b = s & 31;
    for (int i = LIMBS - 1; i >= q; --i) {
        uint64_t v = static_cast<uint64_t>(a.w[i - q]) << b;
        if (b && i - q - 1 >= 0) v |= a.w[i - q - 1] >> (32 - b);
        r.w[i] = static_cast<uint32_t>(v);
    }
    return r;
}

uint32_t mod_small(const Nat &a, uint32_t m) {
    uint64_t r = 0;
    for (int i = LIMBS - 1; i >= 0; --i) r = ((r << 32) | a.w[i]) % m;
    return static_cast<uint32_t>(r);
}

// q = floor(num / den), rem = num - q den (shift-subtract long division).
void divmod(const Nat &num, const Nat &den, Nat &q, Nat &rem) {
    q = Nat();
    rem = Nat();
    for (int i = num.bit_length() - 1; i >= 0; --i) {
        rem = shl(rem, 1);
        rem.w[0] |= num.bit(i) ? 1u : 0u;
        if (cmp(rem, den) >= 0) {
            rem = sub(rem, den);
            q.w[i >> 5] |= 1u << (i & 31);
        }
    }
}

// Nearest-even binary64 of num/den for 0 <= num < den (so no overflow and,
// since den < 2^200, no subnormal result).
double ratio_to_double(const Nat &num, const Nat &den) {
    if (num.is_zero()) return 0.0;
    // e with 2^e <= num/den < 2^(e+1): start from the bit lengths and correct.
    int e = num.bit_length() - den.bit_length();
    auto scaled_ge = [&](int ee) {  // num/den >= 2^ee ?
        return ee >= 0 ? cmp(num, shl(den, ee)) >= 0 : cmp(shl(num, -ee), den) >= 0;
    };
    if (!scaled_ge(e)) --e;
    // q = floor(num 2^(52-e) / den) lies in [2^52, 2^53).
    const int s = 52 - e;
    Nat n2 = s >= 0 ? shl(num, s) : num;
    Nat d2 = s >= 0 ? den : shl(den, -s);
    Nat q, rem;
    divmod(n2, d2, q, rem);
    uint64_t m = static_cast<uint64_t>(q.w[0]) | (static_cast<uint64_t>(q.w[1]) << 32);
    Nat twice = shl(rem, 1);
    int c = cmp(twice, d2);
    if (c > 0 || (c == 0 && (m & 1u))) ++m;  // round half to even
    return std::ldexp(static_cast<double>(m), e - 52);
}

// ---- SHA-256 (FIPS 180-4) ---------------------------------------------------

constexpr uint32_t K256[64] = {
    0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
    0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
    0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
    0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
    0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
    0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
    0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
    0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};

inline uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

void sha256_block(uint32_t H[8], const uint8_t *blk) {
    uint32_t W[64];
    for (int t = 0; t < 16; ++t)
        W[t] = (uint32_t)blk[4 * t] << 24 | (uint32_t)blk[4 * t + 1] << 16 | (uint32_t)blk[4 * t + 2] << 8 |
               (uint32_t)blk[4 * t + 3];
    for (int t = 16; t < 64; ++t) {
        uint32_t s0 = rotr(W[t - 15], 7) ^ rotr(W[t - 15], 18) ^ (W[t - 15] >> 3);
        uint32_t s1 = rotr(W[t - 2], 17) ^ rotr(W[t - 2], 19) ^ (W[t - 2] >> 10);
        W[t] = W[t - 16] + s0 + W[t - 7] + s1;
    }
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
    for (int t = 0; t < 64; ++t) {
        uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        uint32_t ch = (e & f) ^ (~e & g);
        uint32_t T1 = h + S1 + ch + K256[t] + W[t];
        uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
        uint32_t T2 = S0 + maj;
        h = g; g = f; f = e; e = d + T1; d = c; c = b; b = a; a = T1 + T2;
    }
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e; H[5] += f; H[6] += g; H[7] += h;
}

}  // namespace

void sha256(const uint8_t *msg, size_t len, uint8_t out[32]) {
    uint32_t H[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                     0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};
    size_t full = len / 64;
    for (size_t i = 0; i < full; ++i) sha256_block(H, msg + 64 * i);
    uint8_t tail[128];
    size_t rem = len - 64 * full;
    std::memset(tail, 0, sizeof tail);
    std::memcpy(tail, msg + 64 * full, rem);
    tail[rem] = 0x80;
    size_t tlen = rem + 1 + 8 <= 64 ? 64 : 128;
    uint64_t bits = static_cast<uint64_t>(len) * 8;
    for (int i = 0; i < 8; ++i) tail[tlen - 1 - i] = static_cast<uint8_t>(bits >> (8 * i));
    sha256_block(H, tail);
    if (tlen == 128) sha256_block(H, tail + 64);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 4; ++j) out[4 * i + j] = static_cast<uint8_t>(H[i] >> (24 - 8 * j));
}

// Section 3.1.  pi_i of the paper (1-based) is pw[i-1].
int key_setup(const uint8_t *pw, size_t n, const lz_params &prm, lz_key &key) {
    if (!pw || n == 0 || n > LZ_MAX_PASSWORD) return LZ_E_INVAL;
    const size_t L = n / 3;
    auto pi = [&](size_t i) { return static_cast<uint64_t>(pw[i - 1]); };
    auto term = [&](size_t i, size_t byte_pos) { return shl(Nat(pi(i)), static_cast<int>(8 * byte_pos)); };

    Nat a[3];
    // a1: sum_{i=1..L} pi_i 2^(8(i-1)), or with a leading pi_{3L+1} when n mod 3 != 0
    for (size_t i = 1; i <= L; ++i) a[0] = add(a[0], term(i, n % 3 == 0 ? i - 1 : i));
    if (n % 3 != 0) a[0] = add(a[0], Nat(pi(3 * L + 1)));
    // a2: sum_{i=L+1..2L} pi_i 2^(8(i-L-1)), or shifted one byte plus pi_{3L+2} when n mod 3 == 2
    for (size_t i = L + 1; i <= 2 * L; ++i) a[1] = add(a[1], term(i, n % 3 == 2 ? i - L : i - L - 1));
    if (n % 3 == 2) a[1] = add(a[1], Nat(pi(3 * L + 2)));
    // a3: sum_{i=2L+1..3L} pi_i 2^(8(i-2L-1))
    for (size_t i = 2 * L + 1; i <= 3 * L; ++i) a[2] = add(a[2], term(i, i - 2 * L - 1));

    // D = ceil(log10 2^(8(L+1))): the least D with 10^D > 2^(8(L+1)) (never equal).
    const Nat p2 = shl(Nat(1), static_cast<int>(8 * (L + 1)));
    Nat ten_d(1);
    while (cmp(ten_d, p2) <= 0) ten_d = mul(ten_d, Nat(10));

    for (int j = 0; j < 3; ++j) {
        key.a_prime[j] = ratio_to_double(a[j], ten_d);
        key.r0[j] = key.a_prime[j] + prm.lambda[j];
    }

    const uint32_t m0 = mod_small(a[0], 3), m1 = mod_small(a[1], 3), m2 = mod_small(a[2], 3);
    key.mu[0] = static_cast<uint8_t>((m0 + m1 + m2) % 3);
    key.mu[1] = static_cast<uint8_t>((m0 * m1 + m2) % 3);
    key.mu[2] = static_cast<uint8_t>((m0 + m1 * m2) % 3);

    // Omega_i = SHA-256(LE32(i a1) || LE32(i a2) || LE32(i a3)) mod k_i, digest big-endian.
    for (int i = 1; i <= 3; ++i) {
        uint8_t msg[96], dig[32];
        for (int j = 0; j < 3; ++j) {
            Nat ia = mul(a[j], Nat(static_cast<uint64_t>(i)));
            for (int q = 0; q < 32; ++q) msg[32 * j + q] = static_cast<uint8_t>(ia.w[q >> 2] >> (8 * (q & 3)));
        }
        sha256(msg, sizeof msg, dig);
        uint32_t r = 0;
        for (int q = 0; q < 32; ++q) r = (r * 256u + dig[q]) % prm.k[i - 1];
        key.omega[i - 1] = static_cast<uint8_t>(r);
        key.k[i - 1] = prm.k[i - 1];
    }
    std::memset(key.reserved, 0, sizeof key.reserved);
    return LZ_OK;
}

}  // namespace lz
