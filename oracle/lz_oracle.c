/*
 * lz_oracle.c -- CPU oracle for the Lorenz-attractor chaotic cipher of
 * Marco, Martinez and Bruno, "Fast, parallel and secure cryptography
 * algorithm using Lorenz's attractor" (arXiv:1201.3114).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no source with the GPU library (paper_1201_3114_amd/csrc) and includes none
 * of its headers; the hash is OpenSSL's SHA-256, the decimal rounding of a'
 * is glibc's correctly rounded strtod.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        lz_oracle.c -lcrypto -lpthread -lm
 * (x86-64 SSE2 doubles: every operation below is one IEEE binary64
 * round-to-nearest-even operation, no contraction, no reassociation.)
 *
 * Readings of the paper taken here (the paper is silent or garbled at these
 * points):
 *   - the Euler map of Section 3.1 is the standard forward Euler step of the
 *     Lorenz system, evaluated in the fixed order of lorenz_euler_step();
 *   - log in g(x) of Section 3.1 is log10, so D = digit count of 2^(8(L+1))
 *     and nu = floor(log10 2^(xi-6)) = 13;
 *   - lambda = (1,1,1), k = (4,4,4), dt = 0.01, n_it = 3000 Euler steps per
 *     byte (parameters, not constants);
 *   - hash(i a) is SHA-256 of LE32(i a1) || LE32(i a2) || LE32(i a3), the
 *     digest read as a big-endian integer;
 *   - the alpha index [(i+2) mod 3]+1 of Step 3 is evaluated literally
 *     (1-based), which is alpha_i;
 *   - the parallel version (Section 5) cuts the message into blocks of
 *     block_len bytes; block b starts from r0 + b 2^-24 on every coordinate;
 *   - integrity (Abstract, end of Section 2): the ciphertext carries a
 *     24-byte tag, the XOR over blocks of (N(x),N(y),N(z)) of each block's
 *     final state, N(v) = floor(v 1e13) as a two's complement 64-bit integer.
 *
 * Domain.  R and N read floor(v 1e13) as a 64-bit integer, which needs
 * |v| < 2^63 / 1e13.  Forward Euler leaves the attractor for some steps and
 * starting points the paper allows (dt near its bound of 0.027, or a start
 * far outside the lambda ranges); the trajectory then overflows.  The oracle
 * checks every coordinate after each byte's iterations and at the end of a
 * block: a coordinate that is not finite or has |v| >= 2^19 stops the
 * computation with ORC_E_ESCAPED instead of reading an undefined integer.
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <openssl/sha.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---- parameters (Section 3.1) ------------------------------------------ */

typedef struct {
    double dt;          /* Euler step delta t, 0 < dt <= 0.027 in the paper  */
    double lambda[3];   /* offset of the starting point, Eq. r0 = a' + lambda */
    uint32_t n_it;      /* Euler steps applied per byte                       */
    uint32_t block_len; /* bytes per independent block (parallel version)     */
    uint32_t k[3];      /* moduli of the byte indices Omega, 2 < k_i <= 4     */
    uint32_t integrator; /* 0 Euler (the method), 1 Euler with fused multiply-add,
                            2 classical Runge-Kutta 4 (Section 3.1 leaves the
                            integrator open to other schemes)                  */
} orc_params;

/* Output of the password stage of Section 3.1. */
typedef struct {
    double a_prime[3]; /* a' = a / 10^D                 */
    double r0[3];      /* r0 = a' + lambda              */
    int32_t mu[3];     /* coordinate selectors          */
    int32_t omega[3];  /* byte indices                  */
    int32_t k[3];
    int32_t D;         /* decimal exponent of g()       */
    int32_t L;         /* floor(n_pi / 3)               */
} orc_key;

static const double SIGMA = 10.0;
static const double RHO = 28.0;
static const double BETA = 8.0 / 3.0;
static const double SCALE_NU = 1e13; /* 10^nu, nu = floor(log10 2^(52-6)) = 13 */

#define ORC_E_ESCAPED (-4) /* a coordinate left the domain of R and N (see the file header) */

/* |v| < 2^19 keeps |v 1e13| < 2^63; false for infinities and NaN */
static int in_domain(double v) { return fabs(v) < 0x1p19; }

/* ---- little-endian byte bignums for the password integers ---------------- */

#define NB 96 /* bytes; a_j < 2^176, products a_i a_j < 2^352 */
typedef struct { uint8_t b[NB]; } big;

static void big_zero(big *x) { memset(x->b, 0, NB); }

/* x += v * 256^shift, with carry propagation */
static void big_add_shifted(big *x, unsigned v, int shift) {
    unsigned carry = v;
    for (int i = shift; i < NB && carry; i++) {
        unsigned s = x->b[i] + (carry & 0xFFu);
        carry >>= 8;
        x->b[i] = (uint8_t)(s & 0xFFu);
        carry += s >> 8;
    }
}

static void big_add(big *x, const big *y) {
    unsigned carry = 0;
    for (int i = 0; i < NB; i++) {
        unsigned s = (unsigned)x->b[i] + y->b[i] + carry;
        x->b[i] = (uint8_t)s;
        carry = s >> 8;
    }
}

static void big_mul(big *out, const big *x, const big *y) {
    unsigned acc[2 * NB];
    memset(acc, 0, sizeof acc);
    for (int i = 0; i < NB; i++)
        for (int j = 0; i + j < NB; j++)
            acc[i + j] += (unsigned)x->b[i] * y->b[j];
    unsigned carry = 0;
    for (int i = 0; i < NB; i++) {
        unsigned s = acc[i] + carry;
        out->b[i] = (uint8_t)s;
        carry = s >> 8;
    }
}

static void big_mul_small(big *out, const big *x, unsigned m) {
    unsigned carry = 0;
    for (int i = 0; i < NB; i++) {
        unsigned s = (unsigned)x->b[i] * m + carry;
        out->b[i] = (uint8_t)s;
        carry = s >> 8;
    }
}

/* x mod m, x read as a little-endian integer */
static unsigned big_mod_small(const big *x, unsigned m) {
    unsigned r = 0;
    for (int i = NB - 1; i >= 0; i--) r = (r * 256u + x->b[i]) % m;
    return r;
}

/* decimal digits of x (no leading zeros, "0" for zero) */
static void big_to_decimal(const big *x, char *out, size_t cap) {
    big t = *x;
    char rev[512];
    int n = 0;
    for (;;) {
        int nonzero = 0;
        unsigned rem = 0;
        for (int i = NB - 1; i >= 0; i--) {
            unsigned cur = rem * 256u + t.b[i];
            t.b[i] = (uint8_t)(cur / 10u);
            rem = cur % 10u;
            if (t.b[i]) nonzero = 1;
        }
        rev[n++] = (char)('0' + rem);
        if (!nonzero) break;
    }
    if ((size_t)n + 1 > cap) { out[0] = 0; return; }
    for (int i = 0; i < n; i++) out[i] = rev[n - 1 - i];
    out[n] = 0;
}

/* ---- Section 3.1: password -> a = (a1, a2, a3) ---------------------------
 * pi_i (1-based in the paper) is pw[i-1]; L = floor(n_pi / 3).            */
static void pack_password(const uint8_t *pw, size_t n, big a[3]) {
    size_t L = n / 3;
#define PI(i) ((unsigned)pw[(i) - 1])
    for (int j = 0; j < 3; j++) big_zero(&a[j]);
    /* a1 */
    if (n % 3 == 0) {
        for (size_t i = 1; i <= L; i++) big_add_shifted(&a[0], PI(i), (int)(i - 1));
    } else {
        for (size_t i = 1; i <= L; i++) big_add_shifted(&a[0], PI(i), (int)i);
        big_add_shifted(&a[0], PI(3 * L + 1), 0);
    }
    /* a2 */
    if (n % 3 != 2) {
        for (size_t i = L + 1; i <= 2 * L; i++) big_add_shifted(&a[1], PI(i), (int)(i - L - 1));
    } else {
        for (size_t i = L + 1; i <= 2 * L; i++) big_add_shifted(&a[1], PI(i), (int)(i - L));
        big_add_shifted(&a[1], PI(3 * L + 2), 0);
    }
    /* a3 */
    for (size_t i = 2 * L + 1; i <= 3 * L; i++) big_add_shifted(&a[2], PI(i), (int)(i - 2 * L - 1));
#undef PI
}

/* ---- public: key setup (Section 3.1) ------------------------------------- */

int orc_key_setup(const uint8_t *pw, size_t n_pw, const orc_params *prm, orc_key *out,
                  char *a_decimal /* optional, 3 x 128 chars */) {
    if (!pw || !prm || !out || n_pw == 0 || n_pw > 64) return -1;
    big a[3];
    pack_password(pw, n_pw, a);
    int L = (int)(n_pw / 3);
    out->L = L;

    /* D = ceil(log10 2^(8(L+1))) = number of decimal digits of 2^(8(L+1)) */
    big p2;
    big_zero(&p2);
    big_add_shifted(&p2, 1u, L + 1);
    char dec[256];
    big_to_decimal(&p2, dec, sizeof dec);
    int D = (int)strlen(dec);
    out->D = D;

    /* a'_j = a_j / 10^D, correctly rounded: decimal string -> strtod */
    for (int j = 0; j < 3; j++) {
        char num[256], lit[300];
        big_to_decimal(&a[j], num, sizeof num);
        if (a_decimal) snprintf(a_decimal + 128 * j, 128, "%.127s", num);
        snprintf(lit, sizeof lit, "%se-%d", num, D);
        out->a_prime[j] = strtod(lit, NULL);
        /* Eq. r0 = a' + lambda */
        out->r0[j] = out->a_prime[j] + prm->lambda[j];
    }

    /* mu_1 = (a1+a2+a3) mod 3, mu_2 = (a1 a2 + a3) mod 3, mu_3 = (a1 + a2 a3) mod 3 */
    big s, t;
    s = a[0]; big_add(&s, &a[1]); big_add(&s, &a[2]);
    out->mu[0] = (int32_t)big_mod_small(&s, 3);
    big_mul(&t, &a[0], &a[1]); big_add(&t, &a[2]);
    out->mu[1] = (int32_t)big_mod_small(&t, 3);
    big_mul(&t, &a[1], &a[2]); big_add(&t, &a[0]);
    out->mu[2] = (int32_t)big_mod_small(&t, 3);

    /* Omega_i = hash(i a) mod k_i, hash = SHA-256 over LE32(i a1)||LE32(i a2)||LE32(i a3) */
    for (int i = 1; i <= 3; i++) {
        uint8_t msg[96], dig[SHA256_DIGEST_LENGTH];
        for (int j = 0; j < 3; j++) {
            big ia;
            big_mul_small(&ia, &a[j], (unsigned)i);
            memcpy(msg + 32 * j, ia.b, 32);
        }
        SHA256(msg, sizeof msg, dig);
        big h; /* digest as a big-endian integer */
        big_zero(&h);
        for (int q = 0; q < 32; q++) h.b[q] = dig[31 - q];
        out->k[i - 1] = (int32_t)prm->k[i - 1];
        out->omega[i - 1] = (int32_t)big_mod_small(&h, prm->k[i - 1]);
    }
    return 0;
}

/* ---- Section 3.1: the dynamical system F ---------------------------------- */

/* One forward Euler step of dx/dt = sigma(y-x), dy/dt = x(rho-z)-y,
 * dz/dt = xy - beta z; every line is one rounding, old x,y,z throughout. */
static void lorenz_euler_step(double r[3], double dt) {
    double x = r[0], y = r[1], z = r[2];
    double dx = SIGMA * (y - x);
    double dy = (x * (RHO - z)) - y;
    double dz = (x * y) - (BETA * z);
    r[0] = x + dt * dx;
    r[1] = y + dt * dy;
    r[2] = z + dt * dz;
}

/* The same forward Euler step with each update fused into one rounding:
 * dy = fma(x, rho - z, -y), dz = fma(x, y, -(beta z)), x += dt dx as fma(dt, dx, x). */
static void lorenz_euler_fma_step(double r[3], double dt) {
    double x = r[0], y = r[1], z = r[2];
    double dx = SIGMA * (y - x);
    double dy = fma(x, RHO - z, -y);
    double dz = fma(x, y, -(BETA * z));
    r[0] = fma(dt, dx, x);
    r[1] = fma(dt, dy, y);
    r[2] = fma(dt, dz, z);
}

/* Lorenz vector field, same evaluation order as the Euler step. */
static void lorenz_field(const double r[3], double k[3]) {
    k[0] = SIGMA * (r[1] - r[0]);
    k[1] = (r[0] * (RHO - r[2])) - r[1];
    k[2] = (r[0] * r[1]) - (BETA * r[2]);
}

/* Classical Runge-Kutta 4: k1 = f(r), k2 = f(r + dt/2 k1), k3 = f(r + dt/2 k2),
 * k4 = f(r + dt k3), r += dt/6 ((k1 + k4) + 2 (k2 + k3)). */
static void lorenz_rk4_step(double r[3], double dt) {
    const double h2 = dt * 0.5, h6 = dt / 6.0;
    double k1[3], k2[3], k3[3], k4[3], t[3];
    lorenz_field(r, k1);
    for (int j = 0; j < 3; j++) t[j] = r[j] + h2 * k1[j];
    lorenz_field(t, k2);
    for (int j = 0; j < 3; j++) t[j] = r[j] + h2 * k2[j];
    lorenz_field(t, k3);
    for (int j = 0; j < 3; j++) t[j] = r[j] + dt * k3[j];
    lorenz_field(t, k4);
    for (int j = 0; j < 3; j++) r[j] = r[j] + h6 * ((k1[j] + k4[j]) + 2.0 * (k2[j] + k3[j]));
}

void orc_lorenz_integrator(double r[3], double dt, uint64_t steps, uint32_t integrator) {
    for (uint64_t t = 0; t < steps; t++) {
        if (integrator == 1) lorenz_euler_fma_step(r, dt);
        else if (integrator == 2) lorenz_rk4_step(r, dt);
        else lorenz_euler_step(r, dt);
    }
}

void orc_lorenz(double r[3], double dt, uint64_t steps) { orc_lorenz_integrator(r, dt, steps, 0); }

/* ---- Eq. R_nu: byte Omega of floor(alpha 10^nu) ---------------------------
 * Returns -1 for alpha outside the domain (never reached from orc_block,
 * which stops first). */

int orc_R(double alpha, int omega) {
    if (!in_domain(alpha)) return -1;
    int64_t N = (int64_t)floor(alpha * SCALE_NU);
    return (int)(((uint64_t)N >> (8 * omega)) & 0xFFu);
}

/* Step 2: Theta = P_i / 10^(3 + Omega_3) */
double orc_theta(int p, int omega3) {
    static const double pow10[7] = {1.0, 10.0, 100.0, 1000.0, 10000.0, 100000.0, 1000000.0};
    return (double)p / pow10[3 + omega3];
}

/* ---- the same functions over arrays, for checking other implementations ----
 * Plain loops over orc_R, orc_theta and orc_lorenz_integrator (the Lorenz
 * states split over nthreads threads); no arithmetic of their own.          */

/* Returns 0, or -1 (out[i] = 0) when some alpha is outside the domain. */
int orc_R_many(const double *alpha, const uint8_t *omega, size_t n, uint8_t *out) {
    int rc = 0;
    for (size_t i = 0; i < n; i++) {
        int v = orc_R(alpha[i], omega[i]);
        if (v < 0) rc = -1;
        out[i] = (uint8_t)(v < 0 ? 0 : v);
    }
    return rc;
}

void orc_theta_many(const uint8_t *p, const uint8_t *omega3, size_t n, double *out) {
    for (size_t i = 0; i < n; i++) out[i] = orc_theta(p[i], omega3[i]);
}

typedef struct {
    double *r;      /* 3 doubles per state */
    size_t n;
    double dt;
    uint64_t steps;
    uint32_t integrator;
    int part, parts;
} lorenz_job_t;

static void *lorenz_worker(void *arg) {
    const lorenz_job_t *J = (const lorenz_job_t *)arg;
    for (size_t i = (size_t)J->part; i < J->n; i += (size_t)J->parts)
        orc_lorenz_integrator(J->r + 3 * i, J->dt, J->steps, J->integrator);
    return NULL;
}

void orc_lorenz_many(double *r, size_t n, double dt, uint64_t steps, uint32_t integrator, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    lorenz_job_t J[64];
    for (int t = 0; t < nthreads; t++) {
        lorenz_job_t j = {r, n, dt, steps, integrator, t, nthreads};
        J[t] = j;
    }
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, lorenz_worker, &J[t]);
    lorenz_worker(&J[0]);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
}

/* N(v) of the integrity digest (v in the domain) */
static uint64_t digest_word(double v) { return (uint64_t)(int64_t)floor(v * SCALE_NU); }

static int state_in_domain(const double r[3]) { return in_domain(r[0]) && in_domain(r[1]) && in_domain(r[2]); }

/* ---- Steps 1-3 of Section 3.2 over one block -------------------------------
 * Block b of the parallel version (Section 5) starts at r0 + b 2^-24.
 * decrypt = 0: in = P bytes, out = C bytes; decrypt = 1: in = C, out = P.
 * Returns 0, or ORC_E_ESCAPED when the trajectory leaves the domain.        */
int orc_block(const orc_key *K, const orc_params *prm, uint64_t b, const uint8_t *in,
              size_t len, uint8_t *out, int decrypt, uint64_t d[3]) {
    double r[3], alpha[3];
    int mu[3], Om[3];
    for (int j = 0; j < 3; j++) r[j] = K->r0[j] + (double)b * 0x1p-24;
    if (!state_in_domain(r)) return ORC_E_ESCAPED;
    for (int i = 0; i < 3; i++) { mu[i] = K->mu[i]; Om[i] = K->omega[i]; }
    for (int i = 0; i < 3; i++) alpha[i] = r[mu[i]]; /* Eq. alpha with n = 0 */

    for (size_t q = 0; q < len; q++) {
        /* Step 1: E or D with R(alpha_1, Omega_1) and R(alpha_2, Omega_2) */
        int R1 = orc_R(alpha[0], Om[0]);
        int R2 = orc_R(alpha[1], Om[1]);
        int p;
        if (!decrypt) {
            p = in[q];
            out[q] = (uint8_t)((p + R1 + R2) % 256);
        } else {
            int c = in[q];
            p = (((c - R1 - R2) % 256) + 256) % 256;
            out[q] = (uint8_t)p;
        }
        /* Step 2: chaotic operation mode: r[mu_3] += Theta, then F^(n_it) */
        double theta = orc_theta(p, Om[2]);
        r[mu[2]] = r[mu[2]] + theta;
        orc_lorenz_integrator(r, prm->dt, prm->n_it, prm->integrator);
        if (!state_in_domain(r)) return ORC_E_ESCAPED;
        /* Step 3 */
        int R3 = orc_R(alpha[2], Om[2]);
        int Rold[3] = {R1, R2, R3};
        for (int i = 0; i < 3; i++) mu[i] = (mu[i] + Rold[i]) % 3;
        for (int i = 0; i < 3; i++) alpha[i] = r[mu[i]];
        for (int i = 0; i < 3; i++) {
            int src = ((i + 1 + 2) % 3) + 1; /* paper's 1-based index [(i+2) mod 3]+1 */
            Om[i] = (Om[i] + orc_R(alpha[src - 1], Om[i])) % K->k[i];
        }
        for (int j = 0; j < 3; j++) r[j] = r[j] + K->a_prime[j];
    }
    if (!state_in_domain(r)) return ORC_E_ESCAPED;
    for (int j = 0; j < 3; j++) d[j] = digest_word(r[j]);
    return 0;
}

/* ---- whole messages, blocks spread over threads ---------------------------- */

typedef struct {
    const orc_key *K;
    const orc_params *prm;
    const uint8_t *in;  /* bytes of blocks b0, b0 + 1, ... */
    uint8_t *out;
    size_t n;
    uint64_t nb;
    uint64_t b0;        /* index in the message of the first block */
    int decrypt;
    uint64_t *digests; /* 3 per block */
    uint64_t next;     /* shared block counter */
    int rc;            /* first error of a block (under lock) */
    pthread_mutex_t lock;
} job_t;

static void *worker(void *arg) {
    job_t *J = (job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        uint64_t b = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (b >= J->nb) break;
        size_t off = (size_t)b * J->prm->block_len;
        size_t len = J->n - off < J->prm->block_len ? J->n - off : J->prm->block_len;
        int rc = orc_block(J->K, J->prm, J->b0 + b, J->in + off, len, J->out + off, J->decrypt,
                           J->digests + 3 * b);
        if (rc) {
            pthread_mutex_lock(&J->lock);
            if (!J->rc) J->rc = rc;
            pthread_mutex_unlock(&J->lock);
        }
    }
    return NULL;
}

/* Blocks b0, b0 + 1, ... covering the n bytes at in (n = 0: the one empty block b0); tag = XOR of
 * their digests. */
static int run_blocks(const orc_key *K, const orc_params *prm, uint64_t b0, const uint8_t *in, size_t n,
                      uint8_t *out, int decrypt, int nthreads, uint64_t tag[3]) {
    uint64_t nb = n == 0 ? 1 : (n + prm->block_len - 1) / prm->block_len;
    job_t J = {K, prm, in, out, n, nb, b0, decrypt, NULL, 0, 0, PTHREAD_MUTEX_INITIALIZER};
    J.digests = (uint64_t *)calloc(3 * nb, sizeof(uint64_t));
    if (!J.digests) return -3;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nb) nthreads = (int)nb;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, worker, &J);
    worker(&J);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    if (J.rc) {
        free(J.digests);
        return J.rc;
    }
    tag[0] = tag[1] = tag[2] = 0;
    for (uint64_t b = 0; b < nb; b++)
        for (int j = 0; j < 3; j++) tag[j] ^= J.digests[3 * b + j];
    free(J.digests);
    return 0;
}

static int check_params(const orc_params *prm) {
    if (!prm || !(prm->dt > 0.0) || prm->n_it == 0 || prm->block_len == 0 || prm->integrator > 2) return -1;
    for (int i = 0; i < 3; i++)
        if (prm->k[i] < 3 || prm->k[i] > 4) return -1;
    return 0;
}

/* C = E(P) || LE64(T1) || LE64(T2) || LE64(T3); C has n + 24 bytes.
 * Returns 0, -1 (bad argument) or ORC_E_ESCAPED (C then undefined).        */
int orc_encrypt(const uint8_t *pw, size_t n_pw, const orc_params *prm, const uint8_t *P,
                size_t n, uint8_t *C, int nthreads) {
    if (check_params(prm) || (!P && n) || !C) return -1;
    orc_key K;
    if (orc_key_setup(pw, n_pw, prm, &K, NULL)) return -1;
    uint64_t tag[3];
    int rc = run_blocks(&K, prm, 0, P, n, C, 0, nthreads, tag);
    if (rc) return rc;
    for (int j = 0; j < 3; j++)
        for (int q = 0; q < 8; q++) C[n + 8 * j + q] = (uint8_t)(tag[j] >> (8 * q));
    return 0;
}

/* Returns 0 and P (n_c - 24 bytes), -2 with P zeroed when the tag fails,
 * -1 for a bad argument, or ORC_E_ESCAPED (P then zeroed).                   */
int orc_decrypt(const uint8_t *pw, size_t n_pw, const orc_params *prm, const uint8_t *C,
                size_t n_c, uint8_t *P, int nthreads) {
    if (check_params(prm) || !C || n_c < 24 || (!P && n_c > 24)) return -1;
    orc_key K;
    if (orc_key_setup(pw, n_pw, prm, &K, NULL)) return -1;
    size_t n = n_c - 24;
    uint64_t tag[3];
    int rc = run_blocks(&K, prm, 0, C, n, P, 1, nthreads, tag);
    if (rc) {
        if (n) memset(P, 0, n);
        return rc;
    }
    int ok = 1;
    for (int j = 0; j < 3; j++) {
        uint64_t stored = 0;
        for (int q = 0; q < 8; q++) stored |= (uint64_t)C[n + 8 * j + q] << (8 * q);
        if (stored != tag[j]) ok = 0;
    }
    if (!ok) {
        if (n) memset(P, 0, n);
        return -2;
    }
    return 0;
}

/* One block of a message, for sampled checks of large messages. */
int orc_crypt_block(const uint8_t *pw, size_t n_pw, const orc_params *prm, uint64_t b,
                    const uint8_t *in, size_t len, uint8_t *out, int decrypt, uint64_t d[3]) {
    if (check_params(prm) || len > prm->block_len) return -1;
    orc_key K;
    if (orc_key_setup(pw, n_pw, prm, &K, NULL)) return -1;
    return orc_block(&K, prm, b, in, len, out, decrypt, d);
}

/* Blocks b0, b0 + 1, ... of a message, covering the len bytes at in (which start at byte b0 block_len
 * of the message), spread over threads: out receives their output bytes and part the XOR of their
 * digests, so that the parts of a message's block ranges XOR to its tag.  For checks of large
 * messages slice by slice. */
int orc_crypt_range(const uint8_t *pw, size_t n_pw, const orc_params *prm, uint64_t b0, const uint8_t *in,
                    size_t len, uint8_t *out, int decrypt, int nthreads, uint64_t part[3]) {
    if (check_params(prm) || (!in && len) || (!out && len) || !part) return -1;
    orc_key K;
    if (orc_key_setup(pw, n_pw, prm, &K, NULL)) return -1;
    return run_blocks(&K, prm, b0, in, len, out, decrypt, nthreads, part);
}
