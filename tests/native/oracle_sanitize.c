/*
 * Test driver: runs the CPU oracle, compiled into this program with host
 * sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer, or
 * ThreadSanitizer), over cases read from stdin, and prints its results so the
 * test can compare them with the oracle's ordinary build.
 *
 * Input lines (hex strings; "-" for an empty one):
 *   E pw n_it block_len integrator nthreads k1 k2 k3 plaintext
 *       -> ciphertext, then "rt=<0|1>" (decryption returns the plaintext) and
 *          "tamper=<rc>" (decryption of the ciphertext with one byte flipped)
 *   L n steps integrator nthreads start
 *       -> the n states after `steps` steps, as hex of their binary64 bytes
 *          (start holds n x 3 binary64 values)
 *   U alpha_count p_count alphas omegas ps omega3s
 *       -> R(alpha, omega) bytes, then the binary64 bytes of theta(p, omega3)
 */
#include "../../oracle/lz_oracle.c"

#include <stdio.h>

static size_t unhex(const char *s, uint8_t **out) {
    if (!strcmp(s, "-")) {
        *out = malloc(1);
        return 0;
    }
    size_t n = strlen(s) / 2;
    *out = malloc(n ? n : 1);
    for (size_t i = 0; i < n; i++) {
        unsigned v;
        sscanf(s + 2 * i, "%2x", &v);
        (*out)[i] = (uint8_t)v;
    }
    return n;
}

static void put_hex(const void *p, size_t n) {
    const uint8_t *b = p;
    if (!n) fputs("-", stdout);
    for (size_t i = 0; i < n; i++) printf("%02x", b[i]);
}

static void run_encrypt(char **f) {
    uint8_t *pw, *P;
    size_t n_pw = unhex(f[1], &pw);
    orc_params prm = {0.01, {1.0, 1.0, 1.0}, (uint32_t)atoi(f[2]), (uint32_t)atoi(f[3]),
                      {(uint32_t)atoi(f[6]), (uint32_t)atoi(f[7]), (uint32_t)atoi(f[8])}, (uint32_t)atoi(f[4])};
    int nthreads = atoi(f[5]);
    size_t n = unhex(f[9], &P);
    uint8_t *C = malloc(n + 24), *Q = malloc(n ? n : 1);
    int rc = orc_encrypt(pw, n_pw, &prm, P, n, C, nthreads);
    if (rc) {
        printf("rc=%d\n", rc);
    } else {
        put_hex(C, n + 24);
        int rt = orc_decrypt(pw, n_pw, &prm, C, n + 24, Q, nthreads) == 0 && (!n || !memcmp(P, Q, n));
        C[(n + 24) / 2] ^= 0x01;
        int tamper = orc_decrypt(pw, n_pw, &prm, C, n + 24, Q, nthreads);
        printf(" rt=%d tamper=%d\n", rt, tamper);
    }
    free(pw);
    free(P);
    free(C);
    free(Q);
}

static void run_lorenz(char **f) {
    size_t n = (size_t)atoll(f[1]);
    uint8_t *r;
    size_t nb = unhex(f[5], &r);
    if (nb != n * 3 * sizeof(double)) {
        puts("bad-input");
    } else {
        orc_lorenz_many((double *)r, n, 0.01, (uint64_t)atoll(f[2]), (uint32_t)atoi(f[3]), atoi(f[4]));
        put_hex(r, nb);
        putchar('\n');
    }
    free(r);
}

static void run_units(char **f) {
    size_t na = (size_t)atoll(f[1]), np = (size_t)atoll(f[2]);
    uint8_t *alpha, *omega, *p, *omega3;
    unhex(f[3], &alpha);
    unhex(f[4], &omega);
    unhex(f[5], &p);
    unhex(f[6], &omega3);
    uint8_t *R = malloc(na ? na : 1);
    double *th = malloc(np ? np * sizeof(double) : 1);
    orc_R_many((const double *)alpha, omega, na, R);
    orc_theta_many(p, omega3, np, th);
    put_hex(R, na);
    putchar(' ');
    put_hex(th, np * sizeof(double));
    putchar('\n');
    free(alpha);
    free(omega);
    free(p);
    free(omega3);
    free(R);
    free(th);
}

int main(void) {
    size_t cap = 1 << 20;
    char *line = malloc(cap);
    while (fgets(line, (int)cap, stdin)) {
        char *f[12] = {0};
        int nf = 0;
        for (char *t = strtok(line, " \n"); t && nf < 12; t = strtok(NULL, " \n")) f[nf++] = t;
        if (nf == 10 && !strcmp(f[0], "E"))
            run_encrypt(f);
        else if (nf == 6 && !strcmp(f[0], "L"))
            run_lorenz(f);
        else if (nf == 7 && !strcmp(f[0], "U"))
            run_units(f);
        else
            puts("bad-line");
        fflush(stdout);
    }
    free(line);
    return 0;
}
