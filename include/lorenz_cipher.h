/*
 * lorenz_cipher.h -- C ABI of the MI355X (gfx950) implementation of the
 * Lorenz-attractor chaotic cipher of Marco, Martinez and Bruno,
 * "Fast, parallel and secure cryptography algorithm using Lorenz's attractor"
 * (arXiv:1201.3114), parallel (fast) version of Section 5.
 *
 * Problem statement (Section 1): C = E_pi(P), P = D_pi(C) = E_pi^-1(C), with
 * P and C strings of bytes and pi the password's bytes.  The integrity claim
 * (Abstract, end of Section 2) is realised as a 24-byte tag appended to C:
 * decryption fails when any byte of C was altered.
 *
 * Conventions for every entry point:
 *  - Return value: LZ_OK (0) or a negative LZ_E_* code.  No exception or
 *    abort crosses the ABI; lz_last_error() gives a thread-local message.
 *  - "Device pointer": memory of the context's GPU (hipMalloc, or a torch
 *    tensor's data_ptr()).  "Host pointer": ordinary process memory.
 *  - The caller owns every buffer it passes and keeps it alive until the
 *    work enqueued on `stream` has completed.  The library owns only what it
 *    allocates inside a context, batch or server object.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Plain and batch
 *    calls are asynchronous on it unless stated otherwise.
 *  - Byte layouts: a ciphertext is body (n bytes) || T1 || T2 || T3, each tag
 *    word a little-endian uint64, so n_c = n + LZ_TAG_BYTES.
 *
 * Method parameters and their readings of the paper:
 *  - Euler step of the Lorenz system (Section 3.1, F) with sigma = 10,
 *    rho = 28, beta = 8/3, step dt, applied n_it times per byte (Step 2);
 *  - the parallel version (Section 5) cuts a message into blocks of
 *    block_len bytes; block b starts at r0 + b 2^-24 (every coordinate);
 *  - r0 = a' + lambda (Section 3.1), Omega_i = SHA-256(i a) mod k_i.
 */
#ifndef LORENZ_CIPHER_H
#define LORENZ_CIPHER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LZ_TAG_BYTES 24
#define LZ_MAX_PASSWORD 64
#define LZ_MAX_MESSAGE (1ull << 32)
/* staging capacity of a stream's deferred updates (input and output each), and chunks per flush */
#define LZ_STREAM_DEFER_BYTES (64ull << 20)
#define LZ_STREAM_DEFER_CHUNKS 4096
/* Block b of a message starts at r0 + b 2^-24 (every coordinate), so a
 * message may have at most 2^24 blocks: every start then lies within 1 of
 * r0.  With the default block_len of 256 every message up to 2^32 bytes
 * fits; a smaller block_len lowers the longest message accordingly. */
#define LZ_MAX_BLOCKS (1ull << 24)
/* Largest accepted Euler step.  The paper allows 0 < dt <= 0.027
 * (Section 3.1), but forward Euler of the Lorenz system leaves the attractor
 * and overflows from some starts inside the lambda ranges once dt reaches
 * about 0.02, and from points of the attractor moved by the per-byte
 * perturbations at 0.024; at 0.015 and below no such escape was found. */
#define LZ_MAX_DT 0.015

enum {
    LZ_OK = 0,
    LZ_E_INVAL = -1,     /* bad argument: NULL pointer, size or parameter out of range   */
    LZ_E_INTEGRITY = -2, /* decryption: the recomputed tag differs from the stored one    */
    LZ_E_NOMEM = -3,     /* device or host allocation failed, or request exceeds a budget */
    LZ_E_HIP = -4,       /* a HIP runtime call failed (message in lz_last_error)          */
    LZ_E_AGAIN = -5,     /* server: nothing to return yet                                 */
    LZ_E_CANCELLED = -6  /* server: the request was cancelled before it completed         */
};

/* Integrator of the dynamical system F (Section 3.1 uses forward Euler and
 * leaves the integrator open to other schemes).  Each value is a
 * distinct ciphertext format.
 *  LZ_INTEGRATOR_EULER      forward Euler, 14 separately rounded operations per
 *                           step (the method; the default);
 *  LZ_INTEGRATOR_EULER_FMA  the same step with each update fused into one
 *                           rounding: dy = fma(x, rho-z, -y), dz = fma(x, y,
 *                           -(beta z)), x += dt dx as fma(dt, dx, x); 9 roundings;
 *  LZ_INTEGRATOR_RK4        classical Runge-Kutta 4 with the same vector field,
 *                           r += dt/6 ((k1 + k4) + 2 (k2 + k3)). */
enum { LZ_INTEGRATOR_EULER = 0, LZ_INTEGRATOR_EULER_FMA = 1, LZ_INTEGRATOR_RK4 = 2 };

/* Parameters of the method (Section 3.1).
 * Defaults (lz_params_default): dt = 0.01, lambda = (1,1,1), n_it = 3000,
 * block_len = 256, k = (4,4,4), integrator = LZ_INTEGRATOR_EULER.  Valid
 * ranges (else LZ_E_INVAL): 0 < dt <= LZ_MAX_DT = 0.015 (see LZ_MAX_DT),
 * each lambda_j inside the paper's open range for its coordinate
 * (-15.67 < lambda_1 < 16.01, -11.28 < lambda_2 < 16.01, 0.090 < lambda_3 <
 * 62), n_it >= 1, block_len >= 1 (block_len >= n gives the sequential
 * version of Section 5: the whole message is one chain), k_i in {3, 4}
 * (2 < k_i <= floor((xi-14)/8) = 4), integrator one of the values above.
 * sigma = 10, rho = 28 and beta = 8/3 are fixed by Section 3.1 and are not
 * parameters.  Every entry point that takes a message also rejects one of
 * more than LZ_MAX_BLOCKS blocks (LZ_E_INVAL), see lz_block_count. */
typedef struct {
    double dt;
    double lambda[3];
    uint32_t n_it;
    uint32_t block_len;
    uint8_t k[3];
    uint8_t integrator;
    uint8_t reserved[4]; /* must be zero */
} lz_params;

/* Output of the password stage of Section 3.1 (64 bytes, plain data). */
typedef struct {
    double a_prime[3]; /* a' = a / 10^D, correctly rounded, D = digits of 2^(8(L+1)) */
    double r0[3];      /* r0 = a' + lambda                                          */
    uint8_t mu[3];     /* mu_1 = (a1+a2+a3) mod 3, mu_2 = (a1 a2 + a3) mod 3, ...   */
    uint8_t omega[3];  /* Omega_i = SHA-256(LE32(i a1)||LE32(i a2)||LE32(i a3)) mod k_i */
    uint8_t k[3];
    uint8_t reserved[7];
} lz_key;

/* Launch shape of the hot kernels.  chains_per_lane: blocks one lane
 * carries at once (1, 2 or 4, interleaved for instruction-level parallelism);
 * wg_size: 64, 128 or 256 threads; tile: bytes per chain staged through LDS
 * per refill (16, 32, 64 or 128); waves_per_simd: resident waves per SIMD of
 * the persistent batched kernel (1..8).  All-zero = use the tuned default. */
typedef struct {
    uint32_t chains_per_lane;
    uint32_t wg_size;
    uint32_t tile;
    uint32_t waves_per_simd;
} lz_launch;

typedef struct lz_ctx lz_ctx;
typedef struct lz_batch lz_batch;
typedef struct lz_server lz_server;
typedef struct lz_stream lz_stream;

/* ---- host-only helpers ---------------------------------------------------- */

/* Fills *out with the defaults above.  LZ_E_INVAL if out is NULL. */
int lz_params_default(lz_params *out);

/* LZ_OK if *prm is within the valid ranges, else LZ_E_INVAL. */
int lz_params_check(const lz_params *prm);

/* n + LZ_TAG_BYTES. */
size_t lz_ciphertext_len(size_t n_plain);

/* Number of blocks (independent chains, Section 5) of an n-byte message
 * under *prm: ceil(n / block_len), 1 for n = 0.  LZ_E_INVAL if prm is
 * invalid, n > 2^32 or the count exceeds LZ_MAX_BLOCKS; the entry points
 * that take a message apply the same rule.  Host only. */
int lz_block_count(const lz_params *prm, uint64_t n, uint64_t *nb);

/* Password stage of Section 3.1 on the host: packing of pi into a = (a1,a2,a3),
 * a' = g(a), r0 = a' + lambda, mu, Omega.  pw: host pointer, 1..64 bytes (any
 * byte values).  Pure function, thread-safe.  LZ_E_INVAL on NULL or length. */
int lz_key_setup(const uint8_t *pw, size_t n_pw, const lz_params *prm, lz_key *out);

/* Thread-local description of the last error of this thread ("" if none). */
const char *lz_last_error(void);

/* ---- context ---------------------------------------------------------------- */

/* Creates a context on HIP device `device` with parameters *prm (NULL =
 * defaults).  The context owns a small device workspace (tag accumulators,
 * statuses) and the tuned launch shape.  Calls that share a context are
 * ordered: a call on a different stream than the previous call first waits
 * for the previous call's work.  A context may be used by one host thread at
 * a time (servers and streams created from it run their own work and may be
 * used concurrently with it).  LZ_E_HIP if the device is unavailable. */
int lz_context_create(int device, const lz_params *prm, lz_ctx **out);
int lz_context_destroy(lz_ctx *ctx);

/* Reads back the context's parameters. */
int lz_context_params(const lz_ctx *ctx, lz_params *out);

/* Sets (shape non-NULL) the launch shape used by the plain path and by
 * batches created later, after validating it; LZ_E_INVAL if out of range.
 * The plain path takes chains_per_lane > 1 only for a message of at least
 * 2 x chains_per_lane waves' worth of blocks per SIMD (more chains per lane
 * lengthen each chain's latency); smaller messages run one chain per lane. */
int lz_context_set_launch(lz_ctx *ctx, const lz_launch *shape);
int lz_context_get_launch(const lz_ctx *ctx, lz_launch *out);

/* ---- plain path (one message) ---------------------------------------------------
 * Section 3.2 Steps 1-3 over every block of the message in parallel
 * (Section 5), one GPU lane per block, with the tag of the integrity claim.
 *
 * lz_encrypt: d_P device pointer, n bytes (0 <= n <= 2^32; NULL allowed when
 * n == 0); d_C device pointer of n + 24 bytes (body then tag).  pw host
 * pointer, 1..64 bytes.  Asynchronous on stream. */
int lz_encrypt(lz_ctx *ctx, const uint8_t *pw, size_t n_pw, const uint8_t *d_P, size_t n,
               uint8_t *d_C, void *stream);

/* lz_decrypt: d_C device pointer of n_c >= 24 bytes; d_P device pointer of
 * n_c - 24 bytes.  If the recomputed tag differs from the stored one the
 * plaintext is zeroed (unauthenticated bytes are never released) and the
 * status is LZ_E_INTEGRITY.  d_status: device int32 receiving LZ_OK or
 * LZ_E_INTEGRITY (asynchronous call); if d_status is NULL the call
 * synchronises the stream and returns that status itself. */
int lz_decrypt(lz_ctx *ctx, const uint8_t *pw, size_t n_pw, const uint8_t *d_C, size_t n_c,
               uint8_t *d_P, int32_t *d_status, void *stream);

/* Plain path with a precomputed key (lz_key_setup) instead of a password. */
int lz_encrypt_key(lz_ctx *ctx, const lz_key *key, const uint8_t *d_P, size_t n, uint8_t *d_C,
                   void *stream);
int lz_decrypt_key(lz_ctx *ctx, const lz_key *key, const uint8_t *d_C, size_t n_c, uint8_t *d_P,
                   int32_t *d_status, void *stream);

/* ---- decrypt without allocation -------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * lz_decrypt_noalloc is lz_decrypt (same kernels, same output, same status)
 * without a context: parameters *prm (NULL = defaults), the current HIP
 * device, the plain path's default launch shape.  It calls no hipMalloc,
 * hipFree or allocating routine.  Its one scratch buffer, the tag
 * accumulator, is a static device array of LZ_NOALLOC_SCRATCH_BYTES held by
 * each GPU until the process ends (its address is resolved once per device,
 * on the first call there); each call clears what it uses first.  Messages
 * up to the plain path's limits (2^32 bytes, LZ_MAX_BLOCKS blocks) fit it;
 * larger ones are rejected with LZ_E_INVAL before anything runs.
 *
 * d_C device pointer of n_c >= 24 bytes; d_P device pointer of n_c - 24
 * bytes; d_status device int32, required (LZ_OK or LZ_E_INTEGRITY; on
 * LZ_E_INTEGRITY the plaintext is zeroed).  stream must belong to the
 * current device.  Asynchronous on stream.
 *
 * Every call on one GPU shares that GPU's scratch: calls on one stream are
 * ordered and safe; calls that overlap on one GPU (other streams, no
 * ordering between them) race and give wrong statuses.  LZ_E_INVAL for a
 * NULL argument, bad parameters or password length, n_c < 24, a message
 * beyond the limits, or a device index >= LZ_NOALLOC_MAX_DEVICES. */
#define LZ_NOALLOC_SCRATCH_BYTES 256
#define LZ_NOALLOC_MAX_DEVICES 64
int lz_decrypt_noalloc(const lz_params *prm, const uint8_t *pw, size_t n_pw, const uint8_t *d_C, size_t n_c,
                       uint8_t *d_P, int32_t *d_status, void *stream);

/* ---- batched path: many messages, one persistent launch in a HIP graph ---------
 * n_msg messages, message i with its own password and plaintext length
 * lens[i] (host arrays).  Encrypt: input i is lens[i] bytes at d_in +
 * in_off[i], output i is lens[i] + 24 bytes at d_out + out_off[i].  Decrypt:
 * input lens[i] + 24 bytes, output lens[i] bytes; d_status[i] (device int32,
 * n_msg entries) receives LZ_OK or LZ_E_INTEGRITY and failed outputs are
 * zeroed.  Passwords: bytes pw[pw_off[i] .. pw_off[i] + pw_len[i]) (host).
 * Output ranges must not overlap each other or the inputs.
 *
 * lz_batch_create does key setup for every message, builds and uploads the
 * work list (full blocks first, then partial blocks longest first), and
 * captures [reset, persistent kernel, finalize] into a HIP graph bound to
 * d_in/d_out; shape NULL = the context's launch shape.  It does not run the
 * batch.  d_status may be NULL (a decrypt batch then takes its statuses from
 * each lz_decrypt_batch call).  The batch owns its device descriptors.
 * LZ_E_INVAL for a NULL argument, n_msg outside [1, 2^30], a message over
 * 2^32 bytes or LZ_MAX_BLOCKS blocks, a bad password length or shape. */
int lz_batch_create(lz_ctx *ctx, int decrypt, size_t n_msg, const uint64_t *lens,
                    const uint64_t *in_off, const uint64_t *out_off, const uint8_t *pw,
                    const uint64_t *pw_off, const uint32_t *pw_len, const uint8_t *d_in,
                    uint8_t *d_out, int32_t *d_status, const lz_launch *shape, lz_batch **out);

/* C_i = E_pi_i(P_i) for every message of the batch at once (Section 1's
 * problem statement over many messages, each split into the parallel
 * version's blocks of Section 5): one replay of the batch's graph on stream,
 * asynchronous, repeatable.  batch must come from lz_batch_create on ctx
 * with decrypt = 0 (else LZ_E_INVAL). */
int lz_encrypt_batch(lz_ctx *ctx, const lz_batch *batch, void *stream);

/* P_i = D_pi_i(C_i) for every message of the batch: one replay on stream,
 * asynchronous.  d_status (device int32, n_msg entries, NOT NULL) receives
 * LZ_OK or LZ_E_INTEGRITY per message; a failed message's output is zeroed.
 * batch must come from lz_batch_create on ctx with decrypt = 1. */
int lz_decrypt_batch(lz_ctx *ctx, const lz_batch *batch, int32_t *d_status, void *stream);

/* Replays the graph with the d_status given at creation (LZ_E_INVAL for a
 * decrypt batch created without one). */
int lz_batch_launch(lz_batch *batch, void *stream);
int lz_batch_destroy(lz_batch *batch);

/* Autotuner: chooses the launch shape of the batched (and plain) kernels on
 * a synthetic batch of about 1.5 resident rounds of the device, with the
 * context's parameters.  Stage 1 times every shape of the grid
 * chains_per_lane {1,2,4} x waves_per_simd {1,2,4,8} (4 to 8 chains in flight
 * per SIMD slot) x wg_size {64,128,256} x tile {16,32,64,128} that fits the
 * device's LDS, at a tenth of n_it (the same per-byte loop in a tenth of the
 * time); stage 2 times the three fastest at the context's n_it.  The winner
 * goes to the context and to *best (may be NULL).  Synchronous; a few
 * seconds at n_it = 3000.  When budget_ms > 0 stage 1 stops after that much
 * measured time (the context's shape is timed first). */
int lz_autotune(lz_ctx *ctx, double budget_ms, lz_launch *best);

/* lz_autotune with a per-device cache: a text file of lines
 * "<gfx arch> cus=<CUs> integrator=<i> n_it=<n> block_len=<b>\t<chains_per_lane>
 * <wg_size> <tile> <waves_per_simd>\t<ms>".  path NULL = $LZ_TUNE_CACHE, else
 * $HOME/.cache/lorenz_cipher/launch_shapes.tsv (no file without HOME).  A
 * valid entry for this device and these parameters is used as is
 * (*from_cache = 1); otherwise the shape is tuned and the entry written
 * (*from_cache = 0; the file is rewritten through a temporary file and a
 * rename, and a failure to write it is not an error).  from_cache may be
 * NULL. */
int lz_autotune_cached(lz_ctx *ctx, const char *path, double budget_ms, lz_launch *best, int *from_cache);

/* ---- streaming: one message of unknown length, chunk by chunk -----------------
 * Encrypts (decrypt = 0) or decrypts one message given as a sequence of
 * chunks.  The concatenated outputs equal the one-shot body (lz_encrypt /
 * lz_decrypt) and the final tag equals its tag: the parallel version's
 * blocks (Section 5) are cut at block boundaries, a partial block's chain
 * state (r, alpha, mu, Omega of Section 3.2) waits on the device for the next
 * chunk.  Decrypted chunks are NOT authenticated until lz_stream_finish
 * reports LZ_OK; the caller must not release them before that.
 *
 * lz_stream_open: pw host pointer, 1..64 bytes; the stream owns about 200
 * bytes of device memory (two chain checkpoints and the running tag) and one
 * event, and from its first deferred update a staging buffer.  Synchronous. */
int lz_stream_open(lz_ctx *ctx, int decrypt, const uint8_t *pw, size_t n_pw, lz_stream **out);

/* Processes the next n bytes: d_in and d_out device pointers of n bytes
 * (plaintext in / ciphertext body out, or the reverse; no tag).  Asynchronous
 * on stream, as one kernel launch (the update's whole blocks and the chains
 * of its partial blocks); calls are ordered among themselves even across
 * streams.  LZ_E_INVAL after lz_stream_finish or past 2^32 bytes in total. */
int lz_stream_update(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out, void *stream);

/* Deferred update: the next n bytes as lz_stream_update computes them, but
 * the chunk is copied (on stream, device to device) into the stream's staging
 * buffer and runs later, together with the chunks queued after it, as one
 * update over their concatenation: at lz_stream_flush, when the queued bytes'
 * blocks reach one chain per lane of a wave on every SIMD of the device (CUs x 4
 * x 64 blocks, 16 MiB on a 256-CU device with 256-byte blocks, where an update
 * already runs at the full rate; at most LZ_STREAM_DEFER_BYTES; a chunk that
 * would pass that point is split between two runs), when LZ_STREAM_DEFER_CHUNKS
 * chunks are queued, before an immediate update, and at lz_stream_finish.  Small
 * chunks then share one launch that fills the device, and the host queues the
 * next ones while it runs.  d_in may be reused as soon
 * as stream reaches the call; d_out is written only by that later launch, on
 * the stream it is made on, and must stay valid until then.  A chunk of that
 * run size or more runs at once, after any queued chunks.  The first deferred update allocates the staging buffer
 * (2 x LZ_STREAM_DEFER_BYTES of device memory, freed by lz_stream_close;
 * LZ_E_NOMEM or LZ_E_HIP if that fails, with nothing queued).  Ordered with the
 * stream's other calls, also across streams.  Errors as lz_stream_update. */
int lz_stream_update_deferred(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out, void *stream);

/* Runs the queued deferred chunks now, on stream (nothing to do: LZ_OK).  Their
 * outputs are complete when stream reaches the end of this call's work.
 * LZ_E_INVAL after lz_stream_finish. */
int lz_stream_flush(lz_stream *st, void *stream);

/* Ends the message (running any queued deferred chunks first).  Encrypt: writes the 24-byte tag to d_tag (device).
 * Decrypt: d_tag holds the received tag (device); the result goes to
 * d_status (device int32: LZ_OK or LZ_E_INTEGRITY), or, with d_status NULL,
 * the call synchronises and returns it. */
int lz_stream_finish(lz_stream *st, uint8_t *d_tag, int32_t *d_status, void *stream);

/* Bytes consumed so far (queued deferred chunks included). */
uint64_t lz_stream_position(const lz_stream *st);

/* Waits for the stream's work and frees it (deferred chunks still queued are
 * dropped: their outputs are never written). */
int lz_stream_close(lz_stream *st);

/* ---- serving: continuous batching ------------------------------------------------
 * A request loop on a library thread.  Requests are admitted in arrival order
 * while chain slots and the device-memory budget allow; their per-block chain
 * state (r, alpha, mu, Omega: an exact checkpoint) and byte buffers stay on
 * the device.  Each tick advances chains by up to tick_bytes bytes, so
 * requests that arrive while others run join at the next tick.
 *
 * Policy LZ_SERVE_ADAPTIVE (the default): a tick runs k waves per SIMD at
 * most, chosen from the backlog (unfinished chains of admitted and waiting
 * requests): 1 while the backlog is at most 3 waves per SIMD, 2 up to 6,
 * then doubling up to run_waves.  Admitted requests join a tick in admission
 * order, each with all of its unfinished chains or none, and later requests
 * that fit fill the room an earlier one leaves (the first request with work
 * always joins, so one larger than the cap still runs).  Policy
 * LZ_SERVE_ALL_CHAINS: every tick runs every admitted chain.  Results are
 * bit-identical to the plain path whatever the policy. */
enum { LZ_SERVE_ADAPTIVE = 0, LZ_SERVE_ALL_CHAINS = 1 };
typedef struct {
    uint64_t hbm_budget;  /* bytes of device memory for request buffers + chain state */
    uint32_t max_chains;  /* chain slots resident on the device (0 = 2 x run_waves waves
                             per SIMD; LZ_SERVE_ALL_CHAINS: run_waves waves per SIMD) */
    uint32_t tick_bytes;  /* bytes per chain per tick (0 = 16)                        */
    uint32_t run_waves;   /* most waves per SIMD one tick runs, 1..8 (0 = 4)          */
    uint32_t policy;      /* LZ_SERVE_ADAPTIVE or LZ_SERVE_ALL_CHAINS                   */
} lz_server_config;

typedef struct {
    uint64_t id;         /* caller's request id                                   */
    int32_t status;      /* LZ_OK, LZ_E_INTEGRITY (decrypt), LZ_E_NOMEM (too big) or
                            LZ_E_CANCELLED                                            */
    int32_t reserved;
    uint64_t arrival_ns; /* monotonic clock, as submitted                         */
    uint64_t admit_ns;   /* when the request got slots and memory                 */
    uint64_t done_ns;    /* when its output was complete in the caller's buffer   */
} lz_completion;

/* Creates the server and starts its thread.  The budget covers everything the
 * server allocates on the device: chain slots (80 bytes each), request records,
 * the two tick slots' staging and a first-fit arena for request buffers (the
 * rest).  LZ_E_INVAL if the budget does not exceed the fixed part,
 * tick_bytes > 2^20, run_waves > 8 or an unknown policy.  Request buffers in device memory are moved by a batched
 * copy kernel, host buffers (pageable or pinned) by hipMemcpyAsync. */
int lz_server_create(lz_ctx *ctx, const lz_server_config *cfg, lz_server **out);

/* Queues a request.  decrypt = 0: src holds n bytes of plaintext, dst
 * receives n + 24; decrypt = 1: src holds n + 24 bytes of ciphertext, dst
 * receives n.  src/dst may be host or device pointers; the caller keeps them
 * valid until the completion is returned.  pw is copied.  arrival_ns is the
 * CLOCK_MONOTONIC time at which the request arrives (0 = now); the server does
 * not see it earlier, which lets a recorded trace be replayed.  Thread-safe. */
int lz_server_submit(lz_server *srv, uint64_t id, int decrypt, const uint8_t *pw, size_t n_pw,
                     const void *src, uint64_t n, void *dst, uint64_t arrival_ns);

/* Queues count requests at once (same meaning as lz_server_submit, element by
 * element): ids[i], decrypt[i] (0/1), password bytes pw[pw_off[i] ..
 * pw_off[i] + pw_len[i]), src[i], n[i], dst[i], arrival_ns[i] (all host
 * arrays).  Key setup runs on the calling thread before any request becomes
 * visible to the server.  On error nothing is queued. */
int lz_server_submit_many(lz_server *srv, size_t count, const uint64_t *ids, const uint8_t *decrypt,
                          const uint8_t *pw, const uint64_t *pw_off, const uint32_t *pw_len,
                          const void *const *src, const uint64_t *n, void *const *dst,
                          const uint64_t *arrival_ns);

/* Asks the server to drop request id (the first queued or running request
 * with that id).  Asynchronous, like submission: the request's completion
 * reports LZ_E_CANCELLED, and its dst is not written; a request still waiting
 * or not yet arrived completes at once, a running one once the tick running
 * its chains has finished (its chain slots and memory are then free for
 * others; the other requests' outputs do not change).  A request that
 * completes before the cancellation takes effect reports its own status; an
 * id that matches no request is ignored.  Thread-safe. */
int lz_server_cancel(lz_server *srv, uint64_t id);

/* Copies up to max completed requests into out, returns how many (>= 0), or
 * a negative error.  timeout_ms < 0 waits until at least one is available. */
int lz_server_poll(lz_server *srv, lz_completion *out, int max, int timeout_ms);

/* Counters: ticks run, chains advanced, peak device bytes in use. */
typedef struct {
    uint64_t ticks;
    uint64_t chain_bytes;
    uint64_t peak_hbm;
    uint64_t admitted;
    uint64_t completed;
    double busy_ms; /* summed device time of tick kernels */
} lz_server_stats;
int lz_server_stats_get(lz_server *srv, lz_server_stats *out);

/* Stops the thread after the queued requests complete, frees everything. */
int lz_server_destroy(lz_server *srv);

/* ---- diagnostics of Section 4 (frequency analysis, autocorrelation) -------------
 * lz_histogram: d_hist (device, 256 uint64, overwritten) receives the count of
 * each byte value of d_data (device, n bytes); the Shannon entropy
 * S = -sum p_i log2 p_i follows from it.  Uses the context's 1 MB merge
 * buffer (calls of one context are ordered across streams, as for the
 * workspace below).  Asynchronous on stream. */
int lz_histogram(lz_ctx *ctx, const uint8_t *d_data, size_t n, uint64_t *d_hist, void *stream);

/* lz_lag_sums: d_sums (device, max_lag + 1 uint64, overwritten) receives the
 * exact integer sums S_k = sum_{i < n-k} x_i x_{i+k}, k = 0..max_lag
 * (max_lag <= 16384), from which the autocorrelation of the byte sequence
 * follows: r_k = (S_k - m (A_k + B_k) + (n-k) m^2) / (S_0 - n m^2), m the mean,
 * A_k = sum_{i < n-k} x_i, B_k = sum_{i >= k} x_i.  Uses the context's merge
 * buffer (calls of one context are ordered across streams).  Asynchronous on
 * stream. */
int lz_lag_sums(lz_ctx *ctx, const uint8_t *d_data, size_t n, uint32_t max_lag, uint64_t *d_sums, void *stream);

/* lz_entropy: d_S (device, 1 double) receives S = -sum p_i log2 p_i, p_i =
 * h_i / n, over the occupied values of the 256-bin histogram d_hist (device,
 * as written by lz_histogram); S = 0 for an empty histogram (Section 4, the
 * entropy formula; S_max = 8).  Asynchronous on stream. */
int lz_entropy(lz_ctx *ctx, const uint64_t *d_hist, double *d_S, void *stream);

/* lz_autocorrelation: d_r (device, max_lag + 1 doubles, overwritten) receives
 * the autocorrelation coefficients of the mean-removed byte sequence d_data
 * (device, n bytes): r_k = sum_{i<n-k} (x_i - m)(x_{i+k} - m) / sum_i (x_i - m)^2,
 * r_0 = 1, r_k = 0 for k >= n, all NaN when every byte is equal or n = 0.
 * Uses the context's diagnostics workspace (calls of one context are ordered
 * across streams).  max_lag <= 16384.  Asynchronous on stream. */
int lz_autocorrelation(lz_ctx *ctx, const uint8_t *d_data, size_t n, uint32_t max_lag, double *d_r, void *stream);

/* Byte matrices (Section 4, the text and image experiments): d_img (device)
 * holds h rows of w bytes, row-major, 1 <= h, w <= 65536, h * w <= 2^24.
 *
 * lz_power_spectrum_2d: d_power (device, h * w doubles, row-major) receives
 * P[u][v] = |sum_{x,y} X[x][y] exp(-2 pi i (u x / h + v y / w))|^2, unshifted
 * (the zero frequency at [0][0]).
 *
 * lz_autocorrelation_2d: d_acf (device, h * w doubles, row-major) receives the
 * circular autocorrelation matrix of the mean-removed matrix,
 * A[dx][dy] = sum_{x,y} Xc[x][y] Xc[(x+dx) mod h][(y+dy) mod w] / sum Xc^2,
 * Xc = X - mean; all NaN for a constant matrix.  It is computed as the inverse
 * 2-D DFT of the mean-removed power spectrum (Wiener-Khinchin).
 *
 * Each 1-D transform along a side runs as an FFT when the side is at most
 * 4096 with no prime factor above 5 and as a direct DFT otherwise; the
 * routes agree within rounding.  Both use the context's diagnostics workspace (about 32 h w bytes,
 * grown on demand: LZ_E_NOMEM if it does not fit) and run asynchronously on
 * stream. */
int lz_power_spectrum_2d(lz_ctx *ctx, const uint8_t *d_img, uint32_t h, uint32_t w, double *d_power, void *stream);
int lz_autocorrelation_2d(lz_ctx *ctx, const uint8_t *d_img, uint32_t h, uint32_t w, double *d_acf, void *stream);

/* ---- the method's scalar pieces, one by one --------------------------------
 * Each evaluates one piece of the per-byte work element by element over
 * device arrays, with the same device code as the cipher kernels, so that it
 * can be checked on its own.  Asynchronous on stream; LZ_E_INVAL for a NULL
 * context or (when n > 0) a NULL array.
 *
 * lz_unit_r: d_out[i] = R(d_alpha[i], d_omega[i]) (Section 3.2, Eq. R_nu):
 * byte Omega (0 = least significant) of floor(alpha 10^13) as a two's
 * complement integer.  Omega values are taken mod 4 (the method uses 0..3). */
int lz_unit_r(lz_ctx *ctx, const double *d_alpha, const uint8_t *d_omega, size_t n, uint8_t *d_out, void *stream);

/* lz_unit_theta: d_out[i] = d_p[i] / 10^(3 + d_omega3[i]), the correctly
 * rounded quotient (Section 3.2, Step 2); omega3 taken mod 4. */
int lz_unit_theta(lz_ctx *ctx, const uint8_t *d_p, const uint8_t *d_omega3, size_t n, double *d_out, void *stream);

/* lz_unit_lorenz: each state (d_r[3i], d_r[3i+1], d_r[3i+2]) = (x, y, z) is
 * advanced in place by `steps` steps of the context's integrator with its dt
 * (Section 3.1; the loop of Step 2).  n <= 2^31. */
int lz_unit_lorenz(lz_ctx *ctx, double *d_r, size_t n, uint32_t steps, void *stream);

/* CLOCK_MONOTONIC now, in ns (the clock of arrival_ns and done_ns). */
uint64_t lz_now_ns(void);

#ifdef __cplusplus
}
#endif
#endif /* LORENZ_CIPHER_H */
