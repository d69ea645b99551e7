// Host runtime of the C ABI: parameters, contexts, the plain path, the batched
// path (persistent kernel captured in a HIP graph) and the launch-shape
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "internal.h"

namespace lz {

namespace {
// fixed storage: reporting an error never allocates
thread_local char g_last_error[512];
}

void set_error(const char *msg) { std::snprintf(g_last_error, sizeof g_last_error, "%s", msg); }

int fail(int code, const char *msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? LZ_E_NOMEM : LZ_E_HIP;
}

int check_params(const lz_params &p) {
    // 0 < dt <= 0.015: above about 0.02 some starts inside the lambda ranges, and some points of the
    // attractor moved by the per-byte perturbations, leave the attractor under forward Euler and overflow
    if (!(p.dt > 0.0 && p.dt <= LZ_MAX_DT)) return fail(LZ_E_INVAL, "dt must be in (0, 0.015]");
    // lambda inside the ranges of Section 3.1 (stable chaotic phases)
    if (!(p.lambda[0] > -15.67 && p.lambda[0] < 16.01) || !(p.lambda[1] > -11.28 && p.lambda[1] < 16.01) ||
        !(p.lambda[2] > 0.090 && p.lambda[2] < 62.0))
        return fail(LZ_E_INVAL, "lambda outside the ranges of Section 3.1");
    if (p.n_it == 0) return fail(LZ_E_INVAL, "n_it must be >= 1");
    if (p.block_len == 0) return fail(LZ_E_INVAL, "block_len must be >= 1");
    if (p.integrator > LZ_INTEGRATOR_RK4) return fail(LZ_E_INVAL, "unknown integrator");
    for (int i = 0; i < 3; ++i)
        if (p.k[i] != 3 && p.k[i] != 4) return fail(LZ_E_INVAL, "k_i must be 3 or 4");
    for (uint8_t r : p.reserved)
        if (r) return fail(LZ_E_INVAL, "reserved bytes of lz_params must be zero");
    return LZ_OK;
}

int check_blocks(const lz_params &p, uint64_t n, uint64_t *nb_out) {
    if (n > LZ_MAX_MESSAGE) return fail(LZ_E_INVAL, "message longer than 2^32 bytes");
    const uint64_t nb = n == 0 ? 1 : (n + p.block_len - 1) / p.block_len;
    // block b starts at r0 + b 2^-24: at most 2^24 blocks keep every start within 1 of r0
    if (nb > LZ_MAX_BLOCKS) return fail(LZ_E_INVAL, "message of more than 2^24 blocks (raise block_len)");
    if (nb_out) *nb_out = nb;
    return LZ_OK;
}

namespace {

KernelShape to_shape(const lz_launch &l) {
    return KernelShape{(int)l.chains_per_lane, (int)l.wg_size, (int)l.tile, (int)l.waves_per_simd};
}

lz_launch to_launch(const KernelShape &s) {
    lz_launch l;
    l.chains_per_lane = (uint32_t)s.m;
    l.wg_size = (uint32_t)s.wg;
    l.tile = (uint32_t)s.tile;
    l.waves_per_simd = (uint32_t)s.wps;
    return l;
}

// Launch shape of the plain path for a message of nb blocks: several chains per lane trade each
// chain's latency for issue density, so they are used only when the message gives every SIMD at
// least two waves of them.
KernelShape plain_shape(const lz_ctx *c, uint64_t nb) {
    KernelShape sh = c->shape;
    if (sh.m > 1 && nb < (uint64_t)sh.m * c->dev.cus * 4 * WAVE_LANES * 2) sh.m = 1;
    return sh;
}

// Orders a call on stream s after the previous call that used the same
// workspace (possibly on another stream).
int order_after(hipStream_t s, hipStream_t &last_stream, hipEvent_t ev, bool &has_last) {
    if (has_last && last_stream != s) LZ_HIP(hipStreamWaitEvent(s, ev, 0));
    return LZ_OK;
}

int record(hipStream_t s, hipStream_t &last_stream, hipEvent_t ev, bool &has_last) {
    LZ_HIP(hipEventRecord(ev, s));
    last_stream = s;
    has_last = true;
    return LZ_OK;
}

}  // namespace
}  // namespace lz

using namespace lz;

// ---- host-only helpers -------------------------------------------------------------

extern "C" int lz_params_default(lz_params *out) {
    if (!out) return fail(LZ_E_INVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    out->dt = 0.01;
    out->lambda[0] = out->lambda[1] = out->lambda[2] = 1.0;
    out->n_it = 3000;
    out->block_len = 256;
    out->k[0] = out->k[1] = out->k[2] = 4;
    return LZ_OK;
}

extern "C" int lz_params_check(const lz_params *prm) {
    if (!prm) return fail(LZ_E_INVAL, "prm is NULL");
    return check_params(*prm);
}

extern "C" size_t lz_ciphertext_len(size_t n_plain) { return n_plain + LZ_TAG_BYTES; }

extern "C" int lz_block_count(const lz_params *prm, uint64_t n, uint64_t *nb) {
    if (!prm || !nb) return fail(LZ_E_INVAL, "NULL argument");
    if (int rc = check_params(*prm)) return rc;
    return check_blocks(*prm, n, nb);
}

extern "C" int lz_key_setup(const uint8_t *pw, size_t n_pw, const lz_params *prm, lz_key *out) {
    if (!pw || !out) return fail(LZ_E_INVAL, "NULL argument");
    lz_params def;
    if (!prm) {
        lz_params_default(&def);
        prm = &def;
    }
    if (int rc = check_params(*prm)) return rc;
    if (n_pw == 0 || n_pw > LZ_MAX_PASSWORD) return fail(LZ_E_INVAL, "password length must be 1..64");
    return key_setup(pw, n_pw, *prm, *out);
}

extern "C" const char *lz_last_error(void) { return g_last_error; }

extern "C" uint64_t lz_now_ns(void) {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---- context ---------------------------------------------------------------------------

extern "C" int lz_context_create(int device, const lz_params *prm, lz_ctx **out) {
    if (!out) return fail(LZ_E_INVAL, "out is NULL");
    *out = nullptr;
    lz_params p;
    if (prm) p = *prm;
    else lz_params_default(&p);
    if (int rc = check_params(p)) return rc;
    int ndev = 0;
    LZ_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(LZ_E_INVAL, "no such HIP device");
    LZ_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    LZ_HIP(hipGetDeviceProperties(&prop, device));
    lz_ctx *c = new (std::nothrow) lz_ctx();
    if (!c) return fail(LZ_E_NOMEM, "host allocation failed");
    c->device = device;
    c->prm = p;
    c->dev.cus = prop.multiProcessorCount;
    c->dev.lds_per_wg_max = (int)prop.sharedMemPerBlock;
    std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    // one chain per lane, 4 waves per workgroup, 128-byte tiles (one L2 line per chain per refill)
    c->shape = KernelShape{1, 256, 128, 4};
    if (!shape_valid(c->shape, c->dev)) c->shape = KernelShape{1, 64, 32, 4};
    hipError_t e = hipMalloc(&c->ws_tag, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&c->ws_status, sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc(&c->host_status, sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->last_event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->diag_event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&c->diag_merge, DIAG_MERGE_WORDS * 8);
    if (e == hipSuccess) e = hipMemset(c->diag_merge, 0, DIAG_MERGE_WORDS * 8);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "context allocation");
        lz_context_destroy(c);
        return rc;
    }
    c->has_last = false;
    c->last_stream = nullptr;
    *out = c;
    return LZ_OK;
}

extern "C" int lz_context_destroy(lz_ctx *c) {
    if (!c) return LZ_OK;
    hipSetDevice(c->device);
    if (c->has_last) hipEventSynchronize(c->last_event);
    if (c->diag_has_last) hipEventSynchronize(c->diag_event);
    if (c->diag_ws) hipFree(c->diag_ws);
    if (c->diag_merge) hipFree(c->diag_merge);
    if (c->diag_event) hipEventDestroy(c->diag_event);
    if (c->ws_tag) hipFree(c->ws_tag);
    if (c->ws_status) hipFree(c->ws_status);
    if (c->host_status) hipHostFree(c->host_status);
    if (c->last_event) hipEventDestroy(c->last_event);
    delete c;
    return LZ_OK;
}

extern "C" int lz_context_params(const lz_ctx *c, lz_params *out) {
    if (!c || !out) return fail(LZ_E_INVAL, "NULL argument");
    *out = c->prm;
    return LZ_OK;
}

extern "C" int lz_context_set_launch(lz_ctx *c, const lz_launch *shape) {
    if (!c || !shape) return fail(LZ_E_INVAL, "NULL argument");
    KernelShape s = to_shape(*shape);
    if (!shape_valid(s, c->dev)) return fail(LZ_E_INVAL, "launch shape out of range or over the LDS limit");
    c->shape = s;
    return LZ_OK;
}

extern "C" int lz_context_get_launch(const lz_ctx *c, lz_launch *out) {
    if (!c || !out) return fail(LZ_E_INVAL, "NULL argument");
    *out = to_launch(c->shape);
    return LZ_OK;
}

// ---- plain path ----------------------------------------------------------------------------

extern "C" int lz_encrypt_key(lz_ctx *c, const lz_key *key, const uint8_t *d_P, size_t n, uint8_t *d_C,
                              void *stream) {
    if (!c || !key || !d_C || (!d_P && n)) return fail(LZ_E_INVAL, "NULL argument");
    uint64_t nb = 0;
    if (int rc = check_blocks(c->prm, n, &nb)) return rc;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    if (int rc = order_after(s, c->last_stream, c->last_event, c->has_last)) return rc;
    LZ_HIP(launch_fill_u64(c->ws_tag, 3, s));
    LZ_HIP(launch_plain(plain_shape(c, nb), *key, c->prm, 0, d_P, d_C, n, c->ws_tag, s));
    LZ_HIP(launch_plain_finalize(0, c->ws_tag, nullptr, d_C + n, nullptr, nullptr, n, s));
    return record(s, c->last_stream, c->last_event, c->has_last);
}

extern "C" int lz_decrypt_key(lz_ctx *c, const lz_key *key, const uint8_t *d_C, size_t n_c, uint8_t *d_P,
                              int32_t *d_status, void *stream) {
    if (!c || !key || !d_C) return fail(LZ_E_INVAL, "NULL argument");
    if (n_c < LZ_TAG_BYTES) return fail(LZ_E_INVAL, "ciphertext shorter than the 24-byte tag");
    const size_t n = n_c - LZ_TAG_BYTES;
    uint64_t nb = 0;
    if (int rc = check_blocks(c->prm, n, &nb)) return rc;
    if (!d_P && n) return fail(LZ_E_INVAL, "NULL plaintext buffer");
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    if (int rc = order_after(s, c->last_stream, c->last_event, c->has_last)) return rc;
    int32_t *st = d_status ? d_status : c->ws_status;
    LZ_HIP(launch_fill_u64(c->ws_tag, 3, s));
    LZ_HIP(launch_plain(plain_shape(c, nb), *key, c->prm, 1, d_C, d_P, n, c->ws_tag, s));
    LZ_HIP(launch_plain_finalize(1, c->ws_tag, d_C + n, nullptr, st, d_P, n, s));
    if (d_status) return record(s, c->last_stream, c->last_event, c->has_last);
    LZ_HIP(hipMemcpyAsync(c->host_status, c->ws_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (int rc = record(s, c->last_stream, c->last_event, c->has_last)) return rc;
    LZ_HIP(hipStreamSynchronize(s));
    if (*c->host_status != LZ_OK) return fail(LZ_E_INTEGRITY, "integrity check failed: ciphertext altered or wrong password");
    return LZ_OK;
}

extern "C" int lz_encrypt(lz_ctx *c, const uint8_t *pw, size_t n_pw, const uint8_t *d_P, size_t n, uint8_t *d_C,
                          void *stream) {
    if (!c || !pw) return fail(LZ_E_INVAL, "NULL argument");
    lz_key key;
    if (int rc = lz_key_setup(pw, n_pw, &c->prm, &key)) return rc;
    return lz_encrypt_key(c, &key, d_P, n, d_C, stream);
}

extern "C" int lz_decrypt(lz_ctx *c, const uint8_t *pw, size_t n_pw, const uint8_t *d_C, size_t n_c, uint8_t *d_P,
                          int32_t *d_status, void *stream) {
    if (!c || !pw) return fail(LZ_E_INVAL, "NULL argument");
    lz_key key;
    if (int rc = lz_key_setup(pw, n_pw, &c->prm, &key)) return rc;
    return lz_decrypt_key(c, &key, d_C, n_c, d_P, d_status, stream);
}

// ---- batched path -----------------------------------------------------------------------------

struct lz_batch {
    lz_ctx *ctx;
    int decrypt;
    KernelShape shape;
    BatchDev dev;
    void *dmem;           // one device allocation holding every descriptor array
    int32_t **status_slot;  // in dmem: the address of the statuses the next replay writes (decrypt)
    int32_t *bound_status;  // statuses given at creation (lz_batch_launch), may be NULL
    hipGraph_t graph;
    hipGraphExec_t exec;
    // replay ordering across streams; a replay changes only these, so calls take a const batch
    mutable hipEvent_t last_event;
    mutable hipStream_t last_stream;
    mutable bool has_last;
};

namespace {

int batch_free(lz_batch *b) {
    if (!b) return LZ_OK;
    hipSetDevice(b->ctx->device);
    if (b->has_last) hipEventSynchronize(b->last_event);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->dmem) hipFree(b->dmem);
    if (b->last_event) hipEventDestroy(b->last_event);
    delete b;
    return LZ_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace {

// lz_batch_create with the method parameters given explicitly (the autotuner ranks shapes on
// a shorter n_it than the context's).
int batch_create(lz_ctx *c, const lz_params &prm, int decrypt, size_t n_msg, const uint64_t *lens,
                 const uint64_t *in_off, const uint64_t *out_off, const uint8_t *pw, const uint64_t *pw_off,
                 const uint32_t *pw_len, const uint8_t *d_in, uint8_t *d_out, int32_t *d_status,
                 const lz_launch *shape, lz_batch **out) {
    if (!out) return fail(LZ_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!c || !lens || !in_off || !out_off || !pw || !pw_off || !pw_len || !d_in || !d_out)
        return fail(LZ_E_INVAL, "NULL argument");
    if (n_msg == 0 || n_msg > (1u << 30)) return fail(LZ_E_INVAL, "n_msg must be in [1, 2^30]");
    KernelShape sh = shape ? to_shape(*shape) : c->shape;
    if (!shape_valid(sh, c->dev)) return fail(LZ_E_INVAL, "launch shape out of range or over the LDS limit");
    LZ_HIP(hipSetDevice(c->device));
    const uint32_t B = prm.block_len;

    std::vector<MsgDesc> md(n_msg);
    std::vector<uint64_t> prefix(n_msg + 1, 0);
    std::vector<uint32_t> tails;
    for (size_t i = 0; i < n_msg; ++i) {
        if (int rc = check_blocks(prm, lens[i], nullptr)) return rc;
        lz_key key;
        if (int rc = lz_key_setup(pw + pw_off[i], pw_len[i], &prm, &key)) return rc;
        MsgDesc &m = md[i];
        std::memset(&m, 0, sizeof m);
        for (int j = 0; j < 3; ++j) {
            m.ap[j] = key.a_prime[j];
            m.r0[j] = key.r0[j];
            m.mu[j] = key.mu[j];
            m.om[j] = key.omega[j];
            m.k[j] = key.k[j];
        }
        m.decrypt = (uint8_t)(decrypt ? 1 : 0);
        m.n = lens[i];
        m.nb = (uint32_t)(lens[i] == 0 ? 1 : (lens[i] + B - 1) / B);
        m.in = d_in + in_off[i];
        m.out = d_out + out_off[i];
        prefix[i + 1] = prefix[i] + lens[i] / B;
        if (lens[i] % B != 0 || lens[i] == 0) tails.push_back((uint32_t)i);
    }
    // partial blocks longest first (a wave's lanes then finish together), ties by index
    std::stable_sort(tails.begin(), tails.end(),
                     [&](uint32_t a, uint32_t b) { return lens[a] % B > lens[b] % B; });

    lz_batch *b = new (std::nothrow) lz_batch();
    if (!b) return fail(LZ_E_NOMEM, "host allocation failed");
    b->ctx = c;
    b->decrypt = decrypt ? 1 : 0;
    b->shape = sh;
    const size_t o_msgs = 0;
    const size_t o_prefix = align_up(o_msgs + n_msg * sizeof(MsgDesc), 256);
    const size_t o_tail = align_up(o_prefix + (n_msg + 1) * sizeof(uint64_t), 256);
    const size_t o_slot = align_up(o_tail + std::max<size_t>(tails.size(), 1) * sizeof(uint32_t), 256);
    const size_t o_tag = o_slot + 256;
    const size_t total = o_tag + (3 * n_msg + 1) * sizeof(unsigned long long);
    hipError_t e = hipMalloc(&b->dmem, total);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "hipMalloc(batch descriptors)");
    }
    char *base = static_cast<char *>(b->dmem);
    e = hipMemcpy(base + o_msgs, md.data(), n_msg * sizeof(MsgDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_prefix, prefix.data(), (n_msg + 1) * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tails.empty())
        e = hipMemcpy(base + o_tail, tails.data(), tails.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    b->status_slot = reinterpret_cast<int32_t **>(base + o_slot);
    b->bound_status = decrypt ? d_status : nullptr;
    if (e == hipSuccess) e = hipMemcpy(b->status_slot, &b->bound_status, sizeof(int32_t *), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "hipMemcpy(batch descriptors)");
    }
    BatchDev &d = b->dev;
    d.msgs = reinterpret_cast<const MsgDesc *>(base + o_msgs);
    d.full_prefix = reinterpret_cast<const uint64_t *>(base + o_prefix);
    d.tail_msg = reinterpret_cast<const uint32_t *>(base + o_tail);
    d.n_msg = (uint32_t)n_msg;
    d.n_tail = (uint32_t)tails.size();
    d.n_full = prefix[n_msg];
    const uint64_t per_task = 64ull * sh.m;
    d.n_tasks = (d.n_full + d.n_tail + per_task - 1) / per_task;
    d.tag_acc = reinterpret_cast<unsigned long long *>(base + o_tag);
    d.counter = d.tag_acc + 3 * n_msg;
    d.status_ref = b->status_slot;

    // capture [reset, persistent kernel, finalize]
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = launch_fill_u64(d.tag_acc, 3 * n_msg + 1, cap);
        hipError_t e2 = e1 == hipSuccess ? launch_batch(sh, c->dev, prm, d, cap) : e1;
        hipError_t e3 = e2 == hipSuccess ? launch_batch_finalize(d, b->decrypt, cap) : e2;
        e = hipStreamEndCapture(cap, &b->graph);
        if (e3 != hipSuccess) e = e3;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    hipStreamDestroy(cap);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->last_event, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch graph capture");
    }
    *out = b;
    return LZ_OK;
}

// One replay of the batch graph on stream; for a decrypt batch the statuses go to d_status.
int batch_replay(const lz_batch *b, int32_t *d_status, hipStream_t s) {
    LZ_HIP(hipSetDevice(b->ctx->device));
    if (int rc = order_after(s, b->last_stream, b->last_event, b->has_last)) return rc;
    if (b->decrypt) LZ_HIP(launch_set_status_ref(b->status_slot, d_status, s));
    LZ_HIP(hipGraphLaunch(b->exec, s));
    return record(s, b->last_stream, b->last_event, b->has_last);
}

}  // namespace

extern "C" int lz_batch_create(lz_ctx *c, int decrypt, size_t n_msg, const uint64_t *lens, const uint64_t *in_off,
                               const uint64_t *out_off, const uint8_t *pw, const uint64_t *pw_off,
                               const uint32_t *pw_len, const uint8_t *d_in, uint8_t *d_out, int32_t *d_status,
                               const lz_launch *shape, lz_batch **out) {
    if (!c) {
        if (out) *out = nullptr;
        return fail(LZ_E_INVAL, "NULL argument");
    }
    return batch_create(c, c->prm, decrypt, n_msg, lens, in_off, out_off, pw, pw_off, pw_len, d_in, d_out, d_status,
                        shape, out);
}

extern "C" int lz_encrypt_batch(lz_ctx *c, const lz_batch *b, void *stream) {
    if (!c || !b) return fail(LZ_E_INVAL, "NULL argument");
    if (b->ctx != c) return fail(LZ_E_INVAL, "batch belongs to another context");
    if (b->decrypt) return fail(LZ_E_INVAL, "batch was created for decryption");
    return batch_replay(b, nullptr, (hipStream_t)stream);
}

extern "C" int lz_decrypt_batch(lz_ctx *c, const lz_batch *b, int32_t *d_status, void *stream) {
    if (!c || !b || !d_status) return fail(LZ_E_INVAL, "NULL argument");
    if (b->ctx != c) return fail(LZ_E_INVAL, "batch belongs to another context");
    if (!b->decrypt) return fail(LZ_E_INVAL, "batch was created for encryption");
    return batch_replay(b, d_status, (hipStream_t)stream);
}

extern "C" int lz_batch_launch(lz_batch *b, void *stream) {
    if (!b) return fail(LZ_E_INVAL, "batch is NULL");
    if (b->decrypt && !b->bound_status)
        return fail(LZ_E_INVAL, "decrypt batch created without d_status: use lz_decrypt_batch");
    return batch_replay(b, b->bound_status, (hipStream_t)stream);
}

extern "C" int lz_batch_destroy(lz_batch *b) { return batch_free(b); }

// ---- autotuner ---------------------------------------------------------------------------------

namespace {

// The candidate grid: 1, 2 or 4 chains per lane and 1..8 resident waves per SIMD with 4 to 8
// chains in flight per SIMD slot, 64-, 128- or 256-thread workgroups, 16- to 128-byte tiles.
std::vector<KernelShape> shape_grid(const KernelShape &first, const DevInfo &dev) {
    std::vector<KernelShape> g;
    if (shape_valid(first, dev)) g.push_back(first);
    for (int m : {1, 2, 4})
        for (int wps : {1, 2, 4, 8})
            for (int wg : {256, 128, 64})
                for (int tile : {128, 64, 32, 16}) {
                    if (m * wps < 4 || m * wps > 8) continue;
                    const KernelShape sh{m, wg, tile, wps};
                    if (!shape_valid(sh, dev)) continue;
                    if (sh.m == first.m && sh.wg == first.wg && sh.tile == first.tile && sh.wps == first.wps) continue;
                    g.push_back(sh);
                }
    return g;
}

// Synthetic batch of the autotuner: about 1.5 resident rounds of single-chain lanes at 4 waves
// per SIMD, in messages of 64 full blocks, every fourth with a ragged tail, random bytes,
// distinct 16-byte passwords.
struct TuneBatch {
    std::vector<uint64_t> lens, in_off, out_off, pw_off;
    std::vector<uint32_t> pw_len;
    std::vector<uint8_t> pw;
    uint8_t *d_in = nullptr, *d_out = nullptr;
    ~TuneBatch() {
        if (d_in) (void)hipFree(d_in);
        if (d_out) (void)hipFree(d_out);
    }
};

int make_tune_batch(const lz_ctx *c, TuneBatch &t) {
    const uint32_t B = c->prm.block_len;
    const uint64_t chains = (uint64_t)c->dev.cus * 4 * 4 * 64 * 3 / 2;
    const uint64_t per_msg = 64;
    const size_t n_msg = (size_t)((chains + per_msg - 1) / per_msg);
    t.lens.resize(n_msg);
    t.in_off.resize(n_msg);
    t.out_off.resize(n_msg);
    t.pw_off.resize(n_msg);
    t.pw_len.resize(n_msg);
    t.pw.resize(n_msg * 16);
    uint64_t tot_in = 0, tot_out = 0;
    uint64_t st = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return st;
    };
    for (size_t i = 0; i < n_msg; ++i) {
        t.lens[i] = per_msg * B - (i % 4 == 3 ? (rnd() % B) : 0);
        t.in_off[i] = tot_in;
        t.out_off[i] = tot_out;
        tot_in += t.lens[i];
        tot_out += t.lens[i] + LZ_TAG_BYTES;
        t.pw_off[i] = 16 * i;
        t.pw_len[i] = 16;
        for (int q = 0; q < 16; ++q) t.pw[16 * i + q] = (uint8_t)(32 + rnd() % 95);
    }
    LZ_HIP(hipMalloc(&t.d_in, tot_in));
    LZ_HIP(hipMalloc(&t.d_out, tot_out));
    std::vector<uint8_t> h(tot_in);
    for (auto &v : h) v = (uint8_t)rnd();
    LZ_HIP(hipMemcpy(t.d_in, h.data(), tot_in, hipMemcpyHostToDevice));
    return LZ_OK;
}

// Time of one launch of the tuning batch in shape sh with parameters prm (after `warm` untimed
// launches); *ms = -1 if the shape cannot run.
int time_shape(lz_ctx *c, const lz_params &prm, const TuneBatch &t, const KernelShape &sh, int warm, hipStream_t s,
               hipEvent_t e0, hipEvent_t e1, double *ms) {
    lz_launch l = to_launch(sh);
    lz_batch *b = nullptr;
    *ms = -1;
    int rc = batch_create(c, prm, 0, t.lens.size(), t.lens.data(), t.in_off.data(), t.out_off.data(), t.pw.data(),
                          t.pw_off.data(), t.pw_len.data(), t.d_in, t.d_out, nullptr, &l, &b);
    if (rc != LZ_OK) return rc;
    for (int i = 0; i < warm && rc == LZ_OK; ++i) rc = lz_batch_launch(b, s);
    hipError_t e = hipSuccess;
    if (rc == LZ_OK) e = hipEventRecord(e0, s);
    if (rc == LZ_OK && e == hipSuccess) rc = lz_batch_launch(b, s);
    if (rc == LZ_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (rc == LZ_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float f = 0;
    if (rc == LZ_OK && e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
    batch_free(b);
    if (rc != LZ_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *ms = f;
    return LZ_OK;
}

}  // namespace

extern "C" int lz_autotune(lz_ctx *c, double budget_ms, lz_launch *best) {
    if (!c) return fail(LZ_E_INVAL, "ctx is NULL");
    LZ_HIP(hipSetDevice(c->device));
    TuneBatch t;
    if (int rc = make_tune_batch(c, t)) return rc;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = e == hipSuccess ? LZ_OK : hip_fail(e, "autotune stream");
    // stage 1: every shape of the grid at a tenth of n_it (the same per-byte loop, a tenth of the
    // time), one untimed launch for each kernel instance's first use
    lz_params quick = c->prm;
    quick.n_it = c->prm.n_it >= 30 ? c->prm.n_it / 10 : c->prm.n_it;
    const std::vector<KernelShape> grid = shape_grid(c->shape, c->dev);
    std::vector<std::pair<double, KernelShape>> ranked;
    double spent = 0;
    bool warmed[5] = {false, false, false, false, false};
    for (const KernelShape &sh : grid) {
        if (rc != LZ_OK || (budget_ms > 0 && spent > budget_ms && !ranked.empty())) break;
        double ms = -1;
        rc = time_shape(c, quick, t, sh, warmed[sh.m] ? 0 : 1, s, e0, e1, &ms);
        warmed[sh.m] = true;
        if (rc == LZ_OK && ms > 0) {
            spent += ms;
            ranked.emplace_back(ms, sh);
        }
    }
    // stage 2: the three fastest at the context's n_it
    KernelShape best_sh = c->shape;
    double best_ms = 1e30;
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<double, KernelShape> &a, const std::pair<double, KernelShape> &b) {
                         return a.first < b.first;
                     });
    for (size_t i = 0; i < ranked.size() && i < 3 && rc == LZ_OK; ++i) {
        double ms = -1;
        rc = time_shape(c, c->prm, t, ranked[i].second, 1, s, e0, e1, &ms);
        if (rc == LZ_OK && ms > 0 && ms < best_ms) {
            best_ms = ms;
            best_sh = ranked[i].second;
        }
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    if (rc != LZ_OK) return rc;
    c->shape = best_sh;
    c->tuned_ms = best_ms < 1e30 ? best_ms : 0;
    if (best) *best = to_launch(best_sh);
    return LZ_OK;
}

namespace {

// Key of a tuned shape: the device (gfx arch, CU count) and the parameters that shape the kernel's
// work (integrator, n_it, block_len).
std::string tune_key(const lz_ctx *c) {
    char k[256];
    std::snprintf(k, sizeof k, "%s cus=%d integrator=%u n_it=%u block_len=%u", c->arch, c->dev.cus,
                  (unsigned)c->prm.integrator, c->prm.n_it, c->prm.block_len);
    return k;
}

std::string default_tune_path() {
    if (const char *p = std::getenv("LZ_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    if (!home || !*home) return "";
    return std::string(home) + "/.cache/lorenz_cipher/launch_shapes.tsv";
}

}  // namespace

extern "C" int lz_autotune_cached(lz_ctx *c, const char *path, double budget_ms, lz_launch *best, int *from_cache) {
    if (!c) return fail(LZ_E_INVAL, "ctx is NULL");
    if (from_cache) *from_cache = 0;
    const std::string file = path ? std::string(path) : default_tune_path();
    const std::string key = tune_key(c);
    std::vector<std::string> lines;
    if (!file.empty()) {
        if (FILE *f = std::fopen(file.c_str(), "r")) {
            char buf[512];
            while (std::fgets(buf, sizeof buf, f)) {
                std::string line(buf);
                while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
                const size_t tab = line.find('\t');
                if (tab != std::string::npos && line.compare(0, tab, key) == 0 && tab == key.size()) {
                    KernelShape sh{};
                    if (std::sscanf(line.c_str() + tab + 1, "%d %d %d %d", &sh.m, &sh.wg, &sh.tile, &sh.wps) == 4 &&
                        shape_valid(sh, c->dev)) {
                        std::fclose(f);
                        c->shape = sh;
                        if (best) *best = to_launch(sh);
                        if (from_cache) *from_cache = 1;
                        return LZ_OK;
                    }
                    continue;  // a damaged entry is dropped and tuned again
                }
                if (!line.empty()) lines.push_back(line);
            }
            std::fclose(f);
        }
    }
    lz_launch l;
    if (int rc = lz_autotune(c, budget_ms, &l)) return rc;
    if (best) *best = l;
    if (file.empty()) return LZ_OK;
    // rewrite the file with this entry added, through a temporary file and a rename
    const size_t slash = file.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = file.substr(0, slash);
        for (size_t p = 1; p <= dir.size(); ++p)
            if (p == dir.size() || dir[p] == '/') (void)mkdir(dir.substr(0, p).c_str(), 0755);
    }
    char entry[512];
    std::snprintf(entry, sizeof entry, "%s\t%u %u %u %u\t%.3f", key.c_str(), l.chains_per_lane, l.wg_size, l.tile,
                  l.waves_per_simd, c->tuned_ms);
    lines.push_back(entry);
    const std::string tmp = file + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return LZ_OK;  // the shape is tuned and set; only the cache could not be written
    for (const std::string &line : lines) std::fprintf(f, "%s\n", line.c_str());
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), file.c_str()) != 0) std::remove(tmp.c_str());
    return LZ_OK;
}
