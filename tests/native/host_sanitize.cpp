// Test driver: the library's host code (argument checks, key setup, the
// serving loop and its threads, streams, batches, the diagnostics' plans)
// built with host sanitizers -- AddressSanitizer + UndefinedBehaviorSanitizer
// or ThreadSanitizer -- and run through the public C ABI.  The kernels are the
// ordinary gfx950 code; the sanitizers see host memory and host threads only.
//
// Every result is checked against the plain path (lz_encrypt / lz_decrypt) or
// against a direct definition (byte counts, lag sums).  Prints one line per
// section and "host sanitize: OK" at the end; exit status 0 on success, 1 on
// a wrong result.  Only valid inputs reach the device: the bad arguments used
// here are ones the library rejects on the host before any launch.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "../../include/lorenz_cipher.h"

namespace {

std::atomic<int> g_fail{0};  // written by the submitter, canceller and polling threads

#define HIPCHECK(x)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) {                                                                  \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);           \
            std::exit(2);                                                                        \
        }                                                                                        \
    } while (0)

#define EXPECT(cond, ...)                                                                        \
    do {                                                                                         \
        if (!(cond)) {                                                                           \
            std::printf("FAIL line %d: ", __LINE__);                                             \
            std::printf(__VA_ARGS__);                                                            \
            std::printf(" (%s)\n", lz_last_error());                                             \
            g_fail = 1;                                                                          \
        }                                                                                        \
    } while (0)

struct DevBuf {
    uint8_t *p = nullptr;
    size_t n = 0;
    explicit DevBuf(size_t bytes) : n(bytes) { HIPCHECK(hipMalloc(&p, bytes ? bytes : 1)); }
    ~DevBuf() { (void)hipFree(p); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

std::vector<uint8_t> to_host(const uint8_t *d, size_t n) {
    std::vector<uint8_t> h(n);
    if (n) HIPCHECK(hipMemcpy(h.data(), d, n, hipMemcpyDeviceToHost));
    return h;
}

void to_dev(uint8_t *d, const std::vector<uint8_t> &h) {
    if (!h.empty()) HIPCHECK(hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice));
}

std::vector<uint8_t> random_bytes(std::mt19937_64 &rng, size_t n, int lo = 0, int hi = 255) {
    std::uniform_int_distribution<int> d(lo, hi);
    std::vector<uint8_t> v(n);
    for (auto &b : v) b = (uint8_t)d(rng);
    return v;
}

// Ciphertext (body + tag) of P under pw by the plain path.
std::vector<uint8_t> plain_encrypt(lz_ctx *ctx, const std::vector<uint8_t> &pw, const std::vector<uint8_t> &P) {
    DevBuf dP(P.size()), dC(P.size() + LZ_TAG_BYTES);
    to_dev(dP.p, P);
    int rc = lz_encrypt(ctx, pw.data(), pw.size(), P.empty() ? nullptr : dP.p, P.size(), dC.p, nullptr);
    EXPECT(rc == LZ_OK, "lz_encrypt rc=%d", rc);
    HIPCHECK(hipDeviceSynchronize());
    return to_host(dC.p, P.size() + LZ_TAG_BYTES);
}

void host_helpers() {
    lz_params p;
    EXPECT(lz_params_default(nullptr) == LZ_E_INVAL, "params_default(NULL)");
    EXPECT(lz_params_default(&p) == LZ_OK && lz_params_check(&p) == LZ_OK, "defaults");
    EXPECT(lz_params_check(nullptr) == LZ_E_INVAL, "check(NULL)");
    auto bad = [&](void (*edit)(lz_params &)) {
        lz_params q;
        lz_params_default(&q);
        edit(q);
        return lz_params_check(&q) == LZ_E_INVAL;
    };
    EXPECT(bad([](lz_params &q) { q.dt = 0.0; }), "dt 0");
    EXPECT(bad([](lz_params &q) { q.dt = 1.0; }), "dt 1");
    EXPECT(bad([](lz_params &q) { q.n_it = 0; }), "n_it 0");
    EXPECT(bad([](lz_params &q) { q.block_len = 0; }), "block_len 0");
    EXPECT(bad([](lz_params &q) { q.k[1] = 2; }), "k 2");
    EXPECT(bad([](lz_params &q) { q.k[2] = 5; }), "k 5");
    EXPECT(bad([](lz_params &q) { q.integrator = 3; }), "integrator 3");
    EXPECT(bad([](lz_params &q) { q.reserved[3] = 1; }), "reserved");
    EXPECT(lz_ciphertext_len(0) == LZ_TAG_BYTES && lz_ciphertext_len(100) == 100 + LZ_TAG_BYTES, "ct len");
    std::mt19937_64 rng(11);
    lz_key k;
    for (size_t n = 0; n <= 65; ++n) {
        auto pw = random_bytes(rng, n);
        int rc = lz_key_setup(n ? pw.data() : nullptr, n, &p, &k);
        EXPECT((n >= 1 && n <= 64) ? rc == LZ_OK : rc == LZ_E_INVAL, "key_setup length %zu rc=%d", n, rc);
    }
    // every byte value in every position, for the decimal conversion of a'
    for (int v = 0; v < 256; ++v) {
        std::vector<uint8_t> pw(64, (uint8_t)v);
        EXPECT(lz_key_setup(pw.data(), pw.size(), &p, &k) == LZ_OK, "key_setup byte %d", v);
    }
    std::printf("host helpers done\n");
}

void plain_round_trips(lz_ctx *ctx) {
    std::mt19937_64 rng(12);
    for (size_t n : {size_t(0), size_t(1), size_t(255), size_t(256), size_t(257), size_t(5000), size_t(100000)}) {
        auto pw = random_bytes(rng, 1 + n % 64, 32, 126);
        auto P = random_bytes(rng, n);
        auto C = plain_encrypt(ctx, pw, P);
        DevBuf dC(C.size()), dP(n);
        to_dev(dC.p, C);
        int rc = lz_decrypt(ctx, pw.data(), pw.size(), dC.p, C.size(), n ? dP.p : nullptr, nullptr, nullptr);
        EXPECT(rc == LZ_OK && to_host(dP.p, n) == P, "round trip n=%zu rc=%d", n, rc);
        C[C.size() / 2] ^= 0x10;
        to_dev(dC.p, C);
        rc = lz_decrypt(ctx, pw.data(), pw.size(), dC.p, C.size(), n ? dP.p : nullptr, nullptr, nullptr);
        EXPECT(rc == LZ_E_INTEGRITY, "tampered n=%zu rc=%d", n, rc);
        EXPECT(to_host(dP.p, n) == std::vector<uint8_t>(n, 0), "tampered output not zeroed n=%zu", n);
    }
    EXPECT(lz_encrypt(ctx, nullptr, 3, nullptr, 0, nullptr, nullptr) == LZ_E_INVAL, "encrypt NULL");
    std::printf("plain path done\n");
}

void streams(lz_ctx *ctx) {
    std::mt19937_64 rng(13);
    for (int dec = 0; dec < 2; ++dec) {
        const size_t n = 70001;
        auto pw = random_bytes(rng, 29, 32, 126);
        auto P = random_bytes(rng, n);
        auto C = plain_encrypt(ctx, pw, P);
        const auto &in = dec ? std::vector<uint8_t>(C.begin(), C.begin() + n) : P;
        DevBuf din(n), dout(n), dtag(LZ_TAG_BYTES), dst(4);
        to_dev(din.p, in);
        if (dec) to_dev(dtag.p, std::vector<uint8_t>(C.begin() + n, C.end()));
        lz_stream *st = nullptr;
        EXPECT(lz_stream_open(ctx, dec, pw.data(), pw.size(), &st) == LZ_OK, "stream open");
        size_t off = 0;
        std::uniform_int_distribution<size_t> cut(0, 3000);
        for (int k = 0; off < n; ++k) {  // immediate and deferred updates mixed, a flush now and then
            size_t len = std::min(n - off, cut(rng));
            if (k % 3 == 2)
                EXPECT(lz_stream_update(st, din.p + off, len, dout.p + off, nullptr) == LZ_OK, "update");
            else
                EXPECT(lz_stream_update_deferred(st, din.p + off, len, dout.p + off, nullptr) == LZ_OK, "deferred update");
            if (k % 7 == 6) EXPECT(lz_stream_flush(st, nullptr) == LZ_OK, "flush");
            off += len;
            EXPECT(lz_stream_position(st) == off, "position after a chunk");
        }
        EXPECT(lz_stream_position(st) == n, "position");
        int rc = lz_stream_finish(st, dtag.p, nullptr, nullptr);
        EXPECT(rc == LZ_OK, "finish rc=%d", rc);
        EXPECT(lz_stream_finish(st, dtag.p, nullptr, nullptr) == LZ_E_INVAL, "finish twice");
        EXPECT(lz_stream_flush(st, nullptr) == LZ_E_INVAL, "flush after finish");
        EXPECT(lz_stream_update_deferred(st, din.p, 1, dout.p, nullptr) == LZ_E_INVAL, "deferred update after finish");
        EXPECT(lz_stream_close(st) == LZ_OK, "close");
        auto out = to_host(dout.p, n);
        EXPECT(out == (dec ? P : std::vector<uint8_t>(C.begin(), C.begin() + n)), "stream body dec=%d", dec);
        if (!dec) EXPECT(to_host(dtag.p, LZ_TAG_BYTES) == std::vector<uint8_t>(C.begin() + n, C.end()), "tag");
    }
    std::printf("streams done\n");
}

void batches(lz_ctx *ctx) {
    std::mt19937_64 rng(14);
    const size_t m = 57;
    std::vector<uint64_t> lens(m), in_off(m), out_off(m), pw_off(m);
    std::vector<uint32_t> pw_len(m);
    std::vector<uint8_t> pw_all, in_all, want;
    std::vector<std::vector<uint8_t>> C(m);
    std::uniform_int_distribution<uint64_t> sz(0, 9000);
    for (size_t i = 0; i < m; ++i) {
        lens[i] = sz(rng);
        auto pw = random_bytes(rng, 1 + i % 64, 32, 126);
        auto P = random_bytes(rng, lens[i]);
        C[i] = plain_encrypt(ctx, pw, P);
        pw_off[i] = pw_all.size();
        pw_len[i] = (uint32_t)pw.size();
        pw_all.insert(pw_all.end(), pw.begin(), pw.end());
        in_off[i] = in_all.size();
        in_all.insert(in_all.end(), P.begin(), P.end());
        out_off[i] = want.size();
        want.insert(want.end(), C[i].begin(), C[i].end());
    }
    DevBuf din(in_all.size()), dout(want.size()), dstat(4 * m);
    to_dev(din.p, in_all);
    lz_batch *b = nullptr;
    int rc = lz_batch_create(ctx, 0, m, lens.data(), in_off.data(), out_off.data(), pw_all.data(), pw_off.data(),
                             pw_len.data(), din.p, dout.p, nullptr, nullptr, &b);
    EXPECT(rc == LZ_OK, "batch create rc=%d", rc);
    if (rc == LZ_OK) {
        for (int rep = 0; rep < 3; ++rep) EXPECT(lz_batch_launch(b, nullptr) == LZ_OK, "batch launch");
        HIPCHECK(hipDeviceSynchronize());
        EXPECT(to_host(dout.p, want.size()) == want, "batch output");
        EXPECT(lz_batch_destroy(b) == LZ_OK, "batch destroy");
    }
    std::printf("batches done\n");
}

struct Req {
    uint64_t id;
    int dec;
    std::vector<uint8_t> pw, in, want;
    bool host_bufs;
    std::vector<uint8_t> h_in, h_out;
    uint8_t *d_in = nullptr, *d_out = nullptr;
    size_t n_in = 0, n_out = 0;
};

void serving(lz_ctx *ctx) {
    std::mt19937_64 rng(15);
    const int count = 420;
    std::vector<Req> reqs(count);
    std::lognormal_distribution<double> sz(std::log(3000.0), 1.2);
    for (int i = 0; i < count; ++i) {
        Req &r = reqs[i];
        r.id = 1000 + i;
        r.dec = i % 2;
        r.pw = random_bytes(rng, 1 + (i * 7) % 64, 32, 126);
        size_t n = std::min<size_t>((size_t)sz(rng), 200000);
        auto P = random_bytes(rng, n);
        auto C = plain_encrypt(ctx, r.pw, P);
        r.in = r.dec ? C : P;
        r.want = r.dec ? P : C;
        r.n_in = r.in.size();
        r.n_out = r.want.size();
        r.host_bufs = i % 3 == 0;
        if (r.host_bufs) {
            r.h_in = r.in;
            r.h_out.assign(r.n_out ? r.n_out : 1, 0xA5);
        } else {
            HIPCHECK(hipMalloc(&r.d_in, r.n_in ? r.n_in : 1));
            HIPCHECK(hipMalloc(&r.d_out, r.n_out ? r.n_out : 1));
            to_dev(r.d_in, r.in);
            HIPCHECK(hipMemset(r.d_out, 0xA5, r.n_out ? r.n_out : 1));
        }
    }
    lz_server_config cfg{64ull << 20, 2048, 8};
    lz_server *srv = nullptr;
    EXPECT(lz_server_create(ctx, &cfg, &srv) == LZ_OK, "server create");
    if (!srv) return;
    const uint64_t t0 = lz_now_ns();
    auto src = [&](Req &r) -> const void * { return r.host_bufs ? (const void *)r.h_in.data() : r.d_in; };
    auto dst = [&](Req &r) -> void * { return r.host_bufs ? (void *)r.h_out.data() : r.d_out; };
    auto n_plain = [](const Req &r) { return r.dec ? r.n_out : r.n_in; };
    // three submitter threads: two one by one (arrivals spread over 30 ms), one with submit_many
    auto one_by_one = [&](int first) {
        for (int i = first; i < count * 2 / 3; i += 2) {
            Req &r = reqs[i];
            int rc = lz_server_submit(srv, r.id, r.dec, r.pw.data(), r.pw.size(), src(r), n_plain(r), dst(r),
                                      t0 + 70000ull * i);
            EXPECT(rc == LZ_OK, "submit %d rc=%d", i, rc);
        }
    };
    auto many = [&]() {
        std::vector<uint64_t> ids, off, ns, arr;
        std::vector<uint8_t> dec, pw;
        std::vector<uint32_t> pl;
        std::vector<const void *> s;
        std::vector<void *> d;
        for (int i = count * 2 / 3; i < count; ++i) {
            Req &r = reqs[i];
            ids.push_back(r.id);
            dec.push_back((uint8_t)r.dec);
            off.push_back(pw.size());
            pl.push_back((uint32_t)r.pw.size());
            pw.insert(pw.end(), r.pw.begin(), r.pw.end());
            s.push_back(src(r));
            ns.push_back(n_plain(r));
            d.push_back(dst(r));
            arr.push_back(t0 + 20000000ull + 50000ull * (i - count * 2 / 3));
        }
        int rc = lz_server_submit_many(srv, ids.size(), ids.data(), dec.data(), pw.data(), off.data(), pl.data(),
                                       s.data(), ns.data(), d.data(), arr.data());
        EXPECT(rc == LZ_OK, "submit_many rc=%d", rc);
    };
    std::atomic<bool> stop_cancel{false};
    auto canceller = [&]() {
        for (int i = 0; i < count && !stop_cancel.load(); i += 7) {
            EXPECT(lz_server_cancel(srv, reqs[i].id) == LZ_OK, "cancel");
            std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
        EXPECT(lz_server_cancel(srv, 999999) == LZ_OK, "cancel unknown id");
    };
    std::thread t1(one_by_one, 0), t2(one_by_one, 1), t3(many), t4(canceller);
    std::map<uint64_t, int> status;
    lz_completion comp[256];
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(120);
    lz_server_stats stats{};
    while ((int)status.size() < count && std::chrono::steady_clock::now() < deadline) {
        int k = lz_server_poll(srv, comp, 256, 50);
        EXPECT(k >= 0, "poll rc=%d", k);
        for (int j = 0; j < k; ++j) status[comp[j].id] = comp[j].status;
        EXPECT(lz_server_stats_get(srv, &stats) == LZ_OK, "stats");
    }
    stop_cancel = true;
    t1.join();
    t2.join();
    t3.join();
    t4.join();
    EXPECT((int)status.size() == count, "completed %zu of %d", status.size(), count);
    int n_cancel = 0;
    for (Req &r : reqs) {
        auto it = status.find(r.id);
        if (it == status.end()) continue;
        std::vector<uint8_t> out = r.host_bufs ? std::vector<uint8_t>(r.h_out.begin(), r.h_out.begin() + r.n_out)
                                               : to_host(r.d_out, r.n_out);
        if (it->second == LZ_E_CANCELLED) {
            ++n_cancel;
            EXPECT(out == std::vector<uint8_t>(r.n_out, 0xA5), "cancelled request %llu wrote its output",
                   (unsigned long long)r.id);
            continue;
        }
        EXPECT(it->second == LZ_OK, "request %llu status %d", (unsigned long long)r.id, it->second);
        EXPECT(out == r.want, "request %llu output", (unsigned long long)r.id);
    }
    EXPECT(lz_server_destroy(srv) == LZ_OK, "server destroy");
    for (Req &r : reqs) {
        if (r.d_in) (void)hipFree(r.d_in);
        if (r.d_out) (void)hipFree(r.d_out);
    }
    std::printf("serving done: %d requests, %d cancelled, %llu ticks\n", count, n_cancel,
                (unsigned long long)stats.ticks);
}

void diagnostics(lz_ctx *ctx) {
    std::mt19937_64 rng(16);
    const size_t n = 1 << 20;
    auto data = random_bytes(rng, n);
    for (size_t i = 0; i < n; i += 3) data[i] = (uint8_t)(data[i] & 0x0F);  // a skewed distribution
    DevBuf d(n), dh(256 * 8), dS(8), dsums(8 * 301), dr(8 * 301);
    to_dev(d.p, data);
    EXPECT(lz_histogram(ctx, d.p, n, (uint64_t *)dh.p, nullptr) == LZ_OK, "histogram");
    EXPECT(lz_entropy(ctx, (const uint64_t *)dh.p, (double *)dS.p, nullptr) == LZ_OK, "entropy");
    EXPECT(lz_lag_sums(ctx, d.p, n, 300, (uint64_t *)dsums.p, nullptr) == LZ_OK, "lag sums");
    EXPECT(lz_autocorrelation(ctx, d.p, n, 300, (double *)dr.p, nullptr) == LZ_OK, "autocorrelation");
    HIPCHECK(hipDeviceSynchronize());
    std::vector<uint64_t> hist(256), sums(301), want_h(256, 0), want_s(301, 0);
    HIPCHECK(hipMemcpy(hist.data(), dh.p, 256 * 8, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(sums.data(), dsums.p, 301 * 8, hipMemcpyDeviceToHost));
    for (uint8_t b : data) ++want_h[b];
    for (size_t k : {size_t(0), size_t(1), size_t(17), size_t(256), size_t(300)}) {
        for (size_t i = 0; i + k < n; ++i) want_s[k] += (uint64_t)data[i] * data[i + k];
        EXPECT(sums[k] == want_s[k], "lag sum %zu", k);
    }
    EXPECT(hist == want_h, "histogram counts");
    for (auto hw : {std::pair<uint32_t, uint32_t>{64, 64}, {50, 60}, {17, 19}, {1, 1}, {128, 1}}) {
        size_t m = (size_t)hw.first * hw.second;
        DevBuf dp(8 * m), da(8 * m);
        EXPECT(lz_power_spectrum_2d(ctx, d.p, hw.first, hw.second, (double *)dp.p, nullptr) == LZ_OK,
               "power spectrum %ux%u", hw.first, hw.second);
        EXPECT(lz_autocorrelation_2d(ctx, d.p, hw.first, hw.second, (double *)da.p, nullptr) == LZ_OK,
               "2-D autocorrelation %ux%u", hw.first, hw.second);
        HIPCHECK(hipDeviceSynchronize());
        std::vector<double> pw(m);
        HIPCHECK(hipMemcpy(pw.data(), dp.p, 8 * m, hipMemcpyDeviceToHost));
        double s = 0;
        for (size_t i = 0; i < m; ++i) s += data[i];
        EXPECT(std::fabs(pw[0] - s * s) <= 1e-9 * s * s, "DC term %ux%u", hw.first, hw.second);
    }
    std::printf("diagnostics done\n");
}

void units(lz_ctx *ctx) {
    const size_t n = 1000;
    std::mt19937_64 rng(17);
    std::uniform_real_distribution<double> u(-40.0, 40.0);
    std::vector<double> alpha(n), r(3 * n);
    for (auto &a : alpha) a = u(rng);
    for (auto &v : r) v = u(rng);
    auto omega = random_bytes(rng, n, 0, 3), p = random_bytes(rng, n), om3 = random_bytes(rng, n, 0, 3);
    DevBuf da(8 * n), dom(n), dout(n), dp(n), dom3(n), dth(8 * n), drr(24 * n);
    HIPCHECK(hipMemcpy(da.p, alpha.data(), 8 * n, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(drr.p, r.data(), 24 * n, hipMemcpyHostToDevice));
    to_dev(dom.p, omega);
    to_dev(dp.p, p);
    to_dev(dom3.p, om3);
    EXPECT(lz_unit_r(ctx, (const double *)da.p, dom.p, n, dout.p, nullptr) == LZ_OK, "unit R");
    EXPECT(lz_unit_theta(ctx, dp.p, dom3.p, n, (double *)dth.p, nullptr) == LZ_OK, "unit theta");
    EXPECT(lz_unit_lorenz(ctx, (double *)drr.p, n, 100, nullptr) == LZ_OK, "unit lorenz");
    HIPCHECK(hipDeviceSynchronize());
    std::vector<double> th(n);
    HIPCHECK(hipMemcpy(th.data(), dth.p, 8 * n, hipMemcpyDeviceToHost));
    static const double p10[7] = {1, 10, 100, 1000, 10000, 100000, 1000000};
    for (size_t i = 0; i < n; ++i) EXPECT(th[i] == p[i] / p10[3 + om3[i]], "theta %zu", i);
    std::printf("unit checks done\n");
}

}  // namespace

int main() {
    host_helpers();
    lz_params prm;
    lz_params_default(&prm);
    prm.n_it = 20;
    lz_ctx *ctx = nullptr;
    int rc = lz_context_create(0, &prm, &ctx);
    if (rc != LZ_OK) {
        std::printf("context: %s\n", lz_last_error());
        return 2;
    }
    plain_round_trips(ctx);
    streams(ctx);
    batches(ctx);
    serving(ctx);
    diagnostics(ctx);
    units(ctx);
    EXPECT(lz_context_destroy(ctx) == LZ_OK, "context destroy");
    std::printf(g_fail.load() ? "host sanitize: FAILED\n" : "host sanitize: OK\n");
    return g_fail.load();
}
