// Continuous-batching request loop (serving).  Each admitted request gets one
// chain slot per block (block b of the parallel version, Section 5), a
// device-side request record and arena space for its input and output bytes.
// A tick advances chains by up to tick_bytes bytes with the exact per-chain
// checkpoint (r, alpha, mu, Omega) kept in device memory, so a request's bytes
// do not depend on what else is admitted or when its chains run.  Requests
// that arrive while a tick runs are admitted at the next tick boundary, as
// chain slots and the device-memory budget allow (FIFO, no overtaking): the
// host prepares and queues the next tick shortly before the running one is
// expected to end (from the measured duration of earlier ticks), so that
// requests arriving during a tick join the very next one.
//
// Every chain of a tick advances at the pace of the most loaded SIMD.  Under
// the adaptive policy a tick holds at most k waves per SIMD, with k chosen
// from the backlog (the unfinished chains of admitted and waiting requests):
// one wave while the backlog is at most 3 waves per SIMD, so that each chain
// runs at its single-wave pace and the rest wait their turn; two up to 6
// waves; then doubling, up to run_waves, where a tick issues as densely as the
// plain kernel.  The tick takes requests in admission order, each with all of
// its unfinished chains or not at all, and fills the room a large request
// leaves with later ones that fit.  The all-chains policy runs every admitted
// chain in every tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

using namespace lz;

namespace {

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
  public:
    explicit Arena(uint64_t size = 0) { reset(size); }
    void reset(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t &off) {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

struct Request {
    uint64_t id, seq;
    int decrypt;
    lz_key key;
    const void *src;
    void *dst;
    bool src_dev = false, dst_dev = false;  // device memory: copied by the batched copy kernel
    uint64_t n;          // plaintext length
    uint64_t arrival_ns;
    uint64_t admit_ns = 0;
    // placement
    uint32_t req_slot = 0;
    uint32_t nb = 0;
    std::vector<uint32_t> slots;  // chain slot of block b
    bool released = false;    // resources returned; leaves the active list at the next compaction
    uint64_t arena_off = 0, arena_bytes = 0;
    uint32_t ticks_full = 0, ticks_tail = 0;  // ticks until full / tail chains finish
    uint32_t ticks_run = 0;
    bool cancelled = false;   // lz_server_cancel: no further ticks; released once no tick in flight lists it
    uint64_t last_tick = 0;   // sequence number of the last tick that listed its chains
};

struct ArrivalLater {
    bool operator()(const Request *a, const Request *b) const {
        return a->arrival_ns != b->arrival_ns ? a->arrival_ns > b->arrival_ns : a->seq > b->seq;
    }
};

uint64_t in_len(const Request &r) { return r.decrypt ? r.n + LZ_TAG_BYTES : r.n; }
uint64_t out_len(const Request &r) { return r.decrypt ? r.n : r.n + LZ_TAG_BYTES; }

uint64_t pieces_of(uint64_t bytes) { return (bytes + COPY_PIECE_BYTES - 1) / COPY_PIECE_BYTES; }

uint64_t chains_of(const Request &r, uint32_t block_len) { return r.n == 0 ? 1 : (r.n + block_len - 1) / block_len; }

// Device memory of any device is copied by kernels; everything else (pageable or
// pinned host memory) by hipMemcpyAsync.
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // pageable memory is not known to the runtime
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Late admission: the next tick is queued a margin before the running one is expected to end,
// time for the host to wake, admit, copy inputs and install records on the staging stream.  The
// margin adapts: when a tick queued this way starts more than LATE_GAP_NS after the one before
// it, the margin grows by LATE_STEP_UP_NS; otherwise it shrinks by LATE_STEP_DOWN_NS, within
// [LATE_MARGIN_MIN_NS, LATE_MARGIN_MAX_NS].
constexpr double LATE_MARGIN_MIN_NS = 150e3, LATE_MARGIN_MAX_NS = 1000e3, LATE_MARGIN_START_NS = 500e3;
constexpr double LATE_STEP_UP_NS = 100e3, LATE_STEP_DOWN_NS = 5e3, LATE_GAP_NS = 20e3;
constexpr uint32_t PIECES_MAX = 4096;  // copy pieces staged per tick (inputs) and per batch (outputs)
constexpr uint64_t DEV_COPY_MAX = (PIECES_MAX / 2) * COPY_PIECE_BYTES;  // larger copies use hipMemcpyAsync

void classify(Request *r) {
    r->src_dev = in_len(*r) <= DEV_COPY_MAX && is_device_ptr(r->src);
    r->dst_dev = out_len(*r) <= DEV_COPY_MAX && is_device_ptr(r->dst);
}

}  // namespace

// Buffers of one tick.  Two of them alternate so that the host prepares and
// queues tick k+1 while tick k runs, and reads tick k's completions while
// tick k+1 runs.
struct TickSlot {
    uint32_t *h_list = nullptr, *d_list = nullptr;  // active chain slots
    uint32_t *h_done = nullptr, *d_done = nullptr;  // [0] count, [1] pad, [2..] completed requests
    ReqDesc *h_req = nullptr, *d_req = nullptr;     // records of the requests admitted for this tick
    uint32_t *h_meta = nullptr, *d_meta = nullptr;  // 3 words per admitted request
    uint32_t *h_idx = nullptr, *d_idx = nullptr;    // chain slots of the admitted requests
    CopyPiece *h_in = nullptr, *d_in = nullptr;     // input copies of admitted requests in device memory
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    bool in_flight = false;
    uint64_t bytes = 0;
    uint64_t seq = 0;     // tick sequence number (1, 2, ...)
    uint32_t waves = 0;   // waves per SIMD of the tick's chains, at most
    bool late = false;    // queued while the tick before it ran: its start shows whether in time
};

struct lz_server {
    lz_ctx *ctx;
    lz_server_config cfg;
    KernelShape shape;
    uint32_t max_chains, max_reqs, max_new;
    uint64_t simd_chains;  // chains of one wave on every SIMD of the device
    uint64_t waiting_chains = 0;  // chains of the requests in `waiting`
    // device memory
    uint8_t *arena_mem = nullptr;
    ChainSlot *slots = nullptr;
    ReqDesc *reqs = nullptr;
    uint32_t *d_zero_ids = nullptr;
    uint32_t *h_zero_ids = nullptr;
    CopyPiece *h_out = nullptr, *d_out = nullptr;  // output copies to device memory
    TickSlot ts[2];
    int cur = 0;
    hipStream_t stream = nullptr;       // installs, ticks
    hipStream_t in_stream = nullptr;    // staging of the next tick (overlaps the running tick)
    hipStream_t copy_stream = nullptr;  // completion reads, zeroing, output copies
    hipEvent_t ev_in = nullptr;         // orders a tick after its staging
    Arena arena;
    // host bookkeeping (server thread only)
    std::vector<uint32_t> free_slots;
    std::vector<uint32_t> free_reqs;
    std::vector<Request *> by_slot;
    std::vector<Request *> active;  // admitted, in admission order
    std::deque<Request *> waiting;  // arrived, not admitted (FIFO); their chains: waiting_chains
    uint64_t hbm_fixed = 0;
    uint64_t tick_seq = 0, done_seq = 0;  // last tick queued, last tick completed (ticks complete in order)
    // late admission (server thread only): a tick's duration per wave per SIMD (a running mean of
    // the measured ticks), when the last completed tick was seen to end, and when the next step
    // may start
    double tick_ns_per_wave = 0, late_margin_ns = LATE_MARGIN_START_NS;
    uint64_t tick_end_ns = 0, next_step_ns = 0;
    // shared with submitters / pollers
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    std::vector<Request *> pending;  // not yet arrived: a heap on (arrival, submission order)
    std::vector<uint64_t> cancels;   // ids from lz_server_cancel, applied by the server thread
    std::deque<lz_completion> done;
    uint64_t seq = 0;
    bool stop = false;
    int error = LZ_OK;
    std::thread th;
    lz_server_stats stats{};
};

namespace {

void finish(lz_server *s, Request *r, int32_t status, uint64_t done_ns) {
    lz_completion c{};
    c.id = r->id;
    c.status = status;
    c.arrival_ns = r->arrival_ns;
    c.admit_ns = r->admit_ns;
    c.done_ns = done_ns;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->done.push_back(c);
        s->stats.completed++;
    }
    s->cv_done.notify_all();
    delete r;
}

// Admits waiting requests in FIFO order while slots, memory and staging room allow.
void admit(lz_server *s, std::vector<Request *> &admitted) {
    const uint32_t B = s->ctx->prm.block_len;
    uint64_t staged_chains = 0, staged_pieces = 0;
    while (!s->waiting.empty() && admitted.size() < s->max_new) {
        Request *r = s->waiting.front();
        const uint64_t nb64 = chains_of(*r, B);
        const uint64_t bytes = ((in_len(*r) + 255) / 256 + (out_len(*r) + 255) / 256) * 256;
        if (nb64 > s->max_chains || bytes > s->arena.size()) {  // can never fit
            s->waiting.pop_front();
            s->waiting_chains -= nb64;
            finish(s, r, LZ_E_NOMEM, lz_now_ns());
            continue;
        }
        const uint32_t nb = (uint32_t)nb64;
        const uint64_t np = r->src_dev ? pieces_of(in_len(*r)) : 0;
        if (s->free_reqs.empty() || s->free_slots.size() < nb || staged_chains + nb > s->max_chains ||
            staged_pieces + np > PIECES_MAX)
            break;
        uint64_t off;
        if (!s->arena.alloc(bytes, off)) break;
        s->waiting.pop_front();
        s->waiting_chains -= nb64;
        r->slots.assign(s->free_slots.end() - nb, s->free_slots.end());
        s->free_slots.resize(s->free_slots.size() - nb);
        staged_chains += nb;
        staged_pieces += np;
        r->nb = nb;
        r->arena_off = off;
        r->arena_bytes = bytes;
        r->req_slot = s->free_reqs.back();
        s->free_reqs.pop_back();
        s->by_slot[r->req_slot] = r;
        r->admit_ns = lz_now_ns();
        const uint32_t T = s->cfg.tick_bytes;
        const uint64_t tail = r->n == 0 ? 0 : r->n - (uint64_t)(nb - 1) * B;
        r->ticks_full = nb > 1 ? (uint32_t)((B + (uint64_t)T - 1) / T) : 0;
        r->ticks_tail = tail == 0 ? 1 : (uint32_t)((tail + T - 1) / T);
        r->ticks_run = 0;
        admitted.push_back(r);
    }
    const uint64_t inuse = s->arena.used() + s->hbm_fixed;
    std::lock_guard<std::mutex> g(s->mu);  // stats are read by lz_server_stats_get on other threads
    s->stats.admitted += admitted.size();
    if (inuse > s->stats.peak_hbm) s->stats.peak_hbm = inuse;
}

uint8_t *req_in(lz_server *s, const Request *r) { return s->arena_mem + r->arena_off; }
uint8_t *req_out(lz_server *s, const Request *r) { return req_in(s, r) + (in_len(*r) + 255) / 256 * 256; }

void release(lz_server *s, Request *r);
void compact_active(lz_server *s);

// Reads a finished tick's completions, zeroes failed decryptions, copies the
// outputs out, frees the requests' slots and memory and reports them.
int complete_tick(lz_server *s, TickSlot &t) {
    hipStream_t cs = s->copy_stream;
    LZ_HIP(hipEventSynchronize(t.ev_end));
    s->tick_end_ns = lz_now_ns();
    float ms = 0;
    const bool timed = hipEventElapsedTime(&ms, t.ev_start, t.ev_end) == hipSuccess;
    if (timed && t.waves) {
        const double per = (double)ms * 1e6 / t.waves;
        s->tick_ns_per_wave = s->tick_ns_per_wave > 0 ? 0.75 * s->tick_ns_per_wave + 0.25 * per : per;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);  // stats are read by lz_server_stats_get on other threads
        if (timed) s->stats.busy_ms += ms;
        s->stats.ticks++;
        s->stats.chain_bytes += t.bytes;
    }
    t.in_flight = false;
    s->done_seq = t.seq;
    LZ_HIP(hipMemcpyAsync(t.h_done, t.d_done, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, cs));
    LZ_HIP(hipStreamSynchronize(cs));
    const uint32_t nd = t.h_done[0];
    if (nd == 0) return LZ_OK;
    LZ_HIP(hipMemcpyAsync(t.h_done + 2, t.d_done + 2, nd * sizeof(uint32_t), hipMemcpyDeviceToHost, cs));
    LZ_HIP(hipStreamSynchronize(cs));
    uint32_t nz = 0;
    for (uint32_t i = 0; i < nd; ++i)
        if (t.h_done[2 + i] & 1u) s->h_zero_ids[nz++] = t.h_done[2 + i] >> 1;
    if (nz) {
        LZ_HIP(hipMemcpyAsync(s->d_zero_ids, s->h_zero_ids, nz * sizeof(uint32_t), hipMemcpyHostToDevice, cs));
        LZ_HIP(launch_req_zero(s->reqs, s->d_zero_ids, nz, cs));
    }
    std::vector<std::pair<Request *, int32_t>> fin;
    fin.reserve(nd);
    uint32_t n_out = 0;
    auto flush_out = [&]() -> int {  // one launch for the staged device-to-device output copies
        if (!n_out) return LZ_OK;
        LZ_HIP(hipMemcpyAsync(s->d_out, s->h_out, n_out * sizeof(CopyPiece), hipMemcpyHostToDevice, cs));
        LZ_HIP(launch_copy_many(s->d_out, n_out, cs));
        LZ_HIP(hipStreamSynchronize(cs));  // the staging array is reused
        n_out = 0;
        return LZ_OK;
    };
    for (uint32_t i = 0; i < nd; ++i) {
        Request *r = s->by_slot[t.h_done[2 + i] >> 1];
        if (!r) return fail(LZ_E_HIP, "server: completion for an empty request slot");
        const int32_t status = (t.h_done[2 + i] & 1u) ? LZ_E_INTEGRITY : LZ_OK;
        const uint64_t len = out_len(*r);
        if (len && r->dst_dev) {
            if (n_out + pieces_of(len) > PIECES_MAX)
                if (int rc = flush_out()) return rc;
            add_copy_pieces(s->h_out, n_out, req_out(s, r), r->dst, len);
        } else if (len) {
            LZ_HIP(hipMemcpyAsync(r->dst, req_out(s, r), len, hipMemcpyDefault, cs));
        }
        fin.emplace_back(r, status);
    }
    if (int rc = flush_out()) return rc;
    LZ_HIP(hipStreamSynchronize(cs));
    const uint64_t now = lz_now_ns();
    for (auto &f : fin) release(s, f.first);
    compact_active(s);
    for (auto &f : fin) finish(s, f.first, f.second, now);
    return LZ_OK;
}

// Frees an admitted request's chain slots, request slot and memory (its chains are in
// no tick still in flight) and marks it for compact_active.
void release(lz_server *s, Request *r) {
    s->arena.release(r->arena_off, r->arena_bytes);
    s->free_slots.insert(s->free_slots.end(), r->slots.begin(), r->slots.end());
    s->free_reqs.push_back(r->req_slot);
    s->by_slot[r->req_slot] = nullptr;
    r->released = true;
}

// Takes the released requests off the active list, keeping the admission order.
void compact_active(lz_server *s) {
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(), [](const Request *r) { return r->released; }),
                    s->active.end());
}

// Applies the cancellations queued by lz_server_cancel: a request not yet admitted
// (waiting, or not arrived yet) completes as cancelled now; an active one gets no
// further ticks and is released by release_cancelled.  Ids that match nothing
// (already completed, or unknown) are dropped.
void apply_cancels(lz_server *s) {
    std::vector<uint64_t> ids;
    {
        std::lock_guard<std::mutex> g(s->mu);
        ids.swap(s->cancels);
    }
    for (uint64_t id : ids) {
        auto w = std::find_if(s->waiting.begin(), s->waiting.end(), [&](Request *r) { return r->id == id; });
        if (w != s->waiting.end()) {
            Request *r = *w;
            s->waiting.erase(w);
            s->waiting_chains -= chains_of(*r, s->ctx->prm.block_len);
            finish(s, r, LZ_E_CANCELLED, lz_now_ns());
            continue;
        }
        auto a = std::find_if(s->active.begin(), s->active.end(),
                              [&](Request *r) { return r->id == id && !r->cancelled; });
        if (a != s->active.end()) {
            (*a)->cancelled = true;
            continue;
        }
        Request *early = nullptr;  // not arrived yet: leaves the arrival heap and completes now
        {
            std::lock_guard<std::mutex> g(s->mu);
            auto p = std::find_if(s->pending.begin(), s->pending.end(), [&](Request *r) { return r->id == id; });
            if (p != s->pending.end()) {
                early = *p;
                s->pending.erase(p);
                std::make_heap(s->pending.begin(), s->pending.end(), ArrivalLater());
            }
        }
        if (early) finish(s, early, LZ_E_CANCELLED, lz_now_ns());
    }
}

// Completes the cancelled active requests whose last tick has completed.
void release_cancelled(lz_server *s) {
    const uint64_t now = lz_now_ns();
    std::vector<Request *> gone;
    for (Request *r : s->active) {
        if (!r->cancelled || r->last_tick > s->done_seq) continue;
        release(s, r);
        gone.push_back(r);
    }
    if (gone.empty()) return;
    compact_active(s);
    for (Request *r : gone) finish(s, r, LZ_E_CANCELLED, now);
}

// One scheduling step: admit into the free tick slot, queue its tick, then
// process the other slot's (previous) tick while the new one runs.
int server_step(lz_server *s) {
    hipStream_t st = s->stream;
    // everything a tick needs before it runs (input copies, request records, chain list,
    // counter reset) goes on the staging stream, overlapping the tick that is running now
    hipStream_t pre = s->in_stream;
    TickSlot &t = s->ts[s->cur];
    if (t.in_flight)
        if (int rc = complete_tick(s, t)) return rc;
    // before this slot's events are recorded again: did the running tick, queued late, start
    // right after this slot's tick ended?  (both events have completed by now)
    const TickSlot &run = s->ts[s->cur ^ 1];
    if (run.in_flight && run.late && t.seq + 1 == run.seq && hipEventQuery(run.ev_start) == hipSuccess) {
        float gap_ms = 0;
        if (hipEventElapsedTime(&gap_ms, t.ev_end, run.ev_start) == hipSuccess)
            s->late_margin_ns = gap_ms * 1e6 > LATE_GAP_NS
                                    ? std::min(s->late_margin_ns + LATE_STEP_UP_NS, LATE_MARGIN_MAX_NS)
                                    : std::max(s->late_margin_ns - LATE_STEP_DOWN_NS, LATE_MARGIN_MIN_NS);
    }
    apply_cancels(s);
    std::vector<Request *> admitted;
    admit(s, admitted);
    if (!admitted.empty()) {
        const size_t k = admitted.size();
        uint32_t n_idx = 0, n_in = 0;
        for (size_t i = 0; i < k; ++i) {
            Request *r = admitted[i];
            ReqDesc &d = t.h_req[i];
            std::memset(&d, 0, sizeof d);
            for (int j = 0; j < 3; ++j) {
                d.m.ap[j] = r->key.a_prime[j];
                d.m.r0[j] = r->key.r0[j];
                d.m.mu[j] = r->key.mu[j];
                d.m.om[j] = r->key.omega[j];
                d.m.k[j] = r->key.k[j];
            }
            d.m.decrypt = (uint8_t)r->decrypt;
            d.m.nb = r->nb;
            d.m.n = r->n;
            d.m.in = req_in(s, r);
            d.m.out = req_out(s, r);
            d.remaining = r->nb;
            d.status = LZ_OK;
            d.stored_tag = req_in(s, r) + r->n;
            t.h_meta[3 * i] = r->req_slot;
            t.h_meta[3 * i + 1] = r->nb;
            t.h_meta[3 * i + 2] = n_idx;
            std::memcpy(t.h_idx + n_idx, r->slots.data(), r->nb * sizeof(uint32_t));
            n_idx += r->nb;
            if (in_len(*r) && r->src_dev) add_copy_pieces(t.h_in, n_in, r->src, req_in(s, r), in_len(*r));
            else if (in_len(*r)) LZ_HIP(hipMemcpyAsync(req_in(s, r), r->src, in_len(*r), hipMemcpyDefault, pre));
            s->active.push_back(r);
        }
        if (n_in) {
            LZ_HIP(hipMemcpyAsync(t.d_in, t.h_in, n_in * sizeof(CopyPiece), hipMemcpyHostToDevice, pre));
            LZ_HIP(launch_copy_many(t.d_in, n_in, pre));
        }
        LZ_HIP(hipMemcpyAsync(t.d_req, t.h_req, k * sizeof(ReqDesc), hipMemcpyHostToDevice, pre));
        LZ_HIP(hipMemcpyAsync(t.d_meta, t.h_meta, 3 * k * sizeof(uint32_t), hipMemcpyHostToDevice, pre));
        LZ_HIP(hipMemcpyAsync(t.d_idx, t.h_idx, n_idx * sizeof(uint32_t), hipMemcpyHostToDevice, pre));
        LZ_HIP(launch_install(s->reqs, s->slots, t.d_req, t.d_meta, t.d_idx, (uint32_t)k, s->ctx->prm.block_len, pre));
    }
    // the chains that still have bytes to process: each request's full chains until they end,
    // its last chain until it ends (the tick count of each is known at admission)
    const uint32_t T = s->cfg.tick_bytes, B = s->ctx->prm.block_len;
    auto unfinished = [&](const Request *r) -> uint32_t {
        const uint32_t tr = r->ticks_run;
        return (tr < r->ticks_full ? r->nb - 1 : 0) + (tr < r->ticks_tail ? 1 : 0);
    };
    // waves per SIMD of this tick, from the backlog
    uint64_t backlog = s->waiting_chains;
    for (const Request *r : s->active)
        if (!r->cancelled) backlog += unfinished(r);
    uint32_t k = 1;
    while (k < s->cfg.run_waves && backlog > 3 * s->simd_chains * k) k = std::min(2 * k, s->cfg.run_waves);
    const uint64_t cap = s->cfg.policy == LZ_SERVE_ALL_CHAINS ? s->max_chains
                                                                : std::min<uint64_t>(k * s->simd_chains, s->max_chains);
    // requests join in admission order, all their unfinished chains or none, up to the cap; the
    // first request with work always joins, so one larger than the cap still runs
    uint32_t n_list = 0;
    uint64_t tick_bytes = 0;
    const uint64_t seq = s->tick_seq + 1;
    for (Request *r : s->active) {
        if (r->cancelled) continue;
        const uint32_t tr = r->ticks_run;
        const uint32_t want = unfinished(r);
        if (want == 0 || (n_list && (uint64_t)n_list + want > cap)) continue;
        if (tr < r->ticks_full) {
            std::memcpy(t.h_list + n_list, r->slots.data(), (r->nb - 1) * sizeof(uint32_t));
            n_list += r->nb - 1;
            tick_bytes += (uint64_t)(r->nb - 1) * std::min<uint64_t>(T, (uint64_t)B - (uint64_t)tr * T);
        }
        if (tr < r->ticks_tail) {
            t.h_list[n_list++] = r->slots[r->nb - 1];
            const uint64_t tail = r->n - (uint64_t)(r->nb - 1) * B;
            const uint64_t done = (uint64_t)tr * T;
            tick_bytes += tail > done ? std::min<uint64_t>(T, tail - done) : 0;
        }
        if (tr < r->ticks_full || tr < r->ticks_tail) {
            r->ticks_run++;
            r->last_tick = seq;
        }
    }
    if (n_list) {
        LZ_HIP(hipMemcpyAsync(t.d_list, t.h_list, n_list * sizeof(uint32_t), hipMemcpyHostToDevice, pre));
        LZ_HIP(launch_fill_u64(reinterpret_cast<unsigned long long *>(t.d_done), 1, pre));
        LZ_HIP(hipEventRecord(s->ev_in, pre));
        LZ_HIP(hipStreamWaitEvent(st, s->ev_in, 0));
        TickDev td;
        td.slots = s->slots;
        td.reqs = s->reqs;
        td.list = t.d_list;
        td.n_list = n_list;
        td.tick_bytes = T;
        td.done_count = t.d_done;
        td.done_queue = t.d_done + 2;
        LZ_HIP(hipEventRecord(t.ev_start, st));
        LZ_HIP(launch_tick(s->shape, s->ctx->prm, td, st));
        LZ_HIP(hipEventRecord(t.ev_end, st));
        t.bytes = tick_bytes;
        t.seq = seq;
        t.waves = (uint32_t)((n_list + s->simd_chains - 1) / s->simd_chains);
        t.late = s->ts[s->cur ^ 1].in_flight;
        s->tick_seq = seq;
        t.in_flight = true;
    }
    s->cur ^= 1;
    TickSlot &prev = s->ts[s->cur];
    s->next_step_ns = 0;
    if (prev.in_flight) {
        if (int rc = complete_tick(s, prev)) return rc;
        // the tick queued above started when the previous one ended: the next step waits until
        // shortly before it is expected to end, so that the tick after it takes the requests
        // that arrive meanwhile (and not one tick later)
        const double est = s->tick_ns_per_wave * t.waves;
        if (t.in_flight && est > s->late_margin_ns)
            s->next_step_ns = s->tick_end_ns + (uint64_t)(est - s->late_margin_ns);
    }
    release_cancelled(s);
    if (!n_list && !prev.in_flight && !s->ts[s->cur ^ 1].in_flight && !s->active.empty())
        return fail(LZ_E_HIP, "server: active requests without pending work");
    return LZ_OK;
}

bool busy(lz_server *s) { return !s->waiting.empty() || !s->active.empty() || s->ts[0].in_flight || s->ts[1].in_flight; }

void server_loop(lz_server *s) {
    hipSetDevice(s->ctx->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            for (uint64_t now = lz_now_ns(); now < s->next_step_ns && !s->stop; now = lz_now_ns())
                s->cv_submit.wait_for(g, std::chrono::nanoseconds(s->next_step_ns - now));
            for (;;) {
                const uint64_t now = lz_now_ns();
                while (!s->pending.empty() && s->pending.front()->arrival_ns <= now) {
                    std::pop_heap(s->pending.begin(), s->pending.end(), ArrivalLater());
                    s->waiting.push_back(s->pending.back());
                    s->waiting_chains += chains_of(*s->waiting.back(), s->ctx->prm.block_len);
                    s->pending.pop_back();
                }
                if (busy(s) || !s->cancels.empty()) break;
                if (s->stop && s->pending.empty()) return;
                if (s->pending.empty()) {
                    s->cv_submit.wait(g);
                } else {
                    const uint64_t dt = s->pending.front()->arrival_ns - now;
                    s->cv_submit.wait_for(g, std::chrono::nanoseconds(dt));
                }
            }
        }
        if (!busy(s)) {  // only cancellations to apply
            apply_cancels(s);
            continue;
        }
        if (int rc = server_step(s)) {
            std::lock_guard<std::mutex> g(s->mu);
            s->error = rc;
            s->stop = true;
            s->cv_done.notify_all();
            return;
        }
    }
}

void server_free(lz_server *s) {
    if (!s) return;
    hipSetDevice(s->ctx->device);
    if (s->stream) hipStreamSynchronize(s->stream);
    if (s->in_stream) hipStreamSynchronize(s->in_stream);
    if (s->copy_stream) hipStreamSynchronize(s->copy_stream);
    hipFree(s->arena_mem);
    hipFree(s->slots);
    hipFree(s->reqs);
    hipFree(s->d_zero_ids);
    hipHostFree(s->h_zero_ids);
    hipFree(s->d_out);
    hipHostFree(s->h_out);
    for (TickSlot &t : s->ts) {
        hipFree(t.d_list);
        hipFree(t.d_done);
        hipFree(t.d_req);
        hipFree(t.d_meta);
        hipFree(t.d_idx);
        hipFree(t.d_in);
        hipHostFree(t.h_in);
        hipHostFree(t.h_list);
        hipHostFree(t.h_done);
        hipHostFree(t.h_req);
        hipHostFree(t.h_meta);
        hipHostFree(t.h_idx);
        if (t.ev_start) hipEventDestroy(t.ev_start);
        if (t.ev_end) hipEventDestroy(t.ev_end);
    }
    if (s->stream) hipStreamDestroy(s->stream);
    if (s->in_stream) hipStreamDestroy(s->in_stream);
    if (s->copy_stream) hipStreamDestroy(s->copy_stream);
    if (s->ev_in) hipEventDestroy(s->ev_in);
    for (Request *r : s->pending) delete r;
    for (Request *r : s->waiting) delete r;
    for (Request *r : s->active) delete r;
    delete s;
}

}  // namespace

extern "C" int lz_server_create(lz_ctx *c, const lz_server_config *cfg, lz_server **out) {
    if (!out) return fail(LZ_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!c || !cfg) return fail(LZ_E_INVAL, "NULL argument");
    LZ_HIP(hipSetDevice(c->device));
    lz_server *s = new (std::nothrow) lz_server();
    if (!s) return fail(LZ_E_NOMEM, "host allocation failed");
    s->ctx = c;
    s->cfg = *cfg;
    if (s->cfg.tick_bytes == 0) s->cfg.tick_bytes = 16;
    if (s->cfg.tick_bytes > (1u << 20)) {
        delete s;
        return fail(LZ_E_INVAL, "tick_bytes must be <= 2^20");
    }
    if (s->cfg.run_waves > 8 || s->cfg.policy > LZ_SERVE_ALL_CHAINS) {
        delete s;
        return fail(LZ_E_INVAL, "run_waves must be <= 8 and policy LZ_SERVE_ADAPTIVE or LZ_SERVE_ALL_CHAINS");
    }
    if (s->cfg.run_waves == 0) s->cfg.run_waves = 4;
    s->simd_chains = (uint64_t)c->dev.cus * 4 * WAVE_LANES;
    // admitted chains: adaptive, twice the largest tick, so that a tick can be filled from requests
    // behind a large one; all chains, the largest tick
    const uint64_t def_chains = (s->cfg.policy == LZ_SERVE_ALL_CHAINS ? 1 : 2) * s->cfg.run_waves * s->simd_chains;
    s->max_chains = cfg->max_chains ? cfg->max_chains : (uint32_t)def_chains;
    s->max_reqs = s->max_chains;
    s->max_new = std::min<uint32_t>(s->max_reqs, 2048);  // admissions per tick (staging size)
    int tile = 16;
    while (tile < (int)s->cfg.tick_bytes && tile < 128) tile *= 2;
    s->shape = KernelShape{1, 256, tile, 4};
    if (!shape_valid(s->shape, c->dev)) s->shape = KernelShape{1, 64, 16, 4};

    // fixed device memory: chain slots, request records, and per tick slot the list, the
    // completion queue and the staging of admitted requests
    const uint64_t per_tick = (uint64_t)s->max_chains * 4 * 2 + ((uint64_t)s->max_reqs + 2) * 4 +
                              (uint64_t)s->max_new * (sizeof(ReqDesc) + 12) + PIECES_MAX * sizeof(CopyPiece);
    const uint64_t fixed = (uint64_t)s->max_chains * sizeof(ChainSlot) + (uint64_t)s->max_reqs * sizeof(ReqDesc) +
                           (uint64_t)s->max_reqs * 4 + 2 * per_tick + PIECES_MAX * sizeof(CopyPiece) + (1u << 20);
    if (cfg->hbm_budget <= fixed + 4096) {
        delete s;
        return fail(LZ_E_INVAL, "hbm_budget too small for the chain slots");
    }
    s->hbm_fixed = fixed;
    const uint64_t arena_bytes = cfg->hbm_budget - fixed;
    hipError_t e = hipMalloc(&s->arena_mem, arena_bytes);
    if (e == hipSuccess) e = hipMalloc(&s->slots, (size_t)s->max_chains * sizeof(ChainSlot));
    if (e == hipSuccess) e = hipMalloc(&s->reqs, (size_t)s->max_reqs * sizeof(ReqDesc));
    if (e == hipSuccess) e = hipMalloc(&s->d_zero_ids, (size_t)s->max_reqs * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc(&s->h_zero_ids, (size_t)s->max_reqs * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&s->d_out, PIECES_MAX * sizeof(CopyPiece));
    if (e == hipSuccess) e = hipHostMalloc(&s->h_out, PIECES_MAX * sizeof(CopyPiece), hipHostMallocDefault);
    for (TickSlot &t : s->ts) {
        if (e == hipSuccess) e = hipMalloc(&t.d_list, (size_t)s->max_chains * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&t.d_done, ((size_t)s->max_reqs + 2) * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&t.d_req, (size_t)s->max_new * sizeof(ReqDesc));
        if (e == hipSuccess) e = hipMalloc(&t.d_meta, 3 * (size_t)s->max_new * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&t.d_idx, (size_t)s->max_chains * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&t.d_in, PIECES_MAX * sizeof(CopyPiece));
        if (e == hipSuccess) e = hipHostMalloc(&t.h_in, PIECES_MAX * sizeof(CopyPiece), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&t.h_list, (size_t)s->max_chains * sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(&t.h_done, ((size_t)s->max_reqs + 2) * sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&t.h_req, (size_t)s->max_new * sizeof(ReqDesc), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(&t.h_meta, 3 * (size_t)s->max_new * sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&t.h_idx, (size_t)s->max_chains * sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreate(&t.ev_start);
        if (e == hipSuccess) e = hipEventCreate(&t.ev_end);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->in_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "server allocation");
        server_free(s);
        return rc;
    }
    s->arena.reset(arena_bytes);
    s->free_slots.resize(s->max_chains);
    for (uint32_t i = 0; i < s->max_chains; ++i) s->free_slots[i] = s->max_chains - 1 - i;
    s->free_reqs.resize(s->max_reqs);
    for (uint32_t i = 0; i < s->max_reqs; ++i) s->free_reqs[i] = s->max_reqs - 1 - i;
    s->by_slot.assign(s->max_reqs, nullptr);
    s->th = std::thread(server_loop, s);
    *out = s;
    return LZ_OK;
}

extern "C" int lz_server_submit(lz_server *s, uint64_t id, int decrypt, const uint8_t *pw, size_t n_pw,
                                const void *src, uint64_t n, void *dst, uint64_t arrival_ns) {
    if (!s || !pw) return fail(LZ_E_INVAL, "NULL argument");
    if (int rc = check_blocks(s->ctx->prm, n, nullptr)) return rc;
    const uint64_t nin = decrypt ? n + LZ_TAG_BYTES : n, nout = decrypt ? n : n + LZ_TAG_BYTES;
    if ((nin && !src) || (nout && !dst)) return fail(LZ_E_INVAL, "NULL buffer");
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(LZ_E_NOMEM, "host allocation failed");
    if (int rc = lz_key_setup(pw, n_pw, &s->ctx->prm, &r->key)) {
        delete r;
        return rc;
    }
    r->id = id;
    r->decrypt = decrypt ? 1 : 0;
    r->src = src;
    r->dst = dst;
    r->n = n;
    classify(r);
    r->arrival_ns = arrival_ns ? arrival_ns : lz_now_ns();
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            delete r;
            return fail(s->error ? s->error : LZ_E_INVAL, "server stopped");
        }
        r->seq = s->seq++;
        s->pending.push_back(r);
        std::push_heap(s->pending.begin(), s->pending.end(), ArrivalLater());
    }
    s->cv_submit.notify_all();
    return LZ_OK;
}

extern "C" int lz_server_submit_many(lz_server *s, size_t count, const uint64_t *ids, const uint8_t *decrypt,
                                     const uint8_t *pw, const uint64_t *pw_off, const uint32_t *pw_len,
                                     const void *const *src, const uint64_t *n, void *const *dst,
                                     const uint64_t *arrival_ns) {
    if (!s || (count && (!ids || !decrypt || !pw || !pw_off || !pw_len || !src || !n || !dst || !arrival_ns)))
        return fail(LZ_E_INVAL, "NULL argument");
    std::vector<Request *> batch;
    batch.reserve(count);
    auto drop = [&] {
        for (Request *r : batch) delete r;
    };
    const uint64_t now = lz_now_ns();
    for (size_t i = 0; i < count; ++i) {
        const int dec = decrypt[i] ? 1 : 0;
        if (int rc = check_blocks(s->ctx->prm, n[i], nullptr)) {
            drop();
            return rc;
        }
        const uint64_t nin = dec ? n[i] + LZ_TAG_BYTES : n[i], nout = dec ? n[i] : n[i] + LZ_TAG_BYTES;
        if ((nin && !src[i]) || (nout && !dst[i])) {
            drop();
            return fail(LZ_E_INVAL, "NULL buffer");
        }
        Request *r = new (std::nothrow) Request();
        if (!r) {
            drop();
            return fail(LZ_E_NOMEM, "host allocation failed");
        }
        batch.push_back(r);
        if (int rc = lz_key_setup(pw + pw_off[i], pw_len[i], &s->ctx->prm, &r->key)) {
            drop();
            return rc;
        }
        r->id = ids[i];
        r->decrypt = dec;
        r->src = src[i];
        r->dst = dst[i];
        r->n = n[i];
        classify(r);
        r->arrival_ns = arrival_ns[i] ? arrival_ns[i] : now;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) {
            drop();
            return fail(s->error ? s->error : LZ_E_INVAL, "server stopped");
        }
        for (Request *r : batch) {
            r->seq = s->seq++;
            s->pending.push_back(r);
            std::push_heap(s->pending.begin(), s->pending.end(), ArrivalLater());
        }
    }
    s->cv_submit.notify_all();
    return LZ_OK;
}

extern "C" int lz_server_cancel(lz_server *s, uint64_t id) {
    if (!s) return fail(LZ_E_INVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return fail(s->error ? s->error : LZ_E_INVAL, "server stopped");
        s->cancels.push_back(id);
    }
    s->cv_submit.notify_all();
    return LZ_OK;
}

extern "C" int lz_server_poll(lz_server *s, lz_completion *out, int max, int timeout_ms) {
    if (!s || (!out && max > 0) || max < 0) return fail(LZ_E_INVAL, "bad argument");
    std::unique_lock<std::mutex> g(s->mu);
    auto ready = [&] { return !s->done.empty() || s->error; };
    if (timeout_ms < 0) s->cv_done.wait(g, ready);
    else if (timeout_ms > 0) s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), ready);
    if (s->error && s->done.empty()) return fail(s->error, "server loop failed");
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    return k;
}

extern "C" int lz_server_stats_get(lz_server *s, lz_server_stats *out) {
    if (!s || !out) return fail(LZ_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    return LZ_OK;
}

extern "C" int lz_server_destroy(lz_server *s) {
    if (!s) return LZ_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_submit.notify_all();
    if (s->th.joinable()) s->th.join();
    const int err = s->error;
    server_free(s);
    return err;
}
