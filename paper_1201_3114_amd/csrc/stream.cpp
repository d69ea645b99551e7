// Streaming (resumable) encryption and decryption of one message whose length
// is not known in advance.  The message is the concatenation of the update
// chunks; the output and the final tag equal those of the one-shot path.
// Each chunk is cut at block boundaries of the parallel version (Section 5):
// the pending partial block continues from its device-resident checkpoint
// (r, alpha, mu, Omega), the full blocks run as one plain launch at the right
// block index, and the remainder starts the next partial block.  All three run
// in one launch on the caller's stream, the two partial blocks (one chain each,
// as slow as a whole block) as the lanes after the full blocks: they are
// independent of the full blocks and of each other, since the new partial block
// keeps its checkpoint in a second slot.
//
// A deferred update copies its chunk into the stream's staging buffer instead
// and remembers where its output goes; a flush (explicit, when the buffer is
// full, before an immediate update or at the end) runs the staged bytes as one
// update and copies each chunk's output out.  Small chunks then share a launch
// that fills the device, and the result is that of one update over their
// concatenation.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace lz;

struct lz_stream {
    lz_ctx *ctx;
    int decrypt;
    lz_key key;
    uint64_t pos;        // bytes consumed so far
    bool finished;
    void *dmem;          // two ChainSlots, then 3 tag words (+1 pad), then the status word
    ChainSlot *slot[2];  // slot[cur] holds the pending partial block's checkpoint
    int cur;
    unsigned long long *tag;
    int32_t *status;
    int32_t *h_status;   // pinned
    hipEvent_t ev;
    hipStream_t last;
    bool has_last;
    // deferred updates: staged input and output (LZ_STREAM_DEFER_BYTES each, on first use)
    struct Deferred {
        uint8_t *out;
        uint64_t off, n;
    };
    uint8_t *stage;      // input, then output
    uint64_t fill;       // staged bytes
    std::vector<Deferred> segs;
    std::vector<CopyPiece> pieces;  // the staged chunks' output copies, built at a flush
};

namespace {

void stream_free(lz_stream *st) {
    if (!st) return;
    hipSetDevice(st->ctx->device);
    if (st->has_last) hipEventSynchronize(st->ev);
    if (st->dmem) hipFree(st->dmem);
    if (st->stage) hipFree(st->stage);
    if (st->h_status) hipHostFree(st->h_status);
    if (st->ev) hipEventDestroy(st->ev);
    delete st;
}

int stream_order(lz_stream *st, hipStream_t s) {
    if (st->has_last && st->last != s) LZ_HIP(hipStreamWaitEvent(s, st->ev, 0));
    return LZ_OK;
}

int stream_record(lz_stream *st, hipStream_t s) {
    LZ_HIP(hipEventRecord(st->ev, s));
    st->last = s;
    st->has_last = true;
    return LZ_OK;
}

}  // namespace

extern "C" int lz_stream_open(lz_ctx *c, int decrypt, const uint8_t *pw, size_t n_pw, lz_stream **out) {
    if (!out) return fail(LZ_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!c || !pw) return fail(LZ_E_INVAL, "NULL argument");
    LZ_HIP(hipSetDevice(c->device));
    lz_stream *st = new (std::nothrow) lz_stream();
    if (!st) return fail(LZ_E_NOMEM, "host allocation failed");
    st->ctx = c;
    st->decrypt = decrypt ? 1 : 0;
    if (int rc = lz_key_setup(pw, n_pw, &c->prm, &st->key)) {
        delete st;
        return rc;
    }
    const size_t bytes = 2 * sizeof(ChainSlot) + 4 * sizeof(unsigned long long) + sizeof(int32_t);
    hipError_t e = hipMalloc(&st->dmem, bytes);
    if (e == hipSuccess) e = hipMemset(st->dmem, 0, bytes);
    if (e == hipSuccess) e = hipHostMalloc(&st->h_status, sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = hip_fail(e, "stream allocation");
        stream_free(st);
        return rc;
    }
    char *base = static_cast<char *>(st->dmem);
    st->slot[0] = reinterpret_cast<ChainSlot *>(base);
    st->slot[1] = reinterpret_cast<ChainSlot *>(base + sizeof(ChainSlot));
    st->cur = 0;
    st->tag = reinterpret_cast<unsigned long long *>(base + 2 * sizeof(ChainSlot));
    st->status = reinterpret_cast<int32_t *>(base + 2 * sizeof(ChainSlot) + 4 * sizeof(unsigned long long));
    *out = st;
    return LZ_OK;
}

namespace {

// One update over n bytes already checked (n > 0), on s, ordered after the stream's last work.
int stream_step(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out, hipStream_t s) {
    lz_ctx *c = st->ctx;
    const uint64_t B = c->prm.block_len;
    const uint64_t r = st->pos % B;
    const uint64_t h = r == 0 ? 0 : (n < B - r ? n : B - r);  // head: finishes the pending partial block
    const uint64_t full = (n - h) / B;                          // body: whole blocks
    const uint64_t rem = n - h - full * B;                      // tail: starts the next partial block
    const uint64_t pos0 = st->pos;
    StreamExtra x{};
    if (h > 0) {  // continues slot[cur]
        x.head_slot = st->slot[st->cur];
        x.head_in = d_in;
        x.head_out = d_out;
        x.head_cnt = (uint32_t)h;
        x.head_complete = r + h == B;
    }
    if (rem > 0) {  // a new chain in the other slot, independent of the head's
        const uint64_t o = h + full * B;
        x.tail_slot = st->slot[st->cur ^ 1];
        x.tail_in = d_in + o;
        x.tail_out = d_out + o;
        x.tail_cnt = (uint32_t)rem;
        x.tail_block = (pos0 + o) / B;
    }
    LZ_HIP(launch_stream_step(c->shape, st->key, c->prm, st->decrypt, d_in + h, d_out + h, full, (pos0 + h) / B, x,
                              st->tag, s));
    if (rem > 0) st->cur ^= 1;
    st->pos = pos0 + n;
    return LZ_OK;
}

// Queued chunks run as soon as their blocks make up a chain per lane of one wave on every SIMD (four
// per CU): such an update already issues at the full rate, and the host queues the next chunks
// while it runs.  One chain more would put a second wave on one SIMD and double the run's time, so
// a run from the stream's position holds at most run_room bytes (its first block may be one that
// an earlier run began), and a chunk that does not fit is split between runs.  At most the
// staging capacity.
uint64_t run_bytes(const lz_stream *st) {
    const uint64_t b = (uint64_t)st->ctx->dev.cus * 4 * WAVE_LANES * st->ctx->prm.block_len;
    return b < LZ_STREAM_DEFER_BYTES ? b : LZ_STREAM_DEFER_BYTES;
}

uint64_t run_room(const lz_stream *st) {
    const uint64_t B = st->ctx->prm.block_len;
    const uint64_t b = (uint64_t)st->ctx->dev.cus * 4 * WAVE_LANES * B - st->pos % B;
    return b < LZ_STREAM_DEFER_BYTES ? b : LZ_STREAM_DEFER_BYTES;
}

// Pieces of the staged chunks' output copies at most: every chunk, plus one per COPY_PIECE_BYTES.
constexpr uint32_t STREAM_PIECES = (uint32_t)(LZ_STREAM_DEFER_BYTES / COPY_PIECE_BYTES) + LZ_STREAM_DEFER_CHUNKS;

// The staging buffer of deferred updates and the host table of their output copies, on first use.
int stream_staging(lz_stream *st) {
    if (st->stage) return LZ_OK;
    try {
        st->pieces.resize(STREAM_PIECES);
    } catch (...) {
        return fail(LZ_E_NOMEM, "host allocation failed");
    }
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, 2 * (size_t)LZ_STREAM_DEFER_BYTES);
    if (e != hipSuccess) return hip_fail(e, "stream staging buffer");
    st->stage = static_cast<uint8_t *>(p);
    return LZ_OK;
}

// Runs the staged chunks as one update, then copies each chunk's output to where it goes: all
// chunks by batched copies whose pieces travel in the kernel arguments.
int stream_flush(lz_stream *st, hipStream_t s) {
    if (st->fill == 0) return LZ_OK;
    uint8_t *in = st->stage, *outb = st->stage + LZ_STREAM_DEFER_BYTES;
    if (int rc = stream_step(st, in, st->fill, outb, s)) return rc;
    uint32_t np = 0;
    for (const lz_stream::Deferred &d : st->segs) add_copy_pieces(st->pieces.data(), np, outb + d.off, d.out, d.n);
    LZ_HIP(launch_copy_pieces_host(st->pieces.data(), np, s));
    st->fill = 0;
    st->segs.clear();
    return LZ_OK;
}

int update_checks(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out) {
    if (!st) return fail(LZ_E_INVAL, "stream is NULL");
    if (st->finished) return fail(LZ_E_INVAL, "stream already finished");
    if (n == 0) return LZ_OK;
    if (!d_in || !d_out) return fail(LZ_E_INVAL, "NULL buffer");
    const uint64_t at = st->pos + st->fill;
    if (n > LZ_MAX_MESSAGE || at + n > LZ_MAX_MESSAGE) return fail(LZ_E_INVAL, "message longer than 2^32 bytes");
    return check_blocks(st->ctx->prm, at + n, nullptr);
}

}  // namespace

extern "C" int lz_stream_update(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out, void *stream) {
    if (int rc = update_checks(st, d_in, n, d_out)) return rc;
    if (n == 0) return LZ_OK;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(st->ctx->device));
    if (int rc = stream_order(st, s)) return rc;
    if (int rc = stream_flush(st, s)) return rc;  // staged chunks come first
    if (int rc = stream_step(st, d_in, n, d_out, s)) return rc;
    return stream_record(st, s);
}

extern "C" int lz_stream_update_deferred(lz_stream *st, const uint8_t *d_in, size_t n, uint8_t *d_out, void *stream) {
    if (int rc = update_checks(st, d_in, n, d_out)) return rc;
    if (n == 0) return LZ_OK;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(st->ctx->device));
    if (int rc = stream_order(st, s)) return rc;
    if (n >= run_bytes(st)) {  // a chunk this large fills the device by itself
        if (int rc = stream_flush(st, s)) return rc;
        if (int rc = stream_step(st, d_in, n, d_out, s)) return rc;
        return stream_record(st, s);
    }
    if (int rc = stream_staging(st)) return rc;
    while (n > 0) {  // fill < run_room here: a full run has been flushed
        if (st->segs.size() >= LZ_STREAM_DEFER_CHUNKS)
            if (int rc = stream_flush(st, s)) return rc;
        const uint64_t room = run_room(st) - st->fill, take = n < room ? n : room;
        LZ_HIP(hipMemcpyAsync(st->stage + st->fill, d_in, take, hipMemcpyDeviceToDevice, s));
        try {
            st->segs.push_back({d_out, st->fill, take});
        } catch (...) {
            return fail(LZ_E_NOMEM, "host allocation failed");
        }
        st->fill += take;
        d_in += take;
        d_out += take;
        n -= take;
        if (st->fill == run_room(st))
            if (int rc = stream_flush(st, s)) return rc;
    }
    return stream_record(st, s);
}

extern "C" int lz_stream_flush(lz_stream *st, void *stream) {
    if (!st) return fail(LZ_E_INVAL, "stream is NULL");
    if (st->finished) return fail(LZ_E_INVAL, "stream already finished");
    if (st->fill == 0) return LZ_OK;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(st->ctx->device));
    if (int rc = stream_order(st, s)) return rc;
    if (int rc = stream_flush(st, s)) return rc;
    return stream_record(st, s);
}

extern "C" int lz_stream_finish(lz_stream *st, uint8_t *d_tag, int32_t *d_status, void *stream) {
    if (!st || !d_tag) return fail(LZ_E_INVAL, "NULL argument");
    if (st->finished) return fail(LZ_E_INVAL, "stream already finished");
    lz_ctx *c = st->ctx;
    hipStream_t s = (hipStream_t)stream;
    LZ_HIP(hipSetDevice(c->device));
    if (int rc = stream_order(st, s)) return rc;
    if (int rc = stream_flush(st, s)) return rc;
    const int pending = st->pos % c->prm.block_len != 0;
    const int empty = st->pos == 0;
    int32_t *status = d_status ? d_status : st->status;
    LZ_HIP(launch_stream_finish(st->slot[st->cur], pending, empty, st->key, st->tag, st->decrypt, d_tag, status, s));
    st->finished = true;
    if (!st->decrypt || d_status) return stream_record(st, s);
    LZ_HIP(hipMemcpyAsync(st->h_status, st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (int rc = stream_record(st, s)) return rc;
    LZ_HIP(hipStreamSynchronize(s));
    if (*st->h_status != LZ_OK) return fail(LZ_E_INTEGRITY, "integrity check failed: stream altered or wrong password");
    return LZ_OK;
}

extern "C" uint64_t lz_stream_position(const lz_stream *st) { return st ? st->pos + st->fill : 0; }

extern "C" int lz_stream_close(lz_stream *st) {
    stream_free(st);
    return LZ_OK;
}
