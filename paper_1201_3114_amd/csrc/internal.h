// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/lorenz_cipher.h"

namespace lz {

// ---- errors -------------------------------------------------------------------
void set_error(const char *msg);
int fail(int code, const char *msg);
int hip_fail(hipError_t e, const char *what);
#define LZ_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::lz::hip_fail(e_, #call); \
    } while (0)

// ---- host key setup (keysetup.cpp) ---------------------------------------------
void sha256(const uint8_t *msg, size_t len, uint8_t out[32]);
int key_setup(const uint8_t *pw, size_t n, const lz_params &prm, lz_key &key);
int check_params(const lz_params &prm);
// n <= 2^32 and at most LZ_MAX_BLOCKS blocks of prm.block_len; *nb (may be NULL) = block count
int check_blocks(const lz_params &prm, uint64_t n, uint64_t *nb);

// ---- device-side descriptors -----------------------------------------------------

// Per-message descriptor of the batched and served paths (device memory).
struct MsgDesc {
    double ap[3];        // a'
    double r0[3];        // r0
    uint8_t mu[3], om[3], k[3], decrypt;
    uint32_t nb;         // blocks (chains) of this message, >= 1
    const uint8_t *in;   // message body in
    uint8_t *out;        // message body out
    uint64_t n;          // body length in bytes
};

// Resumable state of one chain (served path), an exact checkpoint.
struct ChainSlot {
    double r[3];
    double al[3];
    uint8_t mu[3], om[3];
    uint8_t fresh;       // 1: state not yet initialised from the key
    uint8_t pad;
    uint32_t pos;        // bytes of this block already processed
    uint32_t len;        // bytes of this block
    uint32_t req;        // request slot
    uint32_t blk;        // block index within the request
    uint32_t pad2;
};

// The two partial-block chains of a stream update, carried by a plain launch as the
// lanes after its nb whole blocks: the head finishes the pending partial block from
// its checkpoint (its digest joins the tag when it completes the block, else the
// checkpoint is saved back), the tail starts the next partial block and saves its
// checkpoint.  Running them in the same launch keeps them from adding a wave to a
// SIMD that already runs whole-block waves, which would make that SIMD, and so the
// launch, take longer.
struct StreamExtra {
    ChainSlot *head_slot;  // null: no head chain
    const uint8_t *head_in;
    uint8_t *head_out;
    uint32_t head_cnt, head_complete;
    ChainSlot *tail_slot;  // null: no tail chain
    const uint8_t *tail_in;
    uint8_t *tail_out;
    uint32_t tail_cnt;
    uint64_t tail_block;
};

// Per-request record of the served path (device memory).
struct ReqDesc {
    MsgDesc m;
    unsigned long long tag[3];  // XOR accumulator of block digests
    uint32_t remaining;         // chains not yet finished
    int32_t status;
    const uint8_t *stored_tag;  // decrypt: the 24 tag bytes of the input
};

struct KernelShape {
    int m;         // chains per lane
    int wg;        // threads per workgroup
    int tile;      // LDS bytes per chain per refill
    int wps;       // resident waves per SIMD (persistent kernel)
};

struct DevInfo {
    int cus;
    int lds_per_wg_max;
};

constexpr int WAVE_LANES = 64;  // lanes of a gfx950 wavefront

// ---- kernel launchers (kernels.hip) --------------------------------------------------
hipError_t launch_fill_u64(unsigned long long *p, size_t n, hipStream_t s);
hipError_t launch_plain(const KernelShape &sh, const lz_key &key, const lz_params &prm, int decrypt,
                        const uint8_t *in, uint8_t *out, uint64_t n, unsigned long long *tag_acc,
                        hipStream_t s, uint64_t block_base = 0);
// One stream update: its full whole blocks from in / out at global block index
// block_base, plus x's head and tail chains, in one launch of one chain per lane.
hipError_t launch_stream_step(const KernelShape &shape, const lz_key &key, const lz_params &prm, int decrypt,
                              const uint8_t *in, uint8_t *out, uint64_t full, uint64_t block_base,
                              const StreamExtra &x, unsigned long long *tag_acc, hipStream_t s);
hipError_t launch_plain_finalize(int decrypt, const unsigned long long *tag_acc, const uint8_t *stored_tag,
                                 uint8_t *tag_out, int32_t *status, uint8_t *body, uint64_t n,
                                 hipStream_t s);
// Batched persistent kernel.  full_prefix[i] = number of full blocks of messages [0, i);
// tail_msg: messages with a partial (or empty) last block, longest first.
struct BatchDev {
    const MsgDesc *msgs;
    const uint64_t *full_prefix;  // n_msg + 1 entries
    const uint32_t *tail_msg;     // n_tail entries
    uint32_t n_msg;
    uint32_t n_tail;
    uint64_t n_full;              // total full blocks
    uint64_t n_tasks;
    unsigned long long *tag_acc;  // 3 per message
    unsigned long long *counter;  // work-queue head
    int32_t *const *status_ref;   // decrypt: device slot holding the address of the per-message statuses
};
hipError_t launch_batch(const KernelShape &sh, const DevInfo &dev, const lz_params &prm, const BatchDev &b,
                        hipStream_t s);
hipError_t launch_batch_finalize(const BatchDev &b, int decrypt, hipStream_t s);
// One-thread kernel: *slot = status (ordered on s before a batch replay that reads the slot).
hipError_t launch_set_status_ref(int32_t **slot, int32_t *status, hipStream_t s);

// Served path: advance the listed chains by up to tick_bytes bytes each.
struct TickDev {
    ChainSlot *slots;
    ReqDesc *reqs;
    const uint32_t *list;         // active chain slot indices
    uint32_t n_list;
    uint32_t tick_bytes;
    uint32_t *done_queue;         // request slots completed in this tick
    uint32_t *done_count;
};
hipError_t launch_tick(const KernelShape &sh, const lz_params &prm, const TickDev &t, hipStream_t s);
hipError_t launch_install(ReqDesc *reqs, ChainSlot *slots, const ReqDesc *staged, const uint32_t *meta,
                          const uint32_t *idx, uint32_t n_new, uint32_t block_len, hipStream_t s);
hipError_t launch_req_zero(const ReqDesc *reqs, const uint32_t *req_ids, uint32_t n, hipStream_t s);

// One piece of a batched device-to-device copy (the serving loop's request inputs and outputs).
struct CopyPiece {
    const uint8_t *src;
    uint8_t *dst;
    uint64_t len;
};
constexpr uint64_t COPY_PIECE_BYTES = 1ull << 20;  // requests are cut into pieces of at most this size
// Appends the pieces of one copy of len bytes (at most COPY_PIECE_BYTES each) to arr[n...].
inline void add_copy_pieces(CopyPiece *arr, uint32_t &n, const void *src, void *dst, uint64_t len) {
    for (uint64_t o = 0; o < len; o += COPY_PIECE_BYTES) {
        CopyPiece &p = arr[n++];
        p.src = static_cast<const uint8_t *>(src) + o;
        p.dst = static_cast<uint8_t *>(dst) + o;
        p.len = len - o < COPY_PIECE_BYTES ? len - o : COPY_PIECE_BYTES;
    }
}
// diagnostics merge buffer: workgroup b of the histogram and of the lag sums adds its partial
// results into copy b mod DIAG_MERGE; the one-workgroup kernel that follows sums and clears them
constexpr int DIAG_MERGE = 8;
constexpr size_t DIAG_MERGE_WORDS = (size_t)DIAG_MERGE * 16386;  // 64-bit: 256 bins, or up to 16385 lags + the byte total, a copy
hipError_t launch_copy_many(const CopyPiece *pieces, uint32_t n, hipStream_t s);
// the same from a table in host memory, passed in the kernels' arguments (no upload, so nothing
// waits for the stream): one launch per COPY_ARG_PIECES pieces
constexpr uint32_t COPY_ARG_PIECES = 144;  // with the implicit arguments, under 4 KB of kernel arguments
hipError_t launch_copy_pieces_host(const CopyPiece *pieces, uint32_t n, hipStream_t s);

// The method's scalar pieces over device arrays (R, Theta, F^steps), for checking.
hipError_t launch_unit_r(const double *alpha, const uint8_t *om, size_t n, uint8_t *out, hipStream_t s);
hipError_t launch_unit_theta(const uint8_t *p, const uint8_t *o3, size_t n, double *out, hipStream_t s);
hipError_t launch_unit_lorenz(const lz_params &prm, double *r, size_t n, uint32_t steps, hipStream_t s);

// Streaming: fold the pending partial block into the tag, then write or check the tag.
hipError_t launch_stream_finish(const ChainSlot *slot, int pending, int empty, const lz_key &key,
                                unsigned long long *tag_acc, int decrypt, uint8_t *tag, int32_t *status,
                                hipStream_t s);

size_t lds_bytes(const KernelShape &sh);
bool shape_valid(const KernelShape &sh, const DevInfo &dev);

}  // namespace lz

// ---- context (runtime.cpp) ----------------------------------------------------------
struct lz_ctx {
    int device;
    lz_params prm;
    lz::KernelShape shape;
    lz::DevInfo dev;
    char arch[64];               // gcnArchName of the device
    double tuned_ms;             // last autotune: time of the winning shape's launch
    unsigned long long *ws_tag;  // 3 words, plain path tag accumulator
    int32_t *ws_status;          // plain path status (synchronous decrypt)
    int32_t *host_status;        // pinned
    hipStream_t last_stream;
    hipEvent_t last_event;
    bool has_last;
    // diagnostics merge buffer (DIAG_MERGE_WORDS), zero between calls: each call's last kernel clears it
    unsigned long long *diag_merge;
    // diagnostics workspace (grown on demand) and the event that orders its users
    void *diag_ws;
    size_t diag_ws_bytes;
    hipEvent_t diag_event;
    hipStream_t diag_last;
    bool diag_has_last;
};
