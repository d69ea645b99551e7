// lz_decrypt_noalloc: the plain decrypt for callers that cannot allocate
// device memory.  Its only scratch, the tag accumulator that lz_decrypt keeps
// in a context's workspace, lives in a file-scope device array instead.  The
// kernels are the plain path's own (fill, plain_kernel, finalize).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace lz {
namespace {

constexpr size_t SCRATCH_WORDS = LZ_NOALLOC_SCRATCH_BYTES / sizeof(unsigned long long);
constexpr size_t TAG_WORDS = 3;  // XOR accumulator of the block digests (x, y, z words)
static_assert(TAG_WORDS <= SCRATCH_WORDS, "the tag accumulator must fit the scratch array");

// One copy per GPU, held until the process ends.  Host code never passes this name to a kernel or
// a copy: it reaches the memory only through the address hipGetSymbolAddress gave for the device.
static __device__ __align__(256) unsigned long long scratch[SCRATCH_WORDS];

struct DevScratch {
    unsigned long long *ptr;  // this device's copy of `scratch`
    int lds_per_wg_max;
    bool ready;
};

DevScratch g_dev[LZ_NOALLOC_MAX_DEVICES];
std::mutex g_mu;

// Resolves the scratch address of device `dev` (the current device) on its first use.
int device_scratch(int dev, DevScratch *out) {
    std::lock_guard<std::mutex> lock(g_mu);
    DevScratch &d = g_dev[dev];
    if (!d.ready) {
        void *p = nullptr;
        LZ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LZ_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        int lds = 0;
        LZ_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        d.ptr = static_cast<unsigned long long *>(p);
        d.lds_per_wg_max = lds;
        d.ready = true;
    }
    *out = d;
    return LZ_OK;
}

}  // namespace
}  // namespace lz

using namespace lz;

extern "C" int lz_decrypt_noalloc(const lz_params *prm, const uint8_t *pw, size_t n_pw, const uint8_t *d_C,
                                  size_t n_c, uint8_t *d_P, int32_t *d_status, void *stream) {
    // argument checks first: nothing below runs on bad input
    if (!pw || !d_C) return fail(LZ_E_INVAL, "NULL argument");
    if (!d_status) return fail(LZ_E_INVAL, "d_status is required (a synchronous status would need host memory)");
    lz_params p;
    if (prm) p = *prm;
    else lz_params_default(&p);
    if (int rc = check_params(p)) return rc;
    if (n_pw == 0 || n_pw > LZ_MAX_PASSWORD) return fail(LZ_E_INVAL, "password length must be 1..64");
    if (n_c < LZ_TAG_BYTES) return fail(LZ_E_INVAL, "ciphertext shorter than the 24-byte tag");
    const size_t n = n_c - LZ_TAG_BYTES;
    if (int rc = check_blocks(p, n, nullptr)) return rc;
    if (!d_P && n) return fail(LZ_E_INVAL, "NULL plaintext buffer");
    lz_key key;
    if (int rc = key_setup(pw, n_pw, p, key)) return rc;

    int dev = 0;
    LZ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= LZ_NOALLOC_MAX_DEVICES) return fail(LZ_E_INVAL, "device index beyond LZ_NOALLOC_MAX_DEVICES");
    DevScratch d;
    if (int rc = device_scratch(dev, &d)) return rc;
    // the plain path's default shape (one chain per lane, 4 waves per workgroup, 128-byte tiles)
    KernelShape sh{1, 256, 128, 4};
    if (lds_bytes(sh) > (size_t)d.lds_per_wg_max) sh = KernelShape{1, 64, 32, 4};

    hipStream_t s = static_cast<hipStream_t>(stream);
    // the accumulator keeps the previous call's value: clear it with a kernel (no memset node under capture)
    LZ_HIP(launch_fill_u64(d.ptr, TAG_WORDS, s));
    LZ_HIP(launch_plain(sh, key, p, 1, d_C, d_P, n, d.ptr, s));
    LZ_HIP(launch_plain_finalize(1, d.ptr, d_C + n, nullptr, d_status, d_P, n, s));
    return LZ_OK;
}
