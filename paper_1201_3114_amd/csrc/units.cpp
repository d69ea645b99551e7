// The method's scalar pieces as entry points of their own: R (Eq. R_nu), Theta
// (Step 2) and the iterated map F (Section 3.1, Step 2), each evaluated by the
// same device code as the cipher kernels, so that each can be checked on its
// own against a reference.
#include <hip/hip_runtime.h>

#include "internal.h"

using namespace lz;

extern "C" int lz_unit_r(lz_ctx *c, const double *d_alpha, const uint8_t *d_omega, size_t n, uint8_t *d_out,
                         void *stream) {
    if (!c || (n && (!d_alpha || !d_omega || !d_out))) return fail(LZ_E_INVAL, "NULL argument");
    if (n == 0) return LZ_OK;
    LZ_HIP(hipSetDevice(c->device));
    LZ_HIP(launch_unit_r(d_alpha, d_omega, n, d_out, (hipStream_t)stream));
    return LZ_OK;
}

extern "C" int lz_unit_theta(lz_ctx *c, const uint8_t *d_p, const uint8_t *d_omega3, size_t n, double *d_out,
                             void *stream) {
    if (!c || (n && (!d_p || !d_omega3 || !d_out))) return fail(LZ_E_INVAL, "NULL argument");
    if (n == 0) return LZ_OK;
    LZ_HIP(hipSetDevice(c->device));
    LZ_HIP(launch_unit_theta(d_p, d_omega3, n, d_out, (hipStream_t)stream));
    return LZ_OK;
}

extern "C" int lz_unit_lorenz(lz_ctx *c, double *d_r, size_t n, uint32_t steps, void *stream) {
    if (!c || (n && !d_r)) return fail(LZ_E_INVAL, "NULL argument");
    if (n > ((size_t)1 << 31)) return fail(LZ_E_INVAL, "at most 2^31 states per call");
    if (n == 0) return LZ_OK;
    LZ_HIP(hipSetDevice(c->device));
    LZ_HIP(launch_unit_lorenz(c->prm, d_r, n, steps, (hipStream_t)stream));
    return LZ_OK;
}
