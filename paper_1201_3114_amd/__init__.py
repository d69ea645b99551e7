"""MI355X (gfx950) implementation of the Lorenz-attractor chaotic cipher of
arXiv:1201.3114 (parallel fast version): C-ABI library liblorenz_cipher.so
with hand-written HIP kernels, and this thin Python layer over it.

Importing the package loads the library and fails if it is not built.
"""
from .cipher import (TAG_BYTES, Batch, Context, IntegrityError, LaunchShape, LorenzError, Server, Stream,  # noqa: F401
                     autocorrelation, autocorrelation_2d, decrypt_noalloc, entropy, histogram, key_setup, lag_sums, now_ns,
                     packed_offsets, params, power_spectrum_2d, unit_lorenz, unit_r, unit_theta)
