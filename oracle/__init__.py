"""CPU oracle of the Lorenz chaotic cipher (arXiv:1201.3114) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liblzoracle.so`` (built from ``lz_oracle.c``
by :func:`build`) through ctypes; ``pyref`` is an independent pure-Python
implementation of the same reading, for tiny inputs.  Nothing here imports or
links the GPU library, and the GPU library never imports this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblzoracle.so")
SRC_PATH = os.path.join(HERE, "lz_oracle.c")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-msse2", "-mfpmath=sse", "-fPIC", "-shared", "-Wall"]


def build() -> str:
    """Compile the oracle with gcc (no contraction, SSE2 binary64)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC_PATH, "-o", tmp, "-lcrypto", "-lpthread", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("lam", ctypes.c_double * 3), ("n_it", ctypes.c_uint32),
                ("block_len", ctypes.c_uint32), ("k", ctypes.c_uint32 * 3), ("integrator", ctypes.c_uint32)]


class Key(ctypes.Structure):
    _fields_ = [("a_prime", ctypes.c_double * 3), ("r0", ctypes.c_double * 3), ("mu", ctypes.c_int32 * 3),
                ("omega", ctypes.c_int32 * 3), ("k", ctypes.c_int32 * 3), ("D", ctypes.c_int32),
                ("L", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_key_setup.argtypes = [u8p, ctypes.c_size_t, ctypes.POINTER(Params), ctypes.POINTER(Key),
                                    ctypes.c_char_p]
        L.orc_key_setup.restype = ctypes.c_int
        L.orc_lorenz.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_uint64]
        L.orc_lorenz.restype = None
        L.orc_lorenz_integrator.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_uint64,
                                            ctypes.c_uint32]
        L.orc_lorenz_integrator.restype = None
        L.orc_R.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_R.restype = ctypes.c_int
        L.orc_theta.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_theta.restype = ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_R_many.argtypes = [dp, u8p, ctypes.c_size_t, u8p]
        L.orc_R_many.restype = ctypes.c_int
        L.orc_theta_many.argtypes = [u8p, u8p, ctypes.c_size_t, dp]
        L.orc_theta_many.restype = None
        L.orc_lorenz_many.argtypes = [dp, ctypes.c_size_t, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int]
        L.orc_lorenz_many.restype = None
        L.orc_encrypt.argtypes = [u8p, ctypes.c_size_t, ctypes.POINTER(Params), u8p, ctypes.c_size_t, u8p,
                                  ctypes.c_int]
        L.orc_encrypt.restype = ctypes.c_int
        L.orc_decrypt.argtypes = [u8p, ctypes.c_size_t, ctypes.POINTER(Params), u8p, ctypes.c_size_t, u8p,
                                  ctypes.c_int]
        L.orc_decrypt.restype = ctypes.c_int
        L.orc_crypt_block.argtypes = [u8p, ctypes.c_size_t, ctypes.POINTER(Params), ctypes.c_uint64, u8p,
                                      ctypes.c_size_t, u8p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
        L.orc_crypt_block.restype = ctypes.c_int
        L.orc_crypt_range.argtypes = [u8p, ctypes.c_size_t, ctypes.POINTER(Params), ctypes.c_uint64, u8p,
                                      ctypes.c_size_t, u8p, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.orc_crypt_range.restype = ctypes.c_int
        _lib = L
    return _lib


INTEGRATORS = {"euler": 0, "euler_fma": 1, "rk4": 2}

ESCAPED = -4  # the oracle's code for a trajectory that left the domain of R and N


class TrajectoryEscaped(ValueError):
    """A coordinate of the trajectory became non-finite or reached 2^19 in magnitude, where
    floor(v 10^13) no longer fits a 64-bit integer: R and the tag are undefined there."""


def _raise(what: str, rc: int):
    if rc == ESCAPED:
        raise TrajectoryEscaped(f"{what}: the trajectory left the attractor")
    raise ValueError(f"{what} rc={rc}")


def params(dt=0.01, n_it=3000, block_len=256, lam=(1.0, 1.0, 1.0), k=(4, 4, 4), integrator="euler") -> Params:
    p = Params()
    p.integrator = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    p.dt = dt
    p.lam[:] = list(lam)
    p.n_it = n_it
    p.block_len = block_len
    p.k[:] = list(k)
    return p


def _u8(buf):
    arr = np.ascontiguousarray(np.frombuffer(bytes(buf), dtype=np.uint8)) if not isinstance(buf, np.ndarray) \
        else np.ascontiguousarray(buf, dtype=np.uint8)
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def key_setup(pw: bytes, **kw) -> dict:
    prm = params(**kw)
    k = Key()
    a_dec = ctypes.create_string_buffer(3 * 128)
    pwa, pwp = _u8(pw)
    rc = lib().orc_key_setup(pwp, len(pw), ctypes.byref(prm), ctypes.byref(k), a_dec)
    if rc:
        raise ValueError(f"orc_key_setup rc={rc}")
    a = [int(a_dec.raw[128 * j:128 * (j + 1)].split(b"\0")[0]) for j in range(3)]
    return dict(a=a, L=k.L, D=k.D, a_prime=list(k.a_prime), r0=list(k.r0), mu=list(k.mu), omega=list(k.omega),
                k=list(k.k))


def lorenz(r, dt, steps, integrator="euler"):
    arr = (ctypes.c_double * 3)(*r)
    code = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    lib().orc_lorenz_integrator(arr, dt, steps, code)
    return list(arr)


def R(alpha: float, omega: int) -> int:
    return lib().orc_R(alpha, omega)


def theta(p: int, omega3: int) -> float:
    return lib().orc_theta(p, omega3)


def R_many(alpha, omega) -> np.ndarray:
    """R(alpha_i, omega_i) over arrays (loops over orc_R)."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.uint8)
    out = np.empty(len(al), dtype=np.uint8)
    rc = lib().orc_R_many(al.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          om.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(al),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc:
        raise ValueError("R_many: some alpha outside the domain |alpha| < 2^19")
    return out


def theta_many(p, omega3) -> np.ndarray:
    """Theta(p_i, omega3_i) over arrays (loops over orc_theta)."""
    pa = np.ascontiguousarray(p, dtype=np.uint8)
    om = np.ascontiguousarray(omega3, dtype=np.uint8)
    out = np.empty(len(pa), dtype=np.float64)
    lib().orc_theta_many(pa.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                         om.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(pa),
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def lorenz_many(r, dt, steps, integrator="euler", nthreads: int = 8) -> np.ndarray:
    """Each row (x, y, z) of r advanced by `steps` integrator steps (loops over orc_lorenz_integrator)."""
    arr = np.array(r, dtype=np.float64, order="C").reshape(-1, 3)
    code = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    lib().orc_lorenz_many(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(arr), dt, steps, code, nthreads)
    return arr


def encrypt(pw: bytes, P, nthreads: int = 1, **kw) -> np.ndarray:
    prm = params(**kw)
    pa, pp = _u8(P)
    out = np.empty(len(pa) + 24, dtype=np.uint8)
    pwa, pwp = _u8(pw)
    rc = lib().orc_encrypt(pwp, len(pw), ctypes.byref(prm), pp, len(pa),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), nthreads)
    if rc:
        _raise("orc_encrypt", rc)
    return out


def decrypt(pw: bytes, C, nthreads: int = 1, **kw):
    """Returns (plaintext ndarray, ok)."""
    prm = params(**kw)
    ca, cp = _u8(C)
    if len(ca) < 24:
        raise ValueError("ciphertext shorter than the 24-byte tag")
    out = np.empty(len(ca) - 24, dtype=np.uint8)
    pwa, pwp = _u8(pw)
    rc = lib().orc_decrypt(pwp, len(pw), ctypes.byref(prm), cp, len(ca),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), nthreads)
    if rc not in (0, -2):
        _raise("orc_decrypt", rc)
    return out, rc == 0


def crypt_block(pw: bytes, b: int, data, decrypt: bool = False, **kw):
    """Block b of a message alone: returns (output bytes, digest triple)."""
    prm = params(**kw)
    da, dp = _u8(data)
    out = np.empty(len(da), dtype=np.uint8)
    d = (ctypes.c_uint64 * 3)()
    pwa, pwp = _u8(pw)
    rc = lib().orc_crypt_block(pwp, len(pw), ctypes.byref(prm), b, dp, len(da),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(decrypt), d)
    if rc:
        _raise("orc_crypt_block", rc)
    return out, tuple(d)


def crypt_range(pw: bytes, b0: int, data, decrypt: bool = False, nthreads: int = 1, **kw):
    """Blocks b0, b0 + 1, ... of a message (data starts at byte b0 * block_len of it): returns
    (output bytes, XOR of the blocks' digests).  The parts of a message's ranges XOR to its tag."""
    prm = params(**kw)
    da, dp = _u8(data)
    out = np.empty(len(da), dtype=np.uint8)
    d = (ctypes.c_uint64 * 3)()
    pwa, pwp = _u8(pw)
    rc = lib().orc_crypt_range(pwp, len(pw), ctypes.byref(prm), b0, dp, len(da),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(decrypt), nthreads, d)
    if rc:
        _raise("orc_crypt_range", rc)
    return out, tuple(d)
