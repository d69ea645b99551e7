"""ctypes binding of liblorenz_cipher.so: argument marshalling only.

Device buffers are torch uint8 tensors on the ROCm device (their data_ptr()
is handed to the library); streams are torch.cuda streams.  Every byte of the
cipher is computed by the library's HIP kernels; there is no fallback: if
the library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblorenz_cipher.so")

LZ_OK, LZ_E_INVAL, LZ_E_INTEGRITY, LZ_E_NOMEM, LZ_E_HIP, LZ_E_AGAIN, LZ_E_CANCELLED = 0, -1, -2, -3, -4, -5, -6
TAG_BYTES = 24
INTEGRATORS = {"euler": 0, "euler_fma": 1, "rk4": 2}
SERVE_POLICIES = {"adaptive": 0, "all_chains": 1}

u8p = ctypes.POINTER(ctypes.c_uint8)
vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("lam", ctypes.c_double * 3), ("n_it", ctypes.c_uint32),
                ("block_len", ctypes.c_uint32), ("k", ctypes.c_uint8 * 3), ("integrator", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8 * 4)]


class Key(ctypes.Structure):
    _fields_ = [("a_prime", ctypes.c_double * 3), ("r0", ctypes.c_double * 3), ("mu", ctypes.c_uint8 * 3),
                ("omega", ctypes.c_uint8 * 3), ("k", ctypes.c_uint8 * 3), ("reserved", ctypes.c_uint8 * 7)]


class Launch(ctypes.Structure):
    _fields_ = [("chains_per_lane", ctypes.c_uint32), ("wg_size", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("waves_per_simd", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_chains", ctypes.c_uint32), ("tick_bytes", ctypes.c_uint32),
                ("run_waves", ctypes.c_uint32), ("policy", ctypes.c_uint32)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("arrival_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64), ("done_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_uint64), ("chain_bytes", ctypes.c_uint64), ("peak_hbm", ctypes.c_uint64),
                ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("busy_ms", ctypes.c_double)]


# name -> (restype, argtypes); the exported surface of include/lorenz_cipher.h
SIGNATURES = {
    "lz_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "lz_params_check": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "lz_ciphertext_len": (ctypes.c_size_t, [ctypes.c_size_t]),
    "lz_block_count": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "lz_key_setup": (ctypes.c_int, [u8p, ctypes.c_size_t, ctypes.POINTER(Params), ctypes.POINTER(Key)]),
    "lz_last_error": (ctypes.c_char_p, []),
    "lz_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(vp)]),
    "lz_context_destroy": (ctypes.c_int, [vp]),
    "lz_context_params": (ctypes.c_int, [vp, ctypes.POINTER(Params)]),
    "lz_context_set_launch": (ctypes.c_int, [vp, ctypes.POINTER(Launch)]),
    "lz_context_get_launch": (ctypes.c_int, [vp, ctypes.POINTER(Launch)]),
    "lz_encrypt": (ctypes.c_int, [vp, u8p, ctypes.c_size_t, vp, ctypes.c_size_t, vp, vp]),
    "lz_decrypt": (ctypes.c_int, [vp, u8p, ctypes.c_size_t, vp, ctypes.c_size_t, vp, vp, vp]),
    "lz_encrypt_key": (ctypes.c_int, [vp, ctypes.POINTER(Key), vp, ctypes.c_size_t, vp, vp]),
    "lz_decrypt_key": (ctypes.c_int, [vp, ctypes.POINTER(Key), vp, ctypes.c_size_t, vp, vp, vp]),
    "lz_decrypt_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), u8p, ctypes.c_size_t, vp, ctypes.c_size_t, vp,
                                          vp, vp]),
    "lz_batch_create": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), u8p,
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32), vp, vp, vp,
                                       ctypes.POINTER(Launch), ctypes.POINTER(vp)]),
    "lz_batch_launch": (ctypes.c_int, [vp, vp]),
    "lz_encrypt_batch": (ctypes.c_int, [vp, vp, vp]),
    "lz_decrypt_batch": (ctypes.c_int, [vp, vp, vp, vp]),
    "lz_batch_destroy": (ctypes.c_int, [vp]),
    "lz_autotune": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(Launch)]),
    "lz_autotune_cached": (ctypes.c_int, [vp, ctypes.c_char_p, ctypes.c_double, ctypes.POINTER(Launch),
                                          ctypes.POINTER(ctypes.c_int)]),
    "lz_server_create": (ctypes.c_int, [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
    "lz_server_submit": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_int, u8p, ctypes.c_size_t, vp,
                                        ctypes.c_uint64, vp, ctypes.c_uint64]),
    "lz_server_submit_many": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64), u8p, u8p,
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(vp),
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "lz_server_cancel": (ctypes.c_int, [vp, ctypes.c_uint64]),
    "lz_server_poll": (ctypes.c_int, [vp, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_int]),
    "lz_server_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
    "lz_server_destroy": (ctypes.c_int, [vp]),
    "lz_now_ns": (ctypes.c_uint64, []),
    "lz_unit_r": (ctypes.c_int, [vp, vp, vp, ctypes.c_size_t, vp, vp]),
    "lz_unit_theta": (ctypes.c_int, [vp, vp, vp, ctypes.c_size_t, vp, vp]),
    "lz_unit_lorenz": (ctypes.c_int, [vp, vp, ctypes.c_size_t, ctypes.c_uint32, vp]),
    "lz_histogram": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, vp]),
    "lz_lag_sums": (ctypes.c_int, [vp, vp, ctypes.c_size_t, ctypes.c_uint32, vp, vp]),
    "lz_entropy": (ctypes.c_int, [vp, vp, vp, vp]),
    "lz_autocorrelation": (ctypes.c_int, [vp, vp, ctypes.c_size_t, ctypes.c_uint32, vp, vp]),
    "lz_power_spectrum_2d": (ctypes.c_int, [vp, vp, ctypes.c_uint32, ctypes.c_uint32, vp, vp]),
    "lz_autocorrelation_2d": (ctypes.c_int, [vp, vp, ctypes.c_uint32, ctypes.c_uint32, vp, vp]),
    "lz_stream_open": (ctypes.c_int, [vp, ctypes.c_int, u8p, ctypes.c_size_t, ctypes.POINTER(vp)]),
    "lz_stream_update": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, vp]),
    "lz_stream_update_deferred": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, vp]),
    "lz_stream_flush": (ctypes.c_int, [vp, vp]),
    "lz_stream_finish": (ctypes.c_int, [vp, vp, vp, vp]),
    "lz_stream_position": (ctypes.c_uint64, [vp]),
    "lz_stream_close": (ctypes.c_int, [vp]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python __graft_entry__.py build` "
                          "(hipcc, gfx950); there is no fallback implementation")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class LorenzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class IntegrityError(LorenzError):
    pass


def check(rc: int) -> int:
    if rc >= 0:
        return rc
    msg = lib.lz_last_error().decode(errors="replace")
    if rc == LZ_E_INTEGRITY:
        raise IntegrityError(rc, msg)
    raise LorenzError(rc, msg)


def pw_buf(pw: bytes):
    pw = bytes(pw)
    buf = (ctypes.c_uint8 * max(len(pw), 1)).from_buffer_copy(pw if pw else b"\0")
    return buf, len(pw)
