"""Python face of the C ABI (include/lorenz_cipher.h): contexts, the plain
path, batches and the server.  Torch supplies device memory and streams; the
library does all the work.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from .binding import IntegrityError, LorenzError, check  # noqa: F401  (re-exported)

TAG_BYTES = B.TAG_BYTES


def params(dt: float = 0.01, n_it: int = 3000, block_len: int = 256, lam=(1.0, 1.0, 1.0), k=(4, 4, 4),
           integrator="euler") -> B.Params:
    """Method parameters (Section 3.1): step, steps per byte, block length (>= n: the sequential
    version), lambda, k, and the integrator format ("euler", "euler_fma", "rk4")."""
    p = B.Params()
    check(B.lib.lz_params_default(ctypes.byref(p)))
    p.integrator = B.INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    p.dt = dt
    p.n_it = n_it
    p.block_len = block_len
    p.lam[:] = list(lam)
    p.k[:] = list(k)
    return p


def key_setup(pw: bytes, prm: B.Params | None = None) -> dict:
    """Password stage of Section 3.1 (host)."""
    k = B.Key()
    buf, n = B.pw_buf(pw)
    check(B.lib.lz_key_setup(buf, n, ctypes.byref(prm) if prm is not None else None, ctypes.byref(k)))
    return dict(a_prime=list(k.a_prime), r0=list(k.r0), mu=list(k.mu), omega=list(k.omega), k=list(k.k))


def _stream(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if t.dtype != torch.uint8 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous torch.uint8 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class LaunchShape:
    chains_per_lane: int = 1
    wg_size: int = 256
    tile: int = 64
    waves_per_simd: int = 4

    def to_c(self) -> B.Launch:
        return B.Launch(self.chains_per_lane, self.wg_size, self.tile, self.waves_per_simd)

    @staticmethod
    def from_c(l: B.Launch) -> "LaunchShape":
        return LaunchShape(l.chains_per_lane, l.wg_size, l.tile, l.waves_per_simd)


class Context:
    """A device plus method parameters; owns the plain path's small workspace."""

    def __init__(self, device: int = 0, prm: B.Params | None = None):
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        torch.cuda.init()
        check(B.lib.lz_context_create(device, ctypes.byref(prm) if prm is not None else None,
                                      ctypes.byref(self._h)))
        self.params = B.Params()
        check(B.lib.lz_context_params(self._h, ctypes.byref(self.params)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            B.lib.lz_context_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- launch shape
    def get_launch(self) -> LaunchShape:
        l = B.Launch()
        check(B.lib.lz_context_get_launch(self._h, ctypes.byref(l)))
        return LaunchShape.from_c(l)

    def set_launch(self, shape: LaunchShape):
        l = shape.to_c()
        check(B.lib.lz_context_set_launch(self._h, ctypes.byref(l)))

    def autotune(self, budget_ms: float = 0.0) -> LaunchShape:
        l = B.Launch()
        check(B.lib.lz_autotune(self._h, budget_ms, ctypes.byref(l)))
        return LaunchShape.from_c(l)

    def autotune_cached(self, path: str | None = None, budget_ms: float = 0.0) -> tuple[LaunchShape, bool]:
        """lz_autotune_cached: (shape, True if it came from the per-device cache file)."""
        l = B.Launch()
        hit = ctypes.c_int(0)
        check(B.lib.lz_autotune_cached(self._h, path.encode() if path is not None else None, budget_ms,
                                       ctypes.byref(l), ctypes.byref(hit)))
        return LaunchShape.from_c(l), bool(hit.value)

    # ---- plain path
    def encrypt(self, P: torch.Tensor, pw: bytes, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """C = E_pi(P) || tag, asynchronous on the stream."""
        n = P.numel()
        if out is None:
            out = torch.empty(n + TAG_BYTES, dtype=torch.uint8, device=self.device)
        if out.numel() != n + TAG_BYTES:
            raise ValueError("out must hold n + 24 bytes")
        buf, npw = B.pw_buf(pw)
        check(B.lib.lz_encrypt(self._h, buf, npw, _dev_ptr(P) if n else None, n, _dev_ptr(out),
                               _stream(stream, self.device)))
        return out

    def decrypt(self, C: torch.Tensor, pw: bytes, out: torch.Tensor | None = None,
                status: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """P = D_pi(C).  With status=None the call waits and raises IntegrityError on a
        tag mismatch; with a device int32 status tensor it stays asynchronous."""
        nc = C.numel()
        if nc < TAG_BYTES:
            raise ValueError("ciphertext shorter than the 24-byte tag")
        if out is None:
            out = torch.empty(nc - TAG_BYTES, dtype=torch.uint8, device=self.device)
        buf, npw = B.pw_buf(pw)
        st = None
        if status is not None:
            if status.dtype != torch.int32 or not status.is_cuda:
                raise ValueError("status must be a torch.int32 tensor on the GPU")
            st = ctypes.c_void_p(status.data_ptr())
        check(B.lib.lz_decrypt(self._h, buf, npw, _dev_ptr(C), nc, _dev_ptr(out) if nc > TAG_BYTES else None, st,
                               _stream(stream, self.device)))
        return out

    def encrypt_key(self, key: B.Key, P, out, stream=None):
        check(B.lib.lz_encrypt_key(self._h, ctypes.byref(key), _dev_ptr(P) if P.numel() else None, P.numel(),
                                   _dev_ptr(out), _stream(stream, self.device)))
        return out


def decrypt_noalloc(C: torch.Tensor, pw: bytes, out: torch.Tensor, status: torch.Tensor,
                    prm: B.Params | None = None, stream=None) -> torch.Tensor:
    """lz_decrypt_noalloc: lz_decrypt without a context and without device allocation, on the
    current device; out (n_c - 24 bytes) and status (one int32) are caller-provided GPU tensors.
    Calls that overlap on one GPU share its scratch and race; calls on one stream are ordered."""
    nc = C.numel()
    if nc < TAG_BYTES or out.numel() != nc - TAG_BYTES:
        raise ValueError("C must hold at least the 24-byte tag and out n_c - 24 bytes")
    if status.dtype != torch.int32 or not status.is_cuda or status.numel() < 1:
        raise ValueError("status must be a torch.int32 tensor on the GPU")
    buf, npw = B.pw_buf(pw)
    check(B.lib.lz_decrypt_noalloc(ctypes.byref(prm) if prm is not None else None, buf, npw, _dev_ptr(C), nc,
                                   _dev_ptr(out) if out.numel() else None, ctypes.c_void_p(status.data_ptr()),
                                   _stream(stream, C.device)))
    return out


class Batch:
    """Many messages, each with its own password, in one graph-captured persistent launch.

    Inputs and outputs are packed into single device tensors at the given byte offsets."""

    def __init__(self, ctx: Context, decrypt: bool, lens, pws, d_in: torch.Tensor, in_off, d_out: torch.Tensor,
                 out_off, d_status: torch.Tensor | None = None, shape: LaunchShape | None = None):
        n = len(lens)
        self.ctx = ctx
        self.n = n
        self._keep = (d_in, d_out, d_status)
        lens_a = np.ascontiguousarray(lens, dtype=np.uint64)
        in_a = np.ascontiguousarray(in_off, dtype=np.uint64)
        out_a = np.ascontiguousarray(out_off, dtype=np.uint64)
        pw_len = np.array([len(p) for p in pws], dtype=np.uint32)
        pw_off = np.zeros(n, dtype=np.uint64)
        if n > 1:
            pw_off[1:] = np.cumsum(pw_len[:-1], dtype=np.uint64)
        pw_all = np.frombuffer(b"".join(bytes(p) for p in pws) or b"\0", dtype=np.uint8).copy()
        u64p = ctypes.POINTER(ctypes.c_uint64)
        st = None
        if d_status is not None:
            if d_status.dtype != torch.int32 or d_status.numel() < n:
                raise ValueError("d_status must be an int32 tensor with one entry per message")
            st = ctypes.c_void_p(d_status.data_ptr())
        l = shape.to_c() if shape is not None else None
        self._h = ctypes.c_void_p()
        check(B.lib.lz_batch_create(ctx.handle, int(decrypt), n, lens_a.ctypes.data_as(u64p), in_a.ctypes.data_as(u64p),
                                    out_a.ctypes.data_as(u64p), pw_all.ctypes.data_as(B.u8p),
                                    pw_off.ctypes.data_as(u64p), pw_len.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    ctypes.c_void_p(d_in.data_ptr()), ctypes.c_void_p(d_out.data_ptr()), st,
                                    ctypes.byref(l) if l is not None else None, ctypes.byref(self._h)))

        self.decrypt_batch = bool(decrypt)

    def launch(self, stream=None):
        """Replays the batch with the statuses given at creation (lz_batch_launch)."""
        check(B.lib.lz_batch_launch(self._h, _stream(stream, self.ctx.device)))

    def encrypt(self, stream=None):
        """lz_encrypt_batch: every message of an encrypt batch, one replay."""
        check(B.lib.lz_encrypt_batch(self.ctx.handle, self._h, _stream(stream, self.ctx.device)))

    def decrypt(self, d_status: torch.Tensor, stream=None):
        """lz_decrypt_batch: every message of a decrypt batch, statuses into d_status (int32, n)."""
        if d_status.dtype != torch.int32 or not d_status.is_cuda or d_status.numel() < self.n:
            raise ValueError("d_status must be an int32 GPU tensor with one entry per message")
        self._status = d_status
        check(B.lib.lz_decrypt_batch(self.ctx.handle, self._h, ctypes.c_void_p(d_status.data_ptr()),
                                     _stream(stream, self.ctx.device)))

    def close(self):
        if self._h:
            B.lib.lz_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """One message of unknown length, encrypted or decrypted chunk by chunk (lz_stream_*)."""

    def __init__(self, ctx: Context, decrypt: bool, pw: bytes):
        self.ctx = ctx
        self.decrypt = bool(decrypt)
        self._h = ctypes.c_void_p()
        buf, npw = B.pw_buf(pw)
        check(B.lib.lz_stream_open(ctx.handle, int(decrypt), buf, npw, ctypes.byref(self._h)))

    def update(self, chunk: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        n = chunk.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.ctx.device)
        if n:
            check(B.lib.lz_stream_update(self._h, _dev_ptr(chunk), n, _dev_ptr(out), _stream(stream, self.ctx.device)))
            self._deferred = []  # an immediate update runs the queued chunks first
        return out

    def update_deferred(self, chunk: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """lz_stream_update_deferred: `out` is written only when the queued chunks run (flush, a full
        staging buffer, an immediate update or finish); keep it alive until then."""
        n = chunk.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.ctx.device)
        if n:
            self._deferred = getattr(self, "_deferred", [])
            self._deferred.append(out)
            check(B.lib.lz_stream_update_deferred(self._h, _dev_ptr(chunk), n, _dev_ptr(out),
                                                  _stream(stream, self.ctx.device)))
        return out

    def flush(self, stream=None):
        """lz_stream_flush: runs the queued deferred chunks."""
        check(B.lib.lz_stream_flush(self._h, _stream(stream, self.ctx.device)))
        self._deferred = []

    def finish(self, tag: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
        """Encrypt: returns the 24-byte tag tensor.  Decrypt: checks `tag`; raises IntegrityError
        (or writes `status` asynchronously when given)."""
        if not self.decrypt:
            tag = torch.empty(TAG_BYTES, dtype=torch.uint8, device=self.ctx.device) if tag is None else tag
        st = ctypes.c_void_p(status.data_ptr()) if status is not None else None
        check(B.lib.lz_stream_finish(self._h, _dev_ptr(tag), st, _stream(stream, self.ctx.device)))
        self._deferred = []
        return tag

    @property
    def position(self) -> int:
        return int(B.lib.lz_stream_position(self._h))

    def close(self):
        if self._h:
            B.lib.lz_stream_close(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def packed_offsets(lens, extra: int = 0, align: int = 1):
    """Offsets of messages laid end to end (each of len + extra bytes, aligned)."""
    offs = np.zeros(len(lens), dtype=np.uint64)
    pos = 0
    for i, n in enumerate(lens):
        offs[i] = pos
        pos += (int(n) + extra + align - 1) // align * align
    return offs, pos


class Server:
    """Continuous-batching request loop (library thread); see lz_server_* in the header."""

    def __init__(self, ctx: Context, hbm_budget: int, max_chains: int = 0, tick_bytes: int = 0, run_waves: int = 0,
                 policy: str = "adaptive"):
        self.ctx = ctx
        cfg = B.ServerConfig(hbm_budget, max_chains, tick_bytes, run_waves, B.SERVE_POLICIES[policy])
        self._h = ctypes.c_void_p()
        check(B.lib.lz_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(self._h)))

    def submit(self, rid: int, decrypt: bool, pw: bytes, src_ptr: int, n: int, dst_ptr: int, arrival_ns: int = 0):
        buf, npw = B.pw_buf(pw)
        check(B.lib.lz_server_submit(self._h, rid, int(decrypt), buf, npw, ctypes.c_void_p(src_ptr), n,
                                     ctypes.c_void_p(dst_ptr), arrival_ns))

    def submit_many(self, ids, decrypt, pws, src_ptrs, ns, dst_ptrs, arrival_ns):
        """Queues many requests in one call (arrays of equal length; pointers as integers)."""
        count = len(ids)
        u64 = lambda a: np.ascontiguousarray(a, dtype=np.uint64)
        ids_a, n_a, arr_a = u64(ids), u64(ns), u64(arrival_ns)
        src_a, dst_a = u64(src_ptrs), u64(dst_ptrs)
        dec_a = np.ascontiguousarray(decrypt, dtype=np.uint8)
        pw_len = np.array([len(p) for p in pws], dtype=np.uint32)
        pw_off = np.zeros(count, dtype=np.uint64)
        if count > 1:
            pw_off[1:] = np.cumsum(pw_len[:-1], dtype=np.uint64)
        pw_all = np.frombuffer(b"".join(bytes(p) for p in pws) or b"\0", dtype=np.uint8).copy()
        P64 = ctypes.POINTER(ctypes.c_uint64)
        PV = ctypes.POINTER(ctypes.c_void_p)
        check(B.lib.lz_server_submit_many(self._h, count, ids_a.ctypes.data_as(P64), dec_a.ctypes.data_as(B.u8p),
                                          pw_all.ctypes.data_as(B.u8p), pw_off.ctypes.data_as(P64),
                                          pw_len.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                          src_a.ctypes.data_as(PV), n_a.ctypes.data_as(P64), dst_a.ctypes.data_as(PV),
                                          arr_a.ctypes.data_as(P64)))

    def cancel(self, rid: int):
        """Drops request rid; its completion reports LZ_E_CANCELLED (-6) unless it finished first."""
        check(B.lib.lz_server_cancel(self._h, rid))

    def poll(self, max_n: int = 4096, timeout_ms: int = 0):
        arr = (B.Completion * max_n)()
        k = check(B.lib.lz_server_poll(self._h, arr, max_n, timeout_ms))
        return [(c.id, c.status, c.arrival_ns, c.admit_ns, c.done_ns) for c in arr[:k]]

    def stats(self) -> dict:
        s = B.ServerStats()
        check(B.lib.lz_server_stats_get(self._h, ctypes.byref(s)))
        return dict(ticks=s.ticks, chain_bytes=s.chain_bytes, peak_hbm=s.peak_hbm, admitted=s.admitted,
                    completed=s.completed, busy_ms=s.busy_ms)

    def close(self):
        if self._h:
            rc = B.lib.lz_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def histogram(ctx: Context, data: torch.Tensor, stream=None) -> torch.Tensor:
    """Byte histogram on the device (256 int64 counts) -- Section 4's frequency analysis."""
    out = torch.empty(256, dtype=torch.int64, device=ctx.device)
    n = data.numel()
    check(B.lib.lz_histogram(ctx.handle, _dev_ptr(data) if n else None, n, ctypes.c_void_p(out.data_ptr()),
                             _stream(stream, ctx.device)))
    return out


def entropy(ctx: Context, hist: torch.Tensor, stream=None) -> float:
    """Shannon entropy in bits per byte of a device histogram (Section 4), computed on the device."""
    if hist.dtype != torch.int64 or hist.numel() != 256 or not hist.is_cuda or not hist.is_contiguous():
        raise ValueError("expected the 256-bin int64 device histogram of histogram()")
    out = torch.empty(1, dtype=torch.float64, device=ctx.device)
    check(B.lib.lz_entropy(ctx.handle, ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                           _stream(stream, ctx.device)))
    return float(out.item())


def lag_sums(ctx: Context, data: torch.Tensor, max_lag: int, stream=None) -> torch.Tensor:
    """Exact S_k = sum_i x_i x_{i+k}, k = 0..max_lag, on the device (int64)."""
    out = torch.empty(max_lag + 1, dtype=torch.int64, device=ctx.device)
    n = data.numel()
    check(B.lib.lz_lag_sums(ctx.handle, _dev_ptr(data) if n else None, n, max_lag, ctypes.c_void_p(out.data_ptr()),
                            _stream(stream, ctx.device)))
    return out


def autocorrelation(ctx: Context, data: torch.Tensor, max_lag: int, stream=None) -> torch.Tensor:
    """r_k, k = 0..max_lag, of the mean-removed byte sequence, on the device (Section 4, autocorrelation)."""
    out = torch.empty(max_lag + 1, dtype=torch.float64, device=ctx.device)
    n = data.numel()
    check(B.lib.lz_autocorrelation(ctx.handle, _dev_ptr(data) if n else None, n, max_lag,
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream, ctx.device)))
    return out


def _matrix(img: torch.Tensor):
    if img.dim() != 2 or img.dtype != torch.uint8 or not img.is_contiguous():
        raise LorenzError(-1, "expected a contiguous 2-D uint8 tensor")
    return img.shape[0], img.shape[1]


def power_spectrum_2d(ctx: Context, img: torch.Tensor, stream=None) -> torch.Tensor:
    """|DFT2|^2 of a byte matrix (h x w float64, zero frequency at [0, 0]) -- Section 4's image spectrum."""
    h, w = _matrix(img)
    out = torch.empty((h, w), dtype=torch.float64, device=ctx.device)
    check(B.lib.lz_power_spectrum_2d(ctx.handle, _dev_ptr(img), h, w, ctypes.c_void_p(out.data_ptr()),
                                     _stream(stream, ctx.device)))
    return out


def autocorrelation_2d(ctx: Context, img: torch.Tensor, stream=None) -> torch.Tensor:
    """Circular autocorrelation matrix of a mean-removed byte matrix (h x w float64) -- Section 4."""
    h, w = _matrix(img)
    out = torch.empty((h, w), dtype=torch.float64, device=ctx.device)
    check(B.lib.lz_autocorrelation_2d(ctx.handle, _dev_ptr(img), h, w, ctypes.c_void_p(out.data_ptr()),
                                      _stream(stream, ctx.device)))
    return out


def _dev_typed(t: torch.Tensor, dtype):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def unit_r(ctx: Context, alpha: torch.Tensor, omega: torch.Tensor, stream=None) -> torch.Tensor:
    """R(alpha_i, omega_i) (Section 3.2) for float64 alpha and uint8 omega (0..3), as the kernels compute it."""
    if alpha.numel() != omega.numel():
        raise ValueError("alpha and omega differ in length")
    out = torch.empty(alpha.numel(), dtype=torch.uint8, device=alpha.device)
    check(B.lib.lz_unit_r(ctx.handle, _dev_typed(alpha, torch.float64), _dev_typed(omega, torch.uint8),
                          alpha.numel(), _dev_typed(out, torch.uint8), _stream(stream, ctx.device)))
    return out


def unit_theta(ctx: Context, p: torch.Tensor, omega3: torch.Tensor, stream=None) -> torch.Tensor:
    """Theta = p_i / 10^(3 + omega3_i) (Step 2) for uint8 p and omega3, as the kernels compute it."""
    if p.numel() != omega3.numel():
        raise ValueError("p and omega3 differ in length")
    out = torch.empty(p.numel(), dtype=torch.float64, device=p.device)
    check(B.lib.lz_unit_theta(ctx.handle, _dev_typed(p, torch.uint8), _dev_typed(omega3, torch.uint8), p.numel(),
                              _dev_typed(out, torch.float64), _stream(stream, ctx.device)))
    return out


def unit_lorenz(ctx: Context, r: torch.Tensor, steps: int, stream=None) -> torch.Tensor:
    """Advances each row (x, y, z) of the float64 (n, 3) tensor r in place by `steps` steps of the
    context's integrator (Section 3.1); returns r."""
    if r.dim() != 2 or r.shape[1] != 3:
        raise ValueError("expected an (n, 3) tensor")
    check(B.lib.lz_unit_lorenz(ctx.handle, _dev_typed(r, torch.float64), r.shape[0], int(steps),
                               _stream(stream, ctx.device)))
    return r


def now_ns() -> int:
    return int(B.lib.lz_now_ns())
