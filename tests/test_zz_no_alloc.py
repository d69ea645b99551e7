"""lz_decrypt_noalloc (no context, static device scratch) against lz_decrypt, through the C ABI,
called directly and replayed from a captured HIP graph.

Both entry points run the same kernels; the no-allocation one keeps the tag accumulator in a
static device array that every call on the GPU shares.  Each check runs two no-allocation calls
in a row on one stream, the second on a smaller message, so a tag left over from the first call
would show up as a wrong status or a zeroed plaintext in the second.  Outputs and statuses are
compared byte for byte with lz_decrypt's on the same ciphertexts.
"""
import ctypes

import numpy as np
import pytest

from gpu_util import need_gpu, say

PW = b"no-alloc password 0123456789"


@pytest.fixture(scope="module")
def env():
    need_gpu()
    import torch

    import paper_1201_3114_amd as lz
    from paper_1201_3114_amd import binding as B

    return torch, lz, B


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc(torch, B, prm, pw, C, out, st):
    buf, npw = B.pw_buf(pw)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return B.lib.lz_decrypt_noalloc(ctypes.byref(prm) if prm is not None else None, buf, npw, _ptr(C), C.numel(),
                                    _ptr(out) if out.numel() else None, _ptr(st), s)


def _reference(torch, lz, ctx, pw, C):
    """lz_decrypt with a device status: the plaintext (zeroed on failure) and the status."""
    out = torch.full((C.numel() - 24,), 0xAB, dtype=torch.uint8, device="cuda")
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    ctx.decrypt(C, pw, out=out, status=st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.cpu()[0])


def _pair(torch, lz, B, prm, ctx, cases):
    """Runs the no-allocation decrypt on each (ciphertext, password) in order, back to back on the
    current stream, then compares each output and status with lz_decrypt's."""
    outs, sts = [], []
    for C, pw in cases:
        out = torch.full((C.numel() - 24,), 0xAB, dtype=torch.uint8, device="cuda")
        st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        rc = _noalloc(torch, B, prm, pw, C, out, st)
        assert rc == 0, B.lib.lz_last_error()
        outs.append(out)
        sts.append(st)
    torch.cuda.synchronize()
    for (C, pw), out, st in zip(cases, outs, sts):
        want, want_st = _reference(torch, lz, ctx, pw, C)
        assert int(st.cpu()[0]) == want_st
        assert np.array_equal(out.cpu().numpy(), want)
    return [int(s.cpu()[0]) for s in sts]


def _cipher(torch, ctx, rng, n, pw=PW):
    P = torch.from_numpy(rng.integers(0, 256, n, dtype=np.uint8)).cuda()
    C = ctx.encrypt(P, pw)
    torch.cuda.synchronize()
    return P, C


def _altered(C, at, v=0x5A):
    bad = C.clone()
    bad[at] ^= v
    return bad


@pytest.mark.gpu
@pytest.mark.parametrize("n_it", [3000, 30])
def test_noalloc_equals_lz_decrypt_two_calls(env, n_it):
    torch, lz, B = env
    prm = lz.params(n_it=n_it)
    ctx = lz.Context(0, prm)
    rng = np.random.default_rng(900 + n_it)
    P1, C1 = _cipher(torch, ctx, rng, 300 * 256 + 77)  # 301 blocks: two workgroups and a ragged tail
    P2, C2 = _cipher(torch, ctx, rng, 1000)           # smaller: 4 blocks
    say(f"no-alloc decrypt, n_it {n_it}: {C1.numel()} then {C2.numel()} bytes")
    assert _pair(torch, lz, B, prm, ctx, [(C1, PW), (C2, PW)]) == [0, 0]
    # the plaintexts themselves (lz_decrypt's output was compared above)
    out = torch.empty(P2.numel(), dtype=torch.uint8, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    assert _noalloc(torch, B, prm, PW, C2, out, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, P2) and int(st.cpu()[0]) == 0
    # an altered ciphertext first, then a smaller untouched one: the failure must not leak
    say("  altered body byte, then a smaller untouched message")
    assert _pair(torch, lz, B, prm, ctx, [(_altered(C1, 12345), PW), (C2, PW)]) == [B.LZ_E_INTEGRITY, 0]
    say("  untouched, then a smaller message with an altered tag byte")
    assert _pair(torch, lz, B, prm, ctx, [(C1, PW), (_altered(C2, C2.numel() - 3), PW)]) == [0, B.LZ_E_INTEGRITY]
    say("  wrong password on the smaller message")
    assert _pair(torch, lz, B, prm, ctx, [(C1, PW), (C2, b"not the password")]) == [0, B.LZ_E_INTEGRITY]
    ctx.close()


@pytest.mark.gpu
def test_noalloc_empty_and_default_params(env):
    """prm NULL = the defaults; an empty message (ciphertext = tag only) after a longer one."""
    torch, lz, B = env
    ctx = lz.Context(0)
    rng = np.random.default_rng(911)
    _, C1 = _cipher(torch, ctx, rng, 5 * 256 + 3)
    _, C0 = _cipher(torch, ctx, rng, 0)
    say("no-alloc decrypt, defaults: 1283 bytes then the empty message")
    assert _pair(torch, lz, B, None, ctx, [(C1, PW), (C0, PW)]) == [0, 0]
    assert _pair(torch, lz, B, None, ctx, [(C1, PW), (_altered(C0, 0), PW)]) == [0, B.LZ_E_INTEGRITY]
    ctx.close()


@pytest.mark.gpu
def test_noalloc_rejects_before_running(env):
    """Bad arguments return LZ_E_INVAL and leave the outputs untouched."""
    torch, lz, B = env
    prm = lz.params(n_it=30)
    C = torch.zeros(64, dtype=torch.uint8, device="cuda")
    out = torch.full((40,), 7, dtype=torch.uint8, device="cuda")
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    buf, npw = B.pw_buf(PW)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(prm), buf, npw, _ptr(C), 23, _ptr(out), _ptr(st), s) == B.LZ_E_INVAL
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(prm), buf, npw, _ptr(C), 64, _ptr(out), None, s) == B.LZ_E_INVAL
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(prm), buf, 0, _ptr(C), 64, _ptr(out), _ptr(st), s) == B.LZ_E_INVAL
    # past the limits: rejected on the host, nothing is read
    big = (1 << 32) + 1 + 24
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(prm), buf, npw, _ptr(C), big, _ptr(out), _ptr(st), s) == B.LZ_E_INVAL
    assert b"2^32" in B.lib.lz_last_error()
    small_blocks = lz.params(n_it=30, block_len=16)
    big = (1 << 24) * 16 + 1 + 24
    assert B.lib.lz_decrypt_noalloc(ctypes.byref(small_blocks), buf, npw, _ptr(C), big, _ptr(out), _ptr(st),
                                    s) == B.LZ_E_INVAL
    assert b"blocks" in B.lib.lz_last_error()
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == 99 and bool((out == 7).all())


GPW = b"graph-captured decrypt"


@pytest.mark.gpu
def test_noalloc_decrypt_in_a_graph_replays_exactly():
    """One capture of two no-allocation decrypts (an untouched ciphertext, then an altered one); five
    replays with eager work between them (new ciphertext bytes copied into the captured input buffers
    and the outputs poisoned); every replay's plaintexts and statuses equal lz_decrypt's on the same
    bytes."""
    need_gpu()
    import torch

    import paper_1201_3114_amd as lz
    from paper_1201_3114_amd import binding as B

    prm = lz.params(n_it=40)
    ctx = lz.Context(0, prm)
    rng = np.random.default_rng(930)
    n1, n2 = 70 * 256 + 11, 3 * 256 + 5
    C1 = torch.empty(n1 + 24, dtype=torch.uint8, device="cuda")
    C2 = torch.empty(n2 + 24, dtype=torch.uint8, device="cuda")
    out1 = torch.empty(n1, dtype=torch.uint8, device="cuda")
    out2 = torch.empty(n2, dtype=torch.uint8, device="cuda")
    st = torch.empty(2, dtype=torch.int32, device="cuda")
    buf, npw = B.pw_buf(GPW)

    def decrypt_both():
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for C, out, i in ((C1, out1, 0), (C2, out2, 1)):
            rc = B.lib.lz_decrypt_noalloc(ctypes.byref(prm), buf, npw, ctypes.c_void_p(C.data_ptr()), C.numel(),
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.data_ptr() + 4 * i), s)
            assert rc == 0, B.lib.lz_last_error()

    def fresh_inputs(k):
        P1 = torch.from_numpy(rng.integers(0, 256, n1, dtype=np.uint8)).cuda()
        P2 = torch.from_numpy(rng.integers(0, 256, n2, dtype=np.uint8)).cuda()
        C1.copy_(ctx.encrypt(P1, GPW))
        C2.copy_(ctx.encrypt(P2, GPW))
        C2[(37 * k) % (n2 + 24)] ^= 1 + k  # the second message altered, a different byte each time
        return P1

    fresh_inputs(0)
    decrypt_both()  # first call on the device outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        decrypt_both()
    torch.cuda.synchronize()
    for k in range(1, 6):
        P1 = fresh_inputs(k)
        out1.fill_(0xAB)
        out2.fill_(0xAB)
        st.fill_(12345)
        g.replay()
        torch.cuda.synchronize()
        ref1 = torch.empty(n1, dtype=torch.uint8, device="cuda")
        ref2 = torch.empty(n2, dtype=torch.uint8, device="cuda")
        rst = torch.empty(2, dtype=torch.int32, device="cuda")
        ctx.decrypt(C1, GPW, out=ref1, status=rst[0:1])
        ctx.decrypt(C2, GPW, out=ref2, status=rst[1:2])
        torch.cuda.synchronize()
        say(f"replay {k}: statuses {st.tolist()} (lz_decrypt {rst.tolist()})")
        assert st.tolist() == rst.tolist() == [0, B.LZ_E_INTEGRITY]
        assert torch.equal(out1, ref1) and torch.equal(out1, P1)
        assert torch.equal(out2, ref2) and bool((out2 == 0).all())
    ctx.close()
