"""The method's scalar pieces on the GPU, one by one, against the oracle (bit-exact):
R of Eq. R_nu on 10^7 values of alpha (random, negative, next to integers of alpha 10^13,
special values), Theta of Step 2 for all 256 x 4 inputs, and the iterated map F of
Section 3.1 on random states, at the fixed points and for every integrator format."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import host, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lz():
    need_gpu()
    import paper_1201_3114_amd as lz

    return lz


@pytest.fixture(scope="module")
def ctx(lz):
    return lz.Context(0)


def _cuda(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_R_ten_million(lz, ctx):
    rng = np.random.default_rng(200)
    n = 10_000_000
    parts = [
        rng.uniform(-60.0, 60.0, n // 4),                     # the attractor's range and a bit more
        rng.standard_normal(n // 4) * 1e-6,                     # tiny, both signs
        # alpha = k / 1e13 rounded: alpha 1e13 lands next to the integer k, on either side
        rng.integers(-(5 * 10**14), 5 * 10**14, n // 4).astype(np.float64) / 1e13,
        np.nextafter(rng.integers(-(10**14), 10**14, n // 4).astype(np.float64) / 1e13,
                     rng.choice([-np.inf, np.inf], n // 4)),
    ]
    special = np.array([0.0, -0.0, 1e-13, -1e-13, 5e-14, -5e-14, 1.0, -1.0, 53.6, -53.6, 2.0 ** -60, -(2.0 ** -60)])
    alpha = np.concatenate(parts + [special])
    omega = rng.integers(0, 4, alpha.size, dtype=np.uint8)
    say("R on", alpha.size, "values")
    got = host(lz.unit_r(ctx, _cuda(alpha), _cuda(omega)))
    want = oracle.R_many(alpha, omega)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (bad[:5], alpha[bad[:5]], omega[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_theta_exhaustive(lz, ctx):
    p = np.repeat(np.arange(256, dtype=np.uint8), 4)
    o3 = np.tile(np.arange(4, dtype=np.uint8), 256)
    got = host(lz.unit_theta(ctx, _cuda(p), _cuda(o3)))
    want = oracle.theta_many(p, o3)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert got.max() == 0.255  # the bound 0 <= m_i <= 0.255 of Section 3.2


@pytest.mark.parametrize("integrator,n,steps", [("euler", 1 << 20, 3000), ("euler_fma", 1 << 16, 3000),
                                                ("rk4", 1 << 14, 3000), ("euler", 4096, 1), ("euler", 4096, 7)])
def test_lorenz_random_states(lz, integrator, n, steps):
    """Random states around the attractor (and some far from it) after `steps` steps, bit-exact."""
    rng = np.random.default_rng(210 + n + steps)
    r = np.empty((n, 3))
    r[:, 0] = rng.uniform(-20, 20, n)
    r[:, 1] = rng.uniform(-27, 27, n)
    r[:, 2] = rng.uniform(1, 48, n)
    r[: n // 16] *= rng.uniform(0.5, 1.5, (n // 16, 1))
    c = lz.Context(0, lz.params(integrator=integrator))
    say(integrator, n, "states", steps, "steps")
    got = host(lz.unit_lorenz(c, _cuda(r.copy()), steps))
    want = oracle.lorenz_many(r, 0.01, steps, integrator, nthreads=16)
    c.close()
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("integrator", ["euler", "euler_fma", "rk4"])
def test_lorenz_fixed_points(lz, integrator):
    """The origin is an exact fixed point of every format; C+ and C- = (+-sqrt(beta (rho - 1)), ..., rho - 1),
    rounded to binary64, stay within a few ulps of themselves over 3000 steps, as the oracle's do."""
    q = math.sqrt(8.0 / 3.0 * 27.0)
    r = np.array([[0.0, 0.0, 0.0], [-0.0, 0.0, -0.0], [q, q, 27.0], [-q, -q, 27.0]])
    c = lz.Context(0, lz.params(integrator=integrator))
    got = host(lz.unit_lorenz(c, _cuda(r.copy()), 3000))
    c.close()
    want = oracle.lorenz_many(r, 0.01, 3000, integrator, nthreads=1)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert np.all(got[:2] == 0.0)
    assert np.max(np.abs(got[2:] - r[2:])) < 1e-12


def test_unit_arguments(lz, ctx):
    import torch

    with pytest.raises(ValueError):
        lz.unit_r(ctx, torch.zeros(3, dtype=torch.float32, device="cuda"), torch.zeros(3, dtype=torch.uint8,
                                                                                       device="cuda"))
    with pytest.raises(ValueError):
        lz.unit_lorenz(ctx, torch.zeros(6, dtype=torch.float64, device="cuda"), 5)
    # empty inputs are valid and do nothing
    assert lz.unit_r(ctx, torch.zeros(0, dtype=torch.float64, device="cuda"),
                     torch.zeros(0, dtype=torch.uint8, device="cuda")).numel() == 0
