"""Pins of the oracle's analytic adjoints against FP64 central finite
differences (step 1e-6) of the oracle forward maps (no GPU)."""
import numpy as np
import pytest

import oracle

STEP = 1e-6


def _loss(z, s2, cz, cs):
    """A generic real loss touching every output: Re<cz, z> + <cs, s2>."""
    return float(np.sum(np.real(np.conj(cz) * z)) + np.sum(cs * s2))


def _setup(seed, W=2, B=6, U=3):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) * 0.4
    y = rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B))
    cz = rng.standard_normal((W, U)) + 1j * rng.standard_normal((W, U))
    cs = rng.standard_normal((W, U))
    return rng, H, y, cz, cs


def _fd_grad_complex(f, x):
    """Central differences of a real function of a complex array:
    dL/dRe + i dL/dIm for every entry."""
    g = np.zeros_like(x)
    it = np.nditer(np.zeros(x.shape), flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        for part, unit in ((0, 1.0), (1, 1j)):
            xp = x.copy(); xp[idx] += unit * STEP
            xm = x.copy(); xm[idx] -= unit * STEP
            d = (f(xp) - f(xm)) / (2 * STEP)
            g[idx] += d * unit
    return g


@pytest.mark.parametrize("mode", ["pd", "fd", "fd_nu"])
def test_adjoint_vs_finite_differences(mode):
    rng, H, y, cz, cs = _setup(21)
    off = [0, 2, 6]
    n0 = 0.3
    nu = rng.uniform(0.2, 0.8, size=(2, 2, 3)) if mode == "fd_nu" else None

    def fwd(H_, y_, n0_, nu_=nu):
        if mode == "pd":
            z, s2 = oracle.eq_pd(H_, y_, n0_, off)
        else:
            z, s2 = oracle.eq_fd(H_, y_, n0_, off, nu=nu_)
        return _loss(z, s2, cz, cs)

    if mode == "pd":
        gH, gy, gn0 = oracle.pd_backward(H, y, n0, off, cz, cs)
        gnu = None
    else:
        gH, gy, gn0, gnu = oracle.fd_backward(H, y, n0, off, cz, cs, nu=nu)
    nH = _fd_grad_complex(lambda X: fwd(X, y, n0), H)
    ny = _fd_grad_complex(lambda X: fwd(H, X, n0), y)
    nn0 = (fwd(H, y, n0 + STEP) - fwd(H, y, n0 - STEP)) / (2 * STEP)
    np.testing.assert_allclose(gH, nH, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gy, ny, rtol=1e-6, atol=1e-7)
    assert abs(gn0 - nn0) <= 1e-6 * max(1.0, abs(nn0))
    if mode == "fd_nu":
        nnu = np.zeros_like(nu)
        it = np.nditer(np.zeros(nu.shape), flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            p = nu.copy(); p[i] += STEP
            m = nu.copy(); m[i] -= STEP
            nnu[i] = (fwd(H, y, n0, p) - fwd(H, y, n0, m)) / (2 * STEP)
        np.testing.assert_allclose(gnu, nnu, rtol=1e-6, atol=1e-7)
    else:
        assert gnu is None


def test_adjoint_directional_full_shape():
    """Random-direction directional derivative at the B=256, C=8, U=16 shape
    (W=2 slice) of the FD equaliser with an MSE loss on the symbols."""
    rng = np.random.default_rng(22)
    W, B, U = 2, 256, 16
    off = list(range(0, 257, 32))
    H = (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) * np.sqrt(0.5 / B)
    s = (rng.choice([-3, -1, 1, 3], size=(W, U)) + 1j * rng.choice([-3, -1, 1, 3], size=(W, U))) / np.sqrt(10)
    y = (H @ s[..., None])[..., 0] + 0.05 * (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B)))
    n0 = 6.25e-3

    def loss(H_, y_, n0_):
        z, _ = oracle.eq_fd(H_, y_, n0_, off)
        return float(np.mean(np.abs(z - s) ** 2))

    z, _ = oracle.eq_fd(H, y, n0, off)
    gz = 2.0 * (z - s) / z.size
    gH, gy, gn0, _ = oracle.fd_backward(H, y, n0, off, gz)
    dH = rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape)
    dy = rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)
    dn = 1e-3
    num = (loss(H + STEP * dH, y + STEP * dy, n0 + STEP * dn)
           - loss(H - STEP * dH, y - STEP * dy, n0 - STEP * dn)) / (2 * STEP)
    ana = (np.sum(np.real(np.conj(gH) * dH)) + np.sum(np.real(np.conj(gy) * dy)) + gn0 * dn)
    assert abs(num - ana) <= 1e-6 * abs(ana) + 1e-12
