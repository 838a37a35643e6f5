"""GPU adjoint of eq_pd / eq_fd (hand-written backward kernels through the C
ABI and the autograd.Function wrappers) against the FP64 oracle's analytic
gradients (themselves pinned to FP64 finite differences on the CPU) and
against FP64 central differences of the oracle forward map.

Gate (FP32 gradients vs FP64): normwise relative error per gradient tensor
<= 1e-3; the FD backward touches A^{-1} twice, so its error grows like
cond(A)^2 -- the Rayleigh workloads here have cond(A_c) of order 10."""
import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth
from gpu_util import dev, host, need_gpu, torch

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def nrel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-30))


def _upstream(W, U, seed, with_gs=True):
    rng = np.random.default_rng(seed)
    gz = (rng.standard_normal((W, U)) + 1j * rng.standard_normal((W, U))).astype(np.complex64)
    gs = rng.standard_normal((W, U)).astype(np.float32) if with_gs else None
    return gz, gs


CASES = [
    # W, B, U, offsets
    (16, 32, 4, [0, 16, 32]),
    (9, 64, 16, [0, 16, 40, 64]),
    (5, 48, 17, [0, 24, 48]),
    (6, 96, 32, [0, 32, 64, 96]),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"W{c[0]}B{c[1]}U{c[2]}C{len(c[3]) - 1}")
@pytest.mark.parametrize("with_gs", [False, True])
def test_pd_backward_vs_oracle(case, with_gs):
    from paper_1808_04473_amd import api
    W, B, U, off = case
    b = synth.make_batch(W, B, U, 1, 10.0, "16qam", seed=3 + W, cluster_off=off)
    gz, gs = _upstream(W, U, 7, with_gs)
    gH, gy, gn0 = api.eq_pd_backward(dev(b.H), dev(b.y), b.n0, off, gz=dev(gz),
                                     gs=None if gs is None else dev(gs))
    torch.cuda.synchronize()
    rH, ry, rn0 = oracle.pd_backward(b.H, b.y, b.n0, off, gz, gs)
    eH, ey, en0 = nrel(host(gH), rH), nrel(host(gy), ry), abs(float(gn0) - rn0) / abs(rn0)
    print(f"pd bwd {case[:3]} gs={with_gs}: H {eH:.1e} y {ey:.1e} N0 {en0:.1e}", flush=True)
    assert eH <= TOL and ey <= TOL and en0 <= TOL


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"W{c[0]}B{c[1]}U{c[2]}C{len(c[3]) - 1}")
@pytest.mark.parametrize("user_nu", [False, True])
def test_fd_backward_vs_oracle(case, user_nu):
    from paper_1808_04473_amd import api
    W, B, U, off = case
    C = len(off) - 1
    b = synth.make_batch(W, B, U, 1, 10.0, "16qam", seed=5 + W, cluster_off=off)
    gz, gs = _upstream(W, U, 9, True)
    nu = np.random.default_rng(2).uniform(0.1, 0.9, size=(W, C, U)).astype(np.float32) if user_nu else None
    gH, gy, gn0, gnu = api.eq_fd_backward(dev(b.H), dev(b.y), b.n0, off, gz=dev(gz), gs=dev(gs),
                                          nu=None if nu is None else dev(nu))
    torch.cuda.synchronize()
    rH, ry, rn0, rnu = oracle.fd_backward(b.H, b.y, b.n0, off, gz, gs, nu=nu)
    eH, ey, en0 = nrel(host(gH), rH), nrel(host(gy), ry), abs(float(gn0) - rn0) / abs(rn0)
    print(f"fd bwd {case[:3]} nu={user_nu}: H {eH:.1e} y {ey:.1e} N0 {en0:.1e}", flush=True)
    assert eH <= TOL and ey <= TOL and en0 <= TOL
    if user_nu:
        assert nrel(host(gnu), rnu) <= TOL
    else:
        assert gnu is None


def _config5():
    return synth.config_batch(5)


def test_config5_autograd_mse_vs_oracle():
    """FD, B=256, C=8 x 32, U=16, W=1200, MSE loss on the 16-QAM symbols:
    gradients w.r.t. H, y and N0 through EqFD.backward vs the oracle."""
    from paper_1808_04473_amd.autograd import eq_fd
    b = _config5()
    H = dev(b.H).requires_grad_(True)
    y = dev(b.y).requires_grad_(True)
    n0 = torch.tensor(b.n0, dtype=torch.float32, requires_grad=True)
    s = dev(b.s)
    z, _ = eq_fd(H, y, n0, b.cluster_off)
    loss = torch.mean(torch.abs(z - s) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    zr, _ = oracle.eq_fd(b.H, b.y, b.n0, b.cluster_off)
    gz = 2.0 * (zr - b.s.astype(np.complex128)) / zr.size
    rH, ry, rn0, _ = oracle.fd_backward(b.H, b.y, b.n0, b.cluster_off, gz)
    eH, ey = nrel(host(H.grad), rH), nrel(host(y.grad), ry)
    en0 = abs(float(n0.grad) - rn0) / abs(rn0)
    print(f"config5: H {eH:.1e} y {ey:.1e} N0 {en0:.1e}", flush=True)
    assert eH <= TOL and ey <= TOL and en0 <= TOL


def test_config5_directional_fp64_finite_difference():
    """Directional derivative of the MSE loss along a random direction:
    GPU adjoint vs FP64 central differences (step 1e-6) of the oracle, on a
    16-subcarrier slice of the config-5 workload."""
    from paper_1808_04473_amd.autograd import eq_fd
    b = _config5()
    W = 16
    Hn, yn, sn = b.H[:W], b.y[:W], b.s[:W].astype(np.complex128)
    H = dev(Hn).requires_grad_(True)
    y = dev(yn).requires_grad_(True)
    n0 = torch.tensor(b.n0, dtype=torch.float32, requires_grad=True)
    z, _ = eq_fd(H, y, n0, b.cluster_off)
    loss = torch.mean(torch.abs(z - dev(b.s[:W])) ** 2)
    loss.backward()
    rng = np.random.default_rng(11)
    dH = rng.standard_normal(Hn.shape) + 1j * rng.standard_normal(Hn.shape)
    dy = rng.standard_normal(yn.shape) + 1j * rng.standard_normal(yn.shape)
    dn = 1e-2 * b.n0
    h = 1e-6

    def L(Hx, yx, nx):
        zz, _ = oracle.eq_fd(Hx, yx, nx, b.cluster_off)
        return float(np.mean(np.abs(zz - sn) ** 2))

    H64, y64 = Hn.astype(np.complex128), yn.astype(np.complex128)
    num = (L(H64 + h * dH, y64 + h * dy, b.n0 + h * dn) - L(H64 - h * dH, y64 - h * dy, b.n0 - h * dn)) / (2 * h)
    ana = (np.sum(np.real(np.conj(host(H.grad)) * dH)) + np.sum(np.real(np.conj(host(y.grad)) * dy))
           + float(n0.grad) * dn)
    print(f"directional: fd64 {num:.6e} gpu {ana:.6e}", flush=True)
    assert abs(num - ana) <= TOL * abs(num)


def test_pd_autograd_sigma2_loss():
    """A loss on both outputs (z and sigma2) through EqPD."""
    from paper_1808_04473_amd.autograd import eq_pd
    b = synth.make_batch(20, 64, 8, 2, 5.0, "qpsk", seed=21)
    H = dev(b.H).requires_grad_(True)
    y = dev(b.y).requires_grad_(True)
    n0 = torch.tensor(b.n0, dtype=torch.float32, requires_grad=True)
    z, s2 = eq_pd(H, y, n0, b.cluster_off)
    loss = torch.sum(torch.abs(z) ** 2) + 3.0 * torch.sum(s2)
    loss.backward()
    zr, _ = oracle.eq_pd(b.H, b.y, b.n0, b.cluster_off)
    rH, ry, rn0 = oracle.pd_backward(b.H, b.y, b.n0, b.cluster_off, 2.0 * zr, 3.0 * np.ones(zr.shape))
    assert nrel(host(H.grad), rH) <= TOL
    assert nrel(host(y.grad), ry) <= TOL
    assert abs(float(n0.grad) - rn0) <= TOL * abs(rn0)


def _config5_user_weights(W, C, U, seed=13):
    """Weights near the uniform 1/C, perturbed per (w, c, u), given by the user
    (not renormalised), so the loss depends on each of them (Lemma 1's fusion
    rule with given weights)."""
    rng = np.random.default_rng(seed)
    return ((1.0 + 0.3 * rng.uniform(-1, 1, size=(W, C, U))) / C).astype(np.float32)


def test_config5_user_weights_autograd_vs_oracle():
    """FD at the full config-5 shape (B=256, C=8 x 32, U=16, W=1200) with user
    fusion weights nu and an MSE loss on the 16-QAM symbols: dL/dH, dL/dy,
    dL/dN0 and dL/dnu through EqFD.backward vs the oracle's analytic adjoint."""
    from paper_1808_04473_amd.autograd import eq_fd
    b = _config5()
    W, B, U = b.H.shape
    C = len(b.cluster_off) - 1
    nun = _config5_user_weights(W, C, U)
    H = dev(b.H).requires_grad_(True)
    y = dev(b.y).requires_grad_(True)
    nu = dev(nun).requires_grad_(True)
    n0 = torch.tensor(b.n0, dtype=torch.float32, requires_grad=True)
    z, _ = eq_fd(H, y, n0, b.cluster_off, nu=nu)
    loss = torch.mean(torch.abs(z - dev(b.s)) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    zr, _ = oracle.eq_fd(b.H, b.y, b.n0, b.cluster_off, nu=nun)
    gz = 2.0 * (zr - b.s.astype(np.complex128)) / zr.size
    rH, ry, rn0, rnu = oracle.fd_backward(b.H, b.y, b.n0, b.cluster_off, gz, nu=nun)
    eH, ey, enu = nrel(host(H.grad), rH), nrel(host(y.grad), ry), nrel(host(nu.grad), rnu)
    en0 = abs(float(n0.grad) - rn0) / abs(rn0)
    print(f"config5 user nu: H {eH:.1e} y {ey:.1e} N0 {en0:.1e} nu {enu:.1e}", flush=True)
    assert eH <= TOL and ey <= TOL and en0 <= TOL and enu <= TOL


def test_config5_user_weights_directional_fp64_finite_difference():
    """Directional derivative of the MSE loss along a random direction in
    (H, y, N0, nu) on a 16-subcarrier slice of config 5 with user weights:
    GPU adjoint vs FP64 central differences (step 1e-6) of the oracle."""
    from paper_1808_04473_amd.autograd import eq_fd
    b = _config5()
    W = 16
    _, B, U = b.H.shape
    C = len(b.cluster_off) - 1
    Hn, yn, sn = b.H[:W], b.y[:W], b.s[:W].astype(np.complex128)
    nun = _config5_user_weights(W, C, U, seed=17)
    H = dev(Hn).requires_grad_(True)
    y = dev(yn).requires_grad_(True)
    nu = dev(nun).requires_grad_(True)
    n0 = torch.tensor(b.n0, dtype=torch.float32, requires_grad=True)
    z, _ = eq_fd(H, y, n0, b.cluster_off, nu=nu)
    loss = torch.mean(torch.abs(z - dev(b.s[:W])) ** 2)
    loss.backward()
    rng = np.random.default_rng(19)
    dH = rng.standard_normal(Hn.shape) + 1j * rng.standard_normal(Hn.shape)
    dy = rng.standard_normal(yn.shape) + 1j * rng.standard_normal(yn.shape)
    dnu = rng.standard_normal(nun.shape)
    dn = 1e-2 * b.n0
    h = 1e-6

    def L(Hx, yx, nx, nux):
        zz, _ = oracle.eq_fd(Hx, yx, nx, b.cluster_off, nu=nux)
        return float(np.mean(np.abs(zz - sn) ** 2))

    H64, y64, nu64 = Hn.astype(np.complex128), yn.astype(np.complex128), nun.astype(np.float64)
    num = (L(H64 + h * dH, y64 + h * dy, b.n0 + h * dn, nu64 + h * dnu)
           - L(H64 - h * dH, y64 - h * dy, b.n0 - h * dn, nu64 - h * dnu)) / (2 * h)
    ana = (np.sum(np.real(np.conj(host(H.grad)) * dH)) + np.sum(np.real(np.conj(host(y.grad)) * dy))
           + float(n0.grad) * dn + float(np.sum(host(nu.grad) * dnu)))
    nu_part = float(np.sum(host(nu.grad) * dnu))
    print(f"directional (user nu): fd64 {num:.6e} gpu {ana:.6e} (nu part {nu_part:.3e})", flush=True)
    assert abs(nu_part) > 0.05 * abs(ana)  # the nu direction carries weight in the check
    assert abs(num - ana) <= TOL * abs(num)
