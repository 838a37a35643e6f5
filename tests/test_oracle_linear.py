"""Pins of the MRC / ZF / unbiased L-MMSE oracle (Section III-A, Section IV-A,
Lemma 4) to what the mathematics fixes: noise-free recovery, explicit loops
on tiny inputs, Monte-Carlo error variances and gains, exact identities and
closed forms, and the finite-size expectation behind Lemma 4."""
import numpy as np
import pytest

import oracle


def _h(rng, W, B, U):
    return (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) / np.sqrt(2 * B)


def test_zf_recovers_symbols_without_noise():
    """y = H s exactly: ZF returns s (PD, and FD with every B_c >= U)."""
    rng = np.random.default_rng(1)
    H = _h(rng, 6, 24, 5)
    s = rng.choice([-1, 1], (6, 5)) + 1j * rng.choice([-1, 1], (6, 5))
    y = (H @ s[..., None])[..., 0]
    off = [0, 8, 14, 24]
    for fn in (oracle.eq_pd_linear, oracle.eq_fd_linear):
        z, _ = fn(H, y, 1e-3, off, "zf")
        np.testing.assert_allclose(z, s, atol=1e-10)


def test_mrc_explicit_loops():
    """MRC estimate and the per-user form of its variance,
    sigma2_u = N0 / G_uu + E_s sum_{k != u} |G_uk|^2 / G_uu^2, by loops."""
    rng = np.random.default_rng(2)
    H = _h(rng, 2, 7, 3)
    y = rng.standard_normal((2, 7)) + 1j * rng.standard_normal((2, 7))
    n0, es = 0.3, 1.7
    z, s2 = oracle.eq_pd_linear(H, y, n0, [0, 3, 7], "mrc", es=es)
    for w in range(2):
        for u in range(3):
            guu = sum(abs(H[w, b, u]) ** 2 for b in range(7))
            num = sum(np.conj(H[w, b, u]) * y[w, b] for b in range(7))
            assert abs(z[w, u] - num / guu) < 1e-12
            off = 0.0
            for k in range(3):
                if k != u:
                    guk = sum(np.conj(H[w, b, u]) * H[w, b, k] for b in range(7))
                    off += abs(guk) ** 2
            assert abs(s2[w, u] - (n0 / guu + es * off / guu ** 2)) < 1e-12


@pytest.mark.parametrize("kind", ["zf", "mrc", "lmmse_unbiased"])
def test_error_variance_monte_carlo(kind):
    """E|z - s|^2 over symbols and noise for one fixed H matches the
    Section III-A variance (ZF: noise only; MRC and unbiased L-MMSE: noise
    and interference)."""
    rng = np.random.default_rng(3)
    B, U, N, n0 = 10, 3, 200000, 0.2
    H = _h(rng, 1, B, U)[0]
    s = (rng.choice([-1, 1], (N, U)) + 1j * rng.choice([-1, 1], (N, U))) / np.sqrt(2)
    n = (rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))) * np.sqrt(n0 / 2)
    y = s @ H.T + n
    Hb = np.broadcast_to(H, (N, B, U))
    z, _ = oracle.eq_pd_linear(Hb, y, n0, [0, B], kind)
    _, s2 = oracle.eq_pd_linear(H[None], y[:1], n0, [0, B], kind)
    emp = np.mean(np.abs(z - s) ** 2, axis=0)
    np.testing.assert_allclose(emp, s2[0], rtol=0.02)


def test_fd_mrc_with_gram_weights_equals_pd_mrc():
    """With nu_{c,u} = [G_c]_uu / sum_c' [G_c']_uu the fused MRC estimate is
    exactly the PD MRC estimate (sum_c y_c^MRC / sum_c [G_c]_uu)."""
    rng = np.random.default_rng(4)
    H = _h(rng, 5, 30, 4)
    y = rng.standard_normal((5, 30)) + 1j * rng.standard_normal((5, 30))
    off = [0, 6, 19, 30]
    Gc, _ = oracle.local_statistics(H, y, off)
    d = np.real(np.diagonal(Gc, axis1=-2, axis2=-1))
    nu = d / d.sum(axis=1, keepdims=True)
    zf, _ = oracle.eq_fd_linear(H, y, 0.1, off, "mrc", nu=nu)
    zp, _ = oracle.eq_pd_linear(H, y, 0.1, off, "mrc")
    np.testing.assert_allclose(zf, zp, rtol=1e-12)


@pytest.mark.parametrize("kind", ["zf", "mrc", "lmmse", "lmmse_unbiased"])
def test_one_cluster_fd_equals_pd(kind):
    rng = np.random.default_rng(5)
    H = _h(rng, 4, 12, 3)
    y = rng.standard_normal((4, 12)) + 1j * rng.standard_normal((4, 12))
    zp, sp = oracle.eq_pd_linear(H, y, 0.05, [0, 12], kind)
    zf, sf = oracle.eq_fd_linear(H, y, 0.05, [0, 12], kind)
    np.testing.assert_allclose(zf, zp, rtol=1e-12)
    np.testing.assert_allclose(sf, sp, rtol=1e-12)


def test_lmmse_kind_is_the_lmmse_oracle():
    rng = np.random.default_rng(6)
    H = _h(rng, 3, 16, 4)
    y = rng.standard_normal((3, 16)) + 1j * rng.standard_normal((3, 16))
    z1, s1 = oracle.eq_pd_linear(H, y, 0.1, [0, 8, 16], "lmmse")
    z2, s2 = oracle.eq_pd(H, y, 0.1, [0, 8, 16])
    np.testing.assert_allclose(z1, z2, rtol=1e-13)
    np.testing.assert_allclose(s1, s2, rtol=1e-13)


def test_fd_zf_sinr_finite_size_expectation():
    """Lemma 4: the post-fusion ZF SINR is (E_s/N0)(1 - C beta) in the large
    system.  For finite Rayleigh H ~ CN(0, 1/B) it is exact in expectation
    with one more degree of freedom per cluster: 1 / [G_c^{-1}]_uu is
    Gamma(B_c - U + 1, 1/B), so E[E_s / sigma2_FD] = (E_s/N0) sum_c
    (B_c - U + 1) / B."""
    rng = np.random.default_rng(7)
    W, B, U, C, n0 = 3000, 64, 8, 4, 0.5
    H = _h(rng, W, B, U)
    y = np.zeros((W, B), complex)
    off = [0, 16, 32, 48, 64]
    _, s2 = oracle.eq_fd_linear(H, y, n0, off, "zf")
    sinr = np.mean(1.0 / s2)
    expect = (1.0 / n0) * sum((off[c + 1] - off[c] - U + 1) / B for c in range(C))
    assert abs(sinr / expect - 1) < 0.01, (sinr, expect)
    # and Lemma 4's large-system value is the limit of that expectation
    assert abs(expect * n0 - (1 - C * U / B) - C / B) < 1e-12


def test_unbiased_gain_identity():
    """(G + rho I)^{-1} G = I - rho (G + rho I)^{-1}, so the gain of the biased
    L-MMSE estimate is mu_u = 1 - rho d_u = 1 - sigma2_u / E_s; the unbiased
    estimate is z_u / mu_u with variance sigma2_u / mu_u (both from the
    biased L-MMSE oracle), and E_s / sigma2_unbiased = E_s / sigma2 - 1."""
    rng = np.random.default_rng(7)
    H = _h(rng, 6, 20, 5)
    y = rng.standard_normal((6, 20)) + 1j * rng.standard_normal((6, 20))
    n0, es = 0.08, 1.3
    G = np.conj(np.swapaxes(H, 1, 2)) @ H
    zb, sb = oracle.eq_pd(H, y, n0, [0, 20], es=es)
    mu = oracle.lmmse_unbiased_gain(G, n0, es)
    np.testing.assert_allclose(mu, 1.0 - sb / es, rtol=1e-12)
    zu, su = oracle.eq_pd_linear(H, y, n0, [0, 9, 20], "lmmse_unbiased", es=es)
    np.testing.assert_allclose(zu, zb / mu, rtol=1e-11)
    np.testing.assert_allclose(su, sb / mu, rtol=1e-11)
    np.testing.assert_allclose(es / su, es / sb - 1.0, rtol=1e-10)


def test_unbiased_orthogonal_columns_is_zf():
    """H^H H = alpha I: mu = alpha / (alpha + rho), so the unbiased L-MMSE
    estimate is y^MRC / alpha with variance N0 / alpha, the ZF result."""
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 4)) + 1j * rng.standard_normal((12, 4)))
    H = (1.7 * Q)[None]
    y = (rng.standard_normal(12) + 1j * rng.standard_normal(12))[None]
    n0 = 0.3
    z, s2 = oracle.eq_pd_linear(H, y, n0, [0, 12], "lmmse_unbiased")
    m = (np.conj(H[0]).T @ y[0])
    np.testing.assert_allclose(z[0], m / 1.7 ** 2, rtol=1e-12)
    np.testing.assert_allclose(s2[0], np.full(4, n0 / 1.7 ** 2), rtol=1e-12)
    zz, sz = oracle.eq_pd_linear(H, y, n0, [0, 12], "zf")
    np.testing.assert_allclose(z, zz, rtol=1e-12)
    np.testing.assert_allclose(s2, sz, rtol=1e-12)


def test_unbiased_unit_gain_monte_carlo():
    """Regressing the estimate of user u on its symbol over symbols and noise
    gives slope 1 for the unbiased estimate and mu_u for the biased one."""
    rng = np.random.default_rng(9)
    B, U, N, n0 = 8, 3, 200000, 0.4
    H = _h(rng, 1, B, U)[0]
    s = (rng.choice([-1, 1], (N, U)) + 1j * rng.choice([-1, 1], (N, U))) / np.sqrt(2)
    n = (rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))) * np.sqrt(n0 / 2)
    y = s @ H.T + n
    Hb = np.broadcast_to(H, (N, B, U))
    zu, _ = oracle.eq_pd_linear(Hb, y, n0, [0, B], "lmmse_unbiased")
    zb, _ = oracle.eq_pd_linear(Hb, y, n0, [0, B], "lmmse")
    mu = oracle.lmmse_unbiased_gain(np.conj(H).T @ H, n0)
    assert np.all(mu < 0.95)
    slope_u = np.sum(np.conj(s) * zu, axis=0) / np.sum(np.abs(s) ** 2, axis=0)
    slope_b = np.sum(np.conj(s) * zb, axis=0) / np.sum(np.abs(s) ** 2, axis=0)
    np.testing.assert_allclose(slope_u, np.ones(U), atol=0.01)
    np.testing.assert_allclose(slope_b, mu, atol=0.01)
