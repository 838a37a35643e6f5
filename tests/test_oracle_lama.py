"""Pins of the LAMA oracle (Algorithm 1, eq. (F), Theorem 1, Lemma 2, Theorem 3):
the QPSK posterior mean in closed form, the denoiser's limits, the original
H-domain LAMA of the derivation of Algorithm 1, the first iteration, FD with
one cluster, the state evolution of Theorem 1 on a large system, and LAMA-FD
with several clusters against the normalised cluster systems of the proof of
Lemma 2 and their per-cluster state evolution."""
import numpy as np
import pytest

import oracle


def _h(rng, W, B, U):
    return (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) / np.sqrt(2 * B)


def test_qam_points_energy_and_mean():
    for order in (4, 16, 64):
        p = oracle.qam_points(order, es=2.5)
        assert len(p) == order
        assert abs(np.mean(p)) < 1e-12
        assert abs(np.mean(np.abs(p) ** 2) - 2.5) < 1e-12


def test_qpsk_posterior_in_closed_form():
    """QPSK points (+-a +- ja), a = sqrt(E_s/2): per real dimension the
    posterior mean is a tanh(2 a x / tau), the variance a^2 - mean^2."""
    rng = np.random.default_rng(1)
    es, tau = 1.3, 0.7
    a = np.sqrt(es / 2)
    z = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    F, G = oracle.posterior_mean_var(z, np.full(50, tau), oracle.qam_points(4, es))
    fr, fi = a * np.tanh(2 * a * z.real / tau), a * np.tanh(2 * a * z.imag / tau)
    np.testing.assert_allclose(F, fr + 1j * fi, atol=1e-12)
    np.testing.assert_allclose(G, 2 * a * a - fr ** 2 - fi ** 2, atol=1e-12)


def test_denoiser_limits():
    """Large tau: prior mean 0 and variance E_s.  Small tau: the nearest
    constellation point with zero variance."""
    pts = oracle.qam_points(16)
    rng = np.random.default_rng(2)
    z = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    F, G = oracle.posterior_mean_var(z, np.full(40, 1e9), pts)
    np.testing.assert_allclose(F, 0, atol=1e-8)
    np.testing.assert_allclose(G, 1.0, atol=1e-8)
    s = pts[rng.integers(0, 16, 40)]
    F, G = oracle.posterior_mean_var(s + 0.01 * z, np.full(40, 1e-4), pts)
    np.testing.assert_allclose(F, s, atol=1e-12)
    np.testing.assert_allclose(G, 0, atol=1e-12)


@pytest.mark.parametrize("order", [4, 16])
def test_lama_pd_equals_original_lama(order):
    """The derivation of Algorithm 1: LAMA-PD on (H^H H, H^H y) gives the
    estimates and variances of the original LAMA on (H, y), every iteration."""
    rng = np.random.default_rng(3)
    W, B, U = 20, 64, 16
    H = _h(rng, W, B, U)
    pts = oracle.qam_points(order)
    s = pts[rng.integers(0, order, (W, U))]
    n0 = 0.05
    y = (H @ s[..., None])[..., 0] + np.sqrt(n0 / 2) * (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B)))
    G = np.conj(np.swapaxes(H, 1, 2)) @ H
    m = (np.conj(np.swapaxes(H, 1, 2)) @ y[..., None])[..., 0]
    for T in (1, 2, 3, 6):
        z1, s1 = oracle.lama_pd(G, m, n0, U / B, T, pts)
        z2, s2 = oracle.lama_original(H, y, n0, T, pts)
        np.testing.assert_allclose(z1, z2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(s1, s2, rtol=1e-12)


def test_first_iteration_is_the_matched_filter():
    rng = np.random.default_rng(4)
    H = _h(rng, 5, 32, 4)
    y = rng.standard_normal((5, 32)) + 1j * rng.standard_normal((5, 32))
    z, s2 = oracle.eq_pd_lama(H, y, 0.2, [0, 16, 32], 1, 16, es=1.0)
    m = (np.conj(np.swapaxes(H, 1, 2)) @ y[..., None])[..., 0]
    np.testing.assert_allclose(z, m, rtol=1e-13)
    np.testing.assert_allclose(s2, 0.2 + (4 / 32) * 1.0, rtol=1e-13)


def test_fd_one_cluster_equals_pd():
    rng = np.random.default_rng(5)
    H = _h(rng, 6, 48, 8)
    y = rng.standard_normal((6, 48)) + 1j * rng.standard_normal((6, 48))
    zp, sp = oracle.eq_pd_lama(H, y, 0.1, [0, 48], 4, 16)
    zf, sf = oracle.eq_fd_lama(H, y, 0.1, [0, 48], 4, 16)
    np.testing.assert_allclose(zf, zp, rtol=1e-12)
    np.testing.assert_allclose(sf, sp, rtol=1e-12)


def _psi(sigma2, pts, rng, n=400000):
    """Monte-Carlo MSE function of eq. (SE_MSEpsi)."""
    S = pts[rng.integers(0, len(pts), n)]
    Z = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    F, _ = oracle.posterior_mean_var(S + np.sqrt(sigma2) * Z, np.full(n, sigma2), pts)
    return float(np.mean(np.abs(F - S) ** 2))


def test_state_evolution_tracks_lama_pd():
    """Theorem 1 on a large Rayleigh system (B = 512, U = 64, QPSK): the
    variance N0 + beta phi^t that LAMA-PD carries, and the empirical MSE of
    z^t, follow sigma_t^2 = N0 + beta Psi(sigma_{t-1}^2), sigma_1^2 = N0 + beta E_s."""
    rng = np.random.default_rng(6)
    W, B, U, n0 = 40, 512, 64, 0.1
    pts = oracle.qam_points(4)
    H = _h(rng, W, B, U)
    s = pts[rng.integers(0, 4, (W, U))]
    y = (H @ s[..., None])[..., 0] + np.sqrt(n0 / 2) * (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B)))
    beta = U / B
    se = [n0 + beta * 1.0]
    for _ in range(4):
        se.append(n0 + beta * _psi(se[-1], pts, rng))
    Gm = np.conj(np.swapaxes(H, 1, 2)) @ H
    m = (np.conj(np.swapaxes(H, 1, 2)) @ y[..., None])[..., 0]
    _, _, trace = oracle.lama_pd(Gm, m, n0, beta, 5, pts, return_trace=True)
    for t, (z, s2) in enumerate(trace):
        emp = np.mean(np.abs(z - s) ** 2)
        assert abs(np.mean(s2) / se[t] - 1) < 0.05, (t, np.mean(s2), se[t])
        assert abs(emp / se[t] - 1) < 0.08, (t, emp, se[t])


# ---- LAMA-FD with several clusters: the per-cluster normalisation of the
#      proof of Lemma 2, pinned against the H-domain LAMA and Theorem 1.

def _large_system(rng, order, n0, W=40, B=512, U=64):
    pts = oracle.qam_points(order)
    H = _h(rng, W, B, U)
    s = pts[rng.integers(0, order, (W, U))]
    y = (H @ s[..., None])[..., 0] + np.sqrt(n0 / 2) * (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B)))
    return H, y, s, pts


FD_PARTITIONS = {"C2_w_quarter_three_quarters": [0, 128, 512], "C4_uniform": [0, 128, 256, 384, 512]}


@pytest.mark.parametrize("order", [4, 16])
@pytest.mark.parametrize("part", list(FD_PARTITIONS))
def test_fd_lama_clusters_equal_lama_on_normalised_cluster_systems(order, part):
    """Each cluster's LAMA is the original H-domain LAMA (pinned to Algorithm 1
    above) run on the cluster's own system scaled by 1/sqrt(w_c): channel
    H_c / sqrt(w_c) (entries of variance 1/B_c, so that its system ratio is
    U/B_c), receive vector y_c / sqrt(w_c) and noise variance N0 / w_c (proof
    of Lemma 2).  The normalised system is built here from H and y directly,
    not from the oracle's scaled statistics, so a mis-scaled N0 or beta in the
    oracle's cluster iteration fails this test."""
    off = FD_PARTITIONS[part]
    rng = np.random.default_rng(7)
    n0 = 0.1 if order == 4 else 0.02
    H, y, _, pts = _large_system(rng, order, n0, W=8)
    B = H.shape[1]
    T = 5
    _, _, z_c, s2_c, _ = oracle.eq_fd_lama(H, y, n0, off, T, order, return_clusters=True)
    for c in range(len(off) - 1):
        wc = (off[c + 1] - off[c]) / B
        Hc = H[:, off[c]:off[c + 1]] / np.sqrt(wc)
        yc = y[:, off[c]:off[c + 1]] / np.sqrt(wc)
        z_ref, s2_ref = oracle.lama_original(Hc, yc, n0 / wc, T, pts)
        np.testing.assert_allclose(z_c[:, c], z_ref, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(s2_c[:, c], s2_ref, rtol=1e-12)


@pytest.mark.parametrize("order", [4, 16])
@pytest.mark.parametrize("part", list(FD_PARTITIONS))
def test_fd_lama_state_evolution_per_cluster(order, part):
    """Theorem 1 applied to cluster c of the normalised relation (proof of
    Lemma 2): the variance that cluster's iteration carries, N0/w_c +
    (beta/w_c) phi_c^t, and the empirical MSE of its estimate z_c^t follow
    sigma_{c,1}^2 = (N0 + beta E_s)/w_c, sigma_{c,t+1}^2 = (N0 + beta
    Psi(sigma_{c,t}^2))/w_c, within 5% / 8% (B = 512, U = 64; w = (1/4, 3/4)
    and four equal clusters).  The fused variance is (sum_c 1/sigma_c^2)^{-1}
    (Theorem 3), and the empirical MSE of the fused estimate follows it."""
    off = FD_PARTITIONS[part]
    rng = np.random.default_rng(7)
    n0 = 0.1 if order == 4 else 0.02
    H, y, s, pts = _large_system(rng, order, n0)
    W, B, U = H.shape
    beta, T = U / B, 5
    z, s2, _, s2_c, traces = oracle.eq_fd_lama(H, y, n0, off, T, order, return_clusters=True)
    for c in range(len(off) - 1):
        wc = (off[c + 1] - off[c]) / B
        se = [(n0 + beta * 1.0) / wc]
        for _ in range(T - 1):
            se.append((n0 + beta * _psi(se[-1], pts, rng)) / wc)
        for t, (zt, st) in enumerate(traces[c]):
            emp = np.mean(np.abs(zt - s) ** 2)
            assert abs(np.mean(st) / se[t] - 1) < 0.05, (c, t, np.mean(st), se[t])
            assert abs(emp / se[t] - 1) < 0.08, (c, t, emp, se[t])
    fused = 1.0 / np.sum(1.0 / s2_c, axis=1)
    np.testing.assert_allclose(s2, np.repeat(fused[:, None], U, axis=1), rtol=1e-12)
    assert abs(np.mean(np.abs(z - s) ** 2) / np.mean(fused) - 1) < 0.08
