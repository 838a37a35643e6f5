"""Pins of the FP64 oracle's forward equalisers against what the paper and the
mathematics fix (no GPU).  Each test states the passage or identity it pins."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _rand_system(W, B, U, seed, scale=None):
    rng = np.random.default_rng(seed)
    sd = math.sqrt(0.5 / B) if scale is None else scale
    H = (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) * sd
    y = rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B))
    return H, y


# ---------------------------------------------------------------- worked examples
@pytest.mark.parametrize("name", ["WE1", "WE2"])
def test_worked_examples(name):
    """Hand-derived rational examples (orthogonal clusters), tests/golden."""
    ex = json.load(open(GOLDEN))[name]
    H = (np.array(ex["H_re"]) + 1j * np.array(ex["H_im"]))[None]
    y = (np.array(ex["y_re"]) + 1j * np.array(ex["y_im"]))[None]
    off = ex["cluster_off"]
    z, s2 = oracle.eq_pd(H, y, ex["n0"], off)
    np.testing.assert_allclose(z[0], np.array(ex["pd_z_re"]) + 1j * np.array(ex["pd_z_im"]), atol=1e-14)
    np.testing.assert_allclose(s2[0], ex["pd_sigma2"], atol=1e-14)
    z, s2, loc = oracle.eq_fd(H, y, ex["n0"], off, return_local=True)
    np.testing.assert_allclose(z[0], np.array(ex["fd_z_re"]) + 1j * np.array(ex["fd_z_im"]), atol=1e-14)
    np.testing.assert_allclose(s2[0], ex["fd_sigma2"], atol=1e-14)
    np.testing.assert_allclose(loc["nu"][0], ex["fd_nu"], atol=1e-14)


# ---------------------------------------------------------------- PD = centralised
@pytest.mark.parametrize("B,U", [(2, 1), (4, 2), (8, 3), (6, 4), (3, 5)])
def test_pd_push_through_identity(B, U):
    """L-MMSE from the Wiener-filter form z = E_s H^H (E_s H H^H + N0 I_B)^{-1} y,
    an independent B-space formula, equals (G + rho I)^{-1} H^H y (Section III-A).
    Covers U > B (underdetermined), which L-MMSE allows."""
    H, y = _rand_system(5, B, U, seed=B * 10 + U)
    for n0, es in [(0.3, 1.0), (0.05, 2.0)]:
        z, _ = oracle.eq_pd(H, y, n0, [0, B], es=es)
        Cyy = es * H @ np.conj(np.swapaxes(H, 1, 2)) + n0 * np.eye(B)
        z_ref = es * (np.conj(np.swapaxes(H, 1, 2)) @ np.linalg.solve(Cyy, y[..., None]))[..., 0]
        np.testing.assert_allclose(z, z_ref, rtol=1e-11, atol=1e-12)


def test_pd_partition_invariance():
    """PD delivers exactly the centralised estimate for any partition
    (Section III-A, "same estimates"), including one antenna per cluster."""
    H, y = _rand_system(7, 12, 3, seed=1)
    z0, s0 = oracle.eq_centralized(H, y, 0.1)
    for off in ([0, 12], [0, 5, 12], [0, 1, 2, 7, 12], list(range(13))):
        z, s2 = oracle.eq_pd(H, y, 0.1, off)
        np.testing.assert_allclose(z, z0, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(s2, s0, rtol=1e-12)


def test_gram_sum_equals_full_gram():
    """sum_c G_c = H^H H and sum_c y_c^MRC = H^H y (eq. (fullMRC))."""
    H, y = _rand_system(4, 10, 3, seed=2)
    Gc, mc = oracle.local_statistics(H, y, [0, 3, 4, 10])
    np.testing.assert_allclose(Gc.sum(1), np.conj(np.swapaxes(H, 1, 2)) @ H, atol=1e-13)
    np.testing.assert_allclose(mc.sum(1), np.einsum("wbu,wb->wu", np.conj(H), y), atol=1e-13)
    # Hermitian local Grams
    np.testing.assert_allclose(Gc, np.conj(np.swapaxes(Gc, -1, -2)), atol=1e-15)


def test_gram_brute_force_loops():
    """Local statistics against element-by-element Python loops on a tiny case."""
    H, y = _rand_system(2, 5, 2, seed=3)
    off = [0, 2, 5]
    Gc, mc = oracle.local_statistics(H, y, off)
    for w in range(2):
        for c in range(2):
            for i in range(2):
                acc_m = 0j
                for b in range(off[c], off[c + 1]):
                    acc_m += np.conj(H[w, b, i]) * y[w, b]
                assert abs(mc[w, c, i] - acc_m) < 1e-14
                for j in range(2):
                    acc = 0j
                    for b in range(off[c], off[c + 1]):
                        acc += np.conj(H[w, b, i]) * H[w, b, j]
                    assert abs(Gc[w, c, i, j] - acc) < 1e-14


def test_lmmse_estimate_brute_force_2x2():
    """2x2 Hermitian inverse written out by Cramer's rule."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, 2)) + 1j * rng.standard_normal((3, 2))
    G = (np.conj(X.T) @ X)[None]
    m = (rng.standard_normal(2) + 1j * rng.standard_normal(2))[None]
    rho = 0.7
    a, b, c, d = G[0, 0, 0] + rho, G[0, 0, 1], G[0, 1, 0], G[0, 1, 1] + rho
    det = a * d - b * c
    inv = np.array([[d, -b], [-c, a]]) / det
    np.testing.assert_allclose(oracle.lmmse_estimate(G, m, rho)[0], inv @ m[0], rtol=1e-13)
    np.testing.assert_allclose(oracle.lmmse_error_variance_simplified(G, rho)[0],
                               rho * np.real(np.diag(inv)), rtol=1e-13)


# ---------------------------------------------------------------- error variance
def test_error_variance_literal_equals_simplified():
    """Section III-A variance equals N0 diag((G + rho I)^{-1}) when rho = N0/E_s,
    and not otherwise (so the check has teeth)."""
    H, y = _rand_system(6, 9, 4, seed=5)
    G = np.conj(np.swapaxes(H, 1, 2)) @ H
    for n0, es in [(0.2, 1.0), (0.01, 1.0), (0.5, 3.0)]:
        a = oracle.lmmse_error_variance(G, n0, es)
        b = oracle.lmmse_error_variance_simplified(G, n0, es)
        np.testing.assert_allclose(a, b, rtol=1e-12)
    # a mismatched regulariser breaks the identity
    U = G.shape[-1]
    Wm = np.linalg.inv(G + 0.5 * np.eye(U))
    WG = Wm @ G
    S = Wm @ G @ np.conj(np.swapaxes(Wm, 1, 2)) * 0.2 + (WG - np.eye(U)) @ np.conj(np.swapaxes(WG - np.eye(U), 1, 2))
    assert np.max(np.abs(np.real(np.diagonal(S, axis1=1, axis2=2)) - oracle.lmmse_error_variance(G, 0.2))) > 1e-3


def test_error_variance_monte_carlo():
    """sigma^2 is the error variance E|z - s0|^2 of the estimate for a fixed H
    (Section II-A definition), checked by Monte Carlo over QPSK symbols and noise."""
    rng = np.random.default_rng(6)
    B, U, n0 = 8, 4, 0.3
    H = (rng.standard_normal((B, U)) + 1j * rng.standard_normal((B, U))) * math.sqrt(0.5 / B)
    N = 60000
    pts = synth.constellation("qpsk")
    s = pts[rng.integers(0, 4, size=(N, U))]
    n = (rng.standard_normal((N, B)) + 1j * rng.standard_normal((N, B))) * math.sqrt(n0 / 2)
    y = s @ H.T + n
    Hb = np.broadcast_to(H, (N, B, U))
    z, s2 = oracle.eq_pd(Hb, y, n0, [0, B])
    mse = np.mean(np.abs(z - s) ** 2, axis=0)
    # relative standard error of a mean of ~chi2 samples is about sqrt(2/N)
    np.testing.assert_allclose(mse, s2[0], rtol=6 * math.sqrt(2.0 / N) + 5e-3)


def test_noise_free_limit_recovers_symbols():
    """As N0 -> 0 L-MMSE tends to ZF (Section III-A), which inverts y = H s exactly."""
    rng = np.random.default_rng(7)
    W, B, U = 4, 16, 4
    H = (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) * math.sqrt(0.5 / B)
    s = synth.constellation("16qam")[rng.integers(0, 16, size=(W, U))]
    y = (H @ s[..., None])[..., 0]
    z, s2 = oracle.eq_pd(H, y, 1e-12, [0, 8, 16])
    np.testing.assert_allclose(z, s, atol=1e-9)
    assert np.all(s2 < 1e-10)


# ---------------------------------------------------------------- FD
def test_fd_single_cluster_equals_pd():
    """FD and PD coincide for C = 1 (proof of Lemma 3)."""
    H, y = _rand_system(5, 8, 3, seed=8)
    zp, sp = oracle.eq_pd(H, y, 0.2, [0, 8])
    zf, sf = oracle.eq_fd(H, y, 0.2, [0, 8])
    np.testing.assert_allclose(zf, zp, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(sf, sp, rtol=1e-13)


def test_fd_weights_and_fused_variance():
    """Weights sum to one (Definition 3) and the fused variance of the optimal
    weights equals (sum_c sigma_c^-2)^-1 (Theorem 3)."""
    H, y = _rand_system(5, 12, 3, seed=9)
    z, s2, loc = oracle.eq_fd(H, y, 0.2, [0, 3, 7, 12], return_local=True)
    np.testing.assert_allclose(loc["nu"].sum(axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(s2, 1.0 / np.sum(1.0 / loc["s2_c"], axis=1), rtol=1e-13)
    np.testing.assert_allclose(z, np.sum(loc["nu"] * loc["z_c"], axis=1), rtol=1e-14)


def test_fd_optimal_weights_minimise_variance():
    """Lemma 1: no other weights with sum 1 give a smaller sum nu^2 sigma_c^2."""
    rng = np.random.default_rng(10)
    s2c = rng.uniform(0.1, 2.0, size=(200, 4, 3))
    nu = oracle.optimal_fusion_weights(s2c)
    best = np.sum(nu * nu * s2c, axis=1)
    for _ in range(20):
        d = rng.standard_normal(nu.shape) * 0.05
        d -= d.mean(axis=1, keepdims=True)
        assert np.all(np.sum((nu + d) ** 2 * s2c, axis=1) >= best - 1e-15)


def test_fd_orthogonal_cluster_closed_form():
    """If H_c^H H_c = alpha_c I: z_PD = m/(sum alpha + rho), z_FD = m/(sum alpha + C rho),
    sigma2_FD = N0 / sum_c (alpha_c + rho)."""
    rng = np.random.default_rng(11)
    U, Bc, C, n0 = 3, 5, 3, 0.4
    alphas = np.array([0.5, 1.0, 2.5])
    blocks = []
    for c in range(C):
        Q, _ = np.linalg.qr(rng.standard_normal((Bc, U)) + 1j * rng.standard_normal((Bc, U)))
        blocks.append(math.sqrt(alphas[c]) * Q)
    H = np.concatenate(blocks, 0)[None]
    y = (rng.standard_normal(C * Bc) + 1j * rng.standard_normal(C * Bc))[None]
    off = [0, Bc, 2 * Bc, 3 * Bc]
    m = np.conj(H[0].T) @ y[0]
    zp, sp = oracle.eq_pd(H, y, n0, off)
    zf, sf = oracle.eq_fd(H, y, n0, off)
    np.testing.assert_allclose(zp[0], m / (alphas.sum() + n0), rtol=1e-12)
    np.testing.assert_allclose(sp[0], n0 / (alphas.sum() + n0), rtol=1e-12)
    np.testing.assert_allclose(zf[0], m / (alphas.sum() + C * n0), rtol=1e-12)
    np.testing.assert_allclose(sf[0], n0 / np.sum(alphas + n0), rtol=1e-12)


def test_fd_user_weights_used_as_given():
    """User-supplied weights enter eq. (fusionrule) unnormalised."""
    H, y = _rand_system(3, 8, 2, seed=12)
    off = [0, 4, 8]
    nu = np.full((3, 2, 2), 0.3)
    z, s2, loc = oracle.eq_fd(H, y, 0.2, off, nu=nu, return_local=True)
    np.testing.assert_allclose(z, 0.3 * loc["z_c"].sum(axis=1), rtol=1e-14)
    np.testing.assert_allclose(s2, 0.09 * loc["s2_c"].sum(axis=1), rtol=1e-14)


# ---------------------------------------------------------------- condition estimate
def test_cond_estimate_is_upper_bound():
    rng = np.random.default_rng(13)
    X = rng.standard_normal((50, 12, 5)) + 1j * rng.standard_normal((50, 12, 5))
    A = np.conj(np.swapaxes(X, 1, 2)) @ X + 1e-2 * np.eye(5)
    k = oracle.cond_estimate(A)
    assert np.all(k >= np.linalg.cond(A) * (1 - 1e-12))
    assert np.all(k <= 5 * 5 * np.linalg.cond(A))
    # exact for a scaled identity; diagonal case is ||A||_1 * sum 1/a_i
    D = np.diag([1.0, 10.0, 100.0]).astype(complex)[None]
    np.testing.assert_allclose(oracle.cond_estimate(D), 100.0 * 1.11, rtol=1e-14)
    # complex off-diagonal by hand: A = [[2, 1+i], [1-i, 2]] has column sums of
    # |Re| + |Im| equal to 4 and A^{-1} = [[2, -1-i], [-1+i, 2]] / 2 (trace 2);
    # its eigenvalues 2 +- sqrt 2 give kappa_2 = 5.83 < 8
    A2 = np.array([[2.0, 1 + 1j], [1 - 1j, 2.0]])[None]
    np.testing.assert_allclose(oracle.cond_estimate(A2), 8.0, rtol=1e-14)
    # between the modulus form of the 1-norm and sqrt 2 times it
    mod = np.max(np.sum(np.abs(A), axis=-2), axis=-1) * np.real(np.trace(np.linalg.inv(A), axis1=-2, axis2=-1))
    assert np.all(k >= mod * (1 - 1e-12)) and np.all(k <= np.sqrt(2) * mod * (1 + 1e-12))


# ---------------------------------------------------------------- large-system statistics
def test_asymptotic_formulas_self_consistent():
    """Corollary 1 equals E_s/sigma^2 at the Theorem 1 fixed point; Lemma 5
    equals the sum over clusters of the Lemma 2 per-cluster SINRs."""
    for beta, snr_db in [(1 / 16, 10.0), (1 / 32, 0.0), (0.25, 20.0)]:
        n0 = beta / 10 ** (snr_db / 10)
        s2 = oracle.tse_hanly_lmmse_sigma2(beta, n0)
        assert abs(oracle.sinr_pd_lmmse(beta, 1 / n0) - 1 / s2) < 1e-9 * (1 / s2)
        w = [1 / 8] * 8
        s2c = [oracle.tse_hanly_lmmse_sigma2(beta, n0, w=wc) for wc in w]
        assert abs(oracle.sinr_fd_lmmse(beta, 1 / n0, w) - sum(1 / v for v in s2c)) < 1e-8 * sum(1 / v for v in s2c)
    # printed closed forms reduce to the MRC/ZF limits: beta -> 0 gives E_s/N0
    assert abs(oracle.sinr_pd_lmmse(1e-12, 100.0) - 100.0) < 1e-6


def _unbiased_sinr(z, s):
    """SINR of the decoupled model z = mu s + e (eq. (decoupling)): regress out
    the common gain mu = E[conj(s) z]/E_s, then E_s |mu|^2 / E|z - mu s|^2."""
    es = np.mean(np.abs(s) ** 2)
    mu = np.mean(np.conj(s) * z) / es
    return es * abs(mu) ** 2 / np.mean(np.abs(z - mu * s) ** 2)


@pytest.mark.parametrize("snr_db", [0.0, 10.0, 20.0])
def test_empirical_sinr_matches_large_system_limit(snr_db):
    """Config-2 shape (B=256, C=8 x 32, U=16): the empirical SINR of the
    oracle's estimates is within 0.4 dB of Corollary 1 (PD) and Lemma 5 (FD,
    uniform partition), and FD <= PD (Lemma 3)."""
    b = synth.make_batch(W=150, B=256, U=16, C=8, snr_db=snr_db, mod="16qam", seed=99 + int(snr_db))
    beta = 16 / 256
    es_n0 = 1.0 / b.n0
    zp, _ = oracle.eq_pd(b.H, b.y, b.n0, b.cluster_off)
    zf, _ = oracle.eq_fd(b.H, b.y, b.n0, b.cluster_off)
    s = b.s.astype(np.complex128)
    emp_pd = _unbiased_sinr(zp, s)
    emp_fd = _unbiased_sinr(zf, s)
    th_pd = oracle.sinr_pd_lmmse(beta, es_n0)
    th_fd = oracle.sinr_fd_lmmse(beta, es_n0, [1 / 8] * 8)
    assert abs(10 * math.log10(emp_pd / th_pd)) < 0.4
    assert abs(10 * math.log10(emp_fd / th_fd)) < 0.4
    assert emp_fd <= emp_pd
    # for the MMSE estimate (PD) the unbiased SINR is also E_s/MSE - 1
    assert abs(10 * math.log10((1.0 / np.mean(np.abs(zp - s) ** 2) - 1.0) / th_pd)) < 0.4


# ---------------------------------------------------------------- several symbols per channel
def _sym_case(W=5, B=24, U=4, S=3, off=(0, 8, 24), seed=31):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((W, B, U)) + 1j * rng.standard_normal((W, B, U))) / np.sqrt(2 * B)
    Y = rng.standard_normal((W, S, B)) + 1j * rng.standard_normal((W, S, B))
    return H, Y, 0.05, list(off)


def test_symbols_reduce_to_one_vector_per_call():
    """Every symbol of the multi-symbol PD / FD equals the single-vector
    equaliser applied to that symbol's receive vector."""
    H, Y, n0, off = _sym_case()
    Zp, sp = oracle.eq_pd_symbols(H, Y, n0, off)
    Zf, sf = oracle.eq_fd_symbols(H, Y, n0, off)
    for s in range(Y.shape[1]):
        zp, sp1 = oracle.eq_pd(H, Y[:, s], n0, off)
        zf, sf1 = oracle.eq_fd(H, Y[:, s], n0, off)
        np.testing.assert_allclose(Zp[:, s], zp, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(Zf[:, s], zf, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(sp, sp1, rtol=1e-13)
        np.testing.assert_allclose(sf, sf1, rtol=1e-13)


def test_symbols_linear_in_the_receive_vectors():
    """L-MMSE is linear in y: Z(a Y1 + b Y2) = a Z(Y1) + b Z(Y2), for PD and
    FD (the FD weights do not depend on y)."""
    H, Y1, n0, off = _sym_case(seed=32)
    _, Y2, _, _ = _sym_case(seed=33)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    for fn in (oracle.eq_pd_symbols, oracle.eq_fd_symbols):
        Z, _ = fn(H, a * Y1 + b * Y2, n0, off)
        Z1, _ = fn(H, Y1, n0, off)
        Z2, _ = fn(H, Y2, n0, off)
        np.testing.assert_allclose(Z, a * Z1 + b * Z2, rtol=1e-11, atol=1e-13)


def test_symbols_brute_force_inverse():
    """Tiny PD case against an explicit inverse and explicit loops."""
    H, Y, n0, off = _sym_case(W=2, B=6, U=3, S=2, off=(0, 2, 6), seed=34)
    Z, s2 = oracle.eq_pd_symbols(H, Y, n0, off)
    for w in range(2):
        G = H[w].conj().T @ H[w]
        Ainv = np.linalg.inv(G + n0 * np.eye(3))
        for s in range(2):
            m = np.array([sum(np.conj(H[w, b, u]) * Y[w, s, b] for b in range(6)) for u in range(3)])
            np.testing.assert_allclose(Z[w, s], Ainv @ m, rtol=1e-12)
        np.testing.assert_allclose(s2[w], n0 * np.real(np.diag(Ainv)), rtol=1e-12)
