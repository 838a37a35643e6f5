"""LAMA-PD and LAMA-FD (Algorithm 1, Section III-C; Section IV) in complex128
(test oracle only).

Algorithm 1 iterates on the PD statistics (G, y^MRC): starting from
s^1 = E[S] = 0, phi^1 = Var[S] = E_s, v^1 = 0,
    z^t     = y^MRC + (I - G) s^t + v^t
    s^{t+1} = F(z^t, N0 + beta phi^t)
    phi^{t+1} = < G(z^t, N0 + beta phi^t) >          (mean over the users)
    v^{t+1} = beta phi^{t+1} / (N0 + beta phi^t) * (z^t - s^t)
and returns z^T with the error variance N0 + beta phi^T (T = T_max).  F and G
are the posterior mean and variance of a constellation point observed in
CN(0, tau) noise under the uniform prior of eq. (prior) (eq. (F)).

FD: each cluster runs the same algorithm on its statistics normalised by
1/sqrt(w_c), w_c = B_c / B (proof of Lemma 2): G_c / w_c, y_c^MRC / w_c,
noise N0 / w_c and system ratio beta / w_c.  The local estimates are fused
with the weights of Lemma 1 built from the local variances.
"""
import numpy as np

from .lmmse import _c128, _herm, local_statistics


def qam_points(order, es=1.0):
    """Square QAM with `order` points (4, 16, 64), zero mean, E|s|^2 = es."""
    m = int(round(np.sqrt(order)))
    if m * m != order:
        raise ValueError("square QAM only")
    lv = np.arange(-(m - 1), m, 2, dtype=np.float64)
    pts = (lv[:, None] + 1j * lv[None, :]).ravel()
    return pts * np.sqrt(es / np.mean(np.abs(pts) ** 2))


def posterior_mean_var(z, tau, points):
    """F(z, tau) and G(z, tau) of eq. (F): mean and variance of s under
    f(s | z) proportional to exp(-|z - s|^2 / tau) p(s), p uniform over the
    points (the complex sum over every point, no factorisation)."""
    z = _c128(z)
    tau = np.asarray(tau, np.float64)
    d = np.abs(z[..., None] - points) ** 2 / tau[..., None]
    d -= d.min(axis=-1, keepdims=True)
    w = np.exp(-d)
    w /= w.sum(axis=-1, keepdims=True)
    F = np.sum(w * points, axis=-1)
    G = np.sum(w * np.abs(points) ** 2, axis=-1) - np.abs(F) ** 2
    return F, G


def lama_pd(G, m, n0, beta, t_max, points, return_trace=False):
    """Algorithm 1 on statistics G [W][U][U], m [W][U] (one scalar n0 and beta
    for every system).  Returns z^T [W][U] and sigma2 [W] = N0 + beta phi^T."""
    G = _c128(G)
    m = _c128(m)
    W, U = m.shape
    es = float(np.mean(np.abs(points) ** 2))
    s = np.zeros((W, U), np.complex128) + np.mean(points)
    phi = np.full(W, es)
    v = np.zeros((W, U), np.complex128)
    trace = []
    for _ in range(int(t_max)):
        z = m + s - (G @ s[..., None])[..., 0] + v
        tau = n0 + beta * phi
        s_new, g = posterior_mean_var(z, np.broadcast_to(tau[:, None], z.shape), points)
        phi_new = np.mean(g, axis=-1)
        v = (beta * phi_new / (n0 + beta * phi))[:, None] * (z - s)
        trace.append((z, n0 + beta * phi))
        s, phi = s_new, phi_new
    z, s2 = trace[-1]
    return (z, s2, trace) if return_trace else (z, s2)


def lama_original(H, y, n0, t_max, points):
    """The original LAMA on (H, y) as restated in the derivation of
    Algorithm 1: z = s + H^H r, s' = F(z, N0 (1 + tau)),
    tau' = beta / N0 <G(z, N0 (1 + tau))>, r' = y - H s' + tau' / (1 + tau) r,
    with tau^1 = beta E_s / N0 (so that N0 (1 + tau) = N0 + beta phi)."""
    H = _c128(H)
    y = _c128(y)
    W, B, U = H.shape
    beta = U / B
    es = float(np.mean(np.abs(points) ** 2))
    s = np.zeros((W, U), np.complex128)
    tau = np.full(W, beta * es / n0)
    r = y.copy()
    out = None
    for _ in range(int(t_max)):
        z = s + (_herm(H) @ r[..., None])[..., 0]
        c = n0 * (1.0 + tau)
        s_new, g = posterior_mean_var(z, np.broadcast_to(c[:, None], z.shape), points)
        tau_new = beta / n0 * np.mean(g, axis=-1)
        r = y - (H @ s_new[..., None])[..., 0] + (tau_new / (1.0 + tau))[:, None] * r
        out = (z, c)
        s, tau = s_new, tau_new
    return out


def eq_pd_lama(H, y, n0, cluster_off, t_max, order, es=1.0):
    """LAMA-PD: the adder tree sums the local statistics (eq. (fullMRC)),
    beta = U / B.  Returns z [W][U] and sigma2 [W][U] (equal over users)."""
    Gc, mc = local_statistics(H, y, cluster_off)
    W, B, U = np.asarray(H).shape
    z, s2 = lama_pd(Gc.sum(axis=1), mc.sum(axis=1), float(n0), U / B, t_max, qam_points(order, es))
    return z, np.repeat(s2[:, None], U, axis=1)


def eq_fd_lama(H, y, n0, cluster_off, t_max, order, nu=None, es=1.0, return_clusters=False):
    """LAMA-FD: Algorithm 1 in every cluster on the 1/sqrt(w_c)-normalised
    statistics, fused by eq. (fusionrule) with Lemma 1's weights (or `nu`
    [W][C][U], used as given); fused variance sum_c nu^2 sigma_c^2.

    With return_clusters=True also returns the local estimates z_c [W][C][U],
    their variances sigma2_c [W][C] and, per cluster, Algorithm 1's trace
    (a list over iterations of (z_c^t [W][U], sigma2_c^t [W]))."""
    Gc, mc = local_statistics(H, y, cluster_off)
    W, B, U = np.asarray(H).shape
    off = [int(v) for v in cluster_off]
    C = len(off) - 1
    pts = qam_points(order, es)
    z_c = np.empty((W, C, U), np.complex128)
    s2_c = np.empty((W, C, U), np.float64)
    traces = []
    for c in range(C):
        wc = (off[c + 1] - off[c]) / B
        z, s2, tr = lama_pd(Gc[:, c] / wc, mc[:, c] / wc, float(n0) / wc, (U / B) / wc, t_max, pts,
                            return_trace=True)
        z_c[:, c] = z
        s2_c[:, c] = s2[:, None]
        traces.append(tr)
    if nu is None:
        p = 1.0 / s2_c
        w = p / p.sum(axis=1, keepdims=True)
    else:
        w = np.asarray(nu, np.float64)
    z, s2 = np.sum(w * z_c, axis=1), np.sum(w * w * s2_c, axis=1)
    if return_clusters:
        return z, s2, z_c, s2_c[:, :, 0], traces
    return z, s2
