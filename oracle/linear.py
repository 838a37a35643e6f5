"""Forward PD / FD MRC and ZF equalisation in complex128 (test oracle only).

Section III-A defines, besides L-MMSE, two linear equalisers on the PD
statistics (G, y^MRC) of eq. (fullMRC):
  MRC   z = diag(G)^{-1} y^MRC,
        sigma^2 = diag( D^{-1} G D^{-H} N0 + (D^{-1} G - I)(D^{-1} G - I)^H E_s ),
        D = diag(G);
  ZF    z = G^{-1} y^MRC,  sigma^2 = N0 diag(G^{-1}).
The unbiased L-MMSE option is not in the paper (Section III-A gives the
biased estimate only); read here as the L-MMSE estimate scaled to unit gain:
with W = (G + rho I)^{-1}, user u sees the gain mu_u = [W G]_uu, and
  z = diag(mu)^{-1} W y^MRC,
  sigma^2 = diag( E G E^H N0 + (E G - I)(E G - I)^H E_s ),  E = diag(mu)^{-1} W,
the Section III-A variance of a linear equaliser E acting on y^MRC.
In the FD architecture (Section IV-A) every cluster applies the same
equaliser to its own statistics (G_c, y_c^MRC), and the fusion tree combines
the local estimates with the weights of Lemma 1 (eq. (opt_fusion)) or given
ones, exactly as for L-MMSE.
"""
import numpy as np

from .lmmse import _c128, _herm, lmmse_error_variance, lmmse_estimate, local_statistics, \
    optimal_fusion_weights

KINDS = ("lmmse", "zf", "mrc", "lmmse_unbiased")


def mrc_estimate(G, m):
    """z = diag(G)^{-1} y^MRC (Section III-A, MRC)."""
    G = _c128(G)
    d = np.real(np.diagonal(G, axis1=-2, axis2=-1))
    return _c128(m) / d


def mrc_error_variance(G, n0, es=1.0):
    """The Section III-A MRC error variance, term by term:
    diag( D^{-1} G D^{-H} N0 + (D^{-1} G - I)(D^{-1} G - I)^H E_s )."""
    G = _c128(G)
    U = G.shape[-1]
    d = np.real(np.diagonal(G, axis1=-2, axis2=-1))
    Dinv = np.zeros_like(G)
    idx = np.arange(U)
    Dinv[..., idx, idx] = 1.0 / d
    DG = Dinv @ G
    I = np.eye(U)
    S = Dinv @ G @ _herm(Dinv) * float(n0) + (DG - I) @ _herm(DG - I) * float(es)
    return np.real(np.diagonal(S, axis1=-2, axis2=-1)).copy()


def zf_estimate(G, m):
    """z = G^{-1} y^MRC (Section III-A, ZF)."""
    return np.linalg.solve(_c128(G), _c128(m)[..., None])[..., 0]


def zf_error_variance(G, n0):
    """N0 diag(G^{-1}) (Section III-A, ZF)."""
    Gi = np.linalg.inv(_c128(G))
    return float(n0) * np.real(np.diagonal(Gi, axis1=-2, axis2=-1)).copy()


def _unbiased_matrix(G, n0, es):
    """E = diag(mu)^{-1} W with W = (G + rho I)^{-1}, mu_u = [W G]_uu."""
    G = _c128(G)
    U = G.shape[-1]
    W = np.linalg.inv(G + (float(n0) / float(es)) * np.eye(U))
    mu = np.real(np.diagonal(W @ G, axis1=-2, axis2=-1))
    return W / mu[..., :, None], mu


def lmmse_unbiased_gain(G, n0, es=1.0):
    """mu_u = [(G + rho I)^{-1} G]_uu, the gain of user u in the biased L-MMSE estimate."""
    return _unbiased_matrix(G, n0, es)[1]


def lmmse_unbiased_estimate(G, m, n0, es=1.0):
    """z = diag(mu)^{-1} (G + rho I)^{-1} y^MRC (unit gain for every user)."""
    E, _ = _unbiased_matrix(G, n0, es)
    return (E @ _c128(m)[..., None])[..., 0]


def lmmse_unbiased_error_variance(G, n0, es=1.0):
    """The Section III-A error variance of the equaliser E = diag(mu)^{-1} W,
    term by term: diag( E G E^H N0 + (E G - I)(E G - I)^H E_s )."""
    G = _c128(G)
    E, _ = _unbiased_matrix(G, n0, es)
    EG = E @ G
    I = np.eye(G.shape[-1])
    S = E @ G @ _herm(E) * float(n0) + (EG - I) @ _herm(EG - I) * float(es)
    return np.real(np.diagonal(S, axis1=-2, axis2=-1)).copy()


def _equalise(kind, G, m, n0, es):
    if kind == "lmmse":
        return lmmse_estimate(G, m, n0, es), lmmse_error_variance(G, n0, es)
    if kind == "zf":
        return zf_estimate(G, m), zf_error_variance(G, n0)
    if kind == "mrc":
        return mrc_estimate(G, m), mrc_error_variance(G, n0, es)
    if kind == "lmmse_unbiased":
        return lmmse_unbiased_estimate(G, m, n0, es), lmmse_unbiased_error_variance(G, n0, es)
    raise ValueError(f"equaliser {kind!r} is not one of {KINDS}")


def eq_pd_linear(H, y, n0, cluster_off, kind, es=1.0):
    """PD equalisation with `kind` in KINDS: the adder tree
    sums the local statistics (eq. (fullMRC)) and the centralised unit applies
    the equaliser.  Returns z [W][U], sigma2 [W][U]."""
    Gc, mc = local_statistics(H, y, cluster_off)
    return _equalise(kind, Gc.sum(axis=1), mc.sum(axis=1), n0, es)


def eq_fd_linear(H, y, n0, cluster_off, kind, nu=None, es=1.0):
    """FD equalisation with `kind`: local estimates and variances per cluster,
    fused by eq. (fusionrule) with the weights of Lemma 1 (or `nu` [W][C][U],
    used as given); fused variance sum_c nu^2 sigma_c^2."""
    Gc, mc = local_statistics(H, y, cluster_off)
    z_c, s2_c = _equalise(kind, Gc, mc, n0, es)
    w = optimal_fusion_weights(s2_c) if nu is None else np.asarray(nu, np.float64)
    return np.sum(w * z_c, axis=1), np.sum(w * w * s2_c, axis=1)
