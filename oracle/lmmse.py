"""Forward PD / FD L-MMSE equalisation in complex128 (test oracle only).

Array conventions (all batched over W independent systems, "subcarriers"):
  H [W][B][U], y [W][B] (any complex dtype; promoted to complex128),
  cluster_off [C+1] contiguous row offsets 0 = off[0] < ... < off[C] = B.
"""
from __future__ import annotations

import numpy as np


def _c128(a):
    return np.asarray(a).astype(np.complex128)


def _herm(a):
    """Conjugate transpose of the last two axes."""
    return np.conj(np.swapaxes(a, -1, -2))


def local_statistics(H, y, cluster_off):
    """Per-cluster Gram matrix G_c = H_c^H H_c and MRC vector y_c^MRC = H_c^H y_c.

    Section II-C (PD architecture, first step): each cluster c forms its local
    MRC output and local Gram matrix from its own rows H_c, y_c of the
    partitioned system (eq. (perclusterInOutrelation)).
    Returns G [W][C][U][U], m [W][C][U].
    """
    H = _c128(H)
    y = _c128(y)
    off = [int(v) for v in cluster_off]
    W, _, U = H.shape
    C = len(off) - 1
    G = np.empty((W, C, U, U), np.complex128)
    m = np.empty((W, C, U), np.complex128)
    for c in range(C):
        Hc = H[:, off[c]:off[c + 1], :]
        yc = y[:, off[c]:off[c + 1]]
        G[:, c] = _herm(Hc) @ Hc
        m[:, c] = (_herm(Hc) @ yc[:, :, None])[:, :, 0]
    return G, m


def lmmse_estimate(G, m, n0, es=1.0):
    """z = (G + rho I)^{-1} y^MRC with rho = N0/E_s (Section III-A, L-MMSE)."""
    U = G.shape[-1]
    rho = float(n0) / float(es)
    A = G + rho * np.eye(U)
    return np.linalg.solve(A, m[..., None])[..., 0]


def lmmse_error_variance(G, n0, es=1.0):
    """Post-equalisation error variance of L-MMSE, the Section III-A formula:

      sigma^2 = diag( W G W^H N0 + (W G - I)(W G - I)^H E_s ),  W = (G + rho I)^{-1}.
    """
    U = G.shape[-1]
    rho = float(n0) / float(es)
    I = np.eye(U)
    Wm = np.linalg.inv(G + rho * I)
    WG = Wm @ G
    S = Wm @ G @ _herm(Wm) * float(n0) + (WG - I) @ _herm(WG - I) * float(es)
    return np.real(np.diagonal(S, axis1=-2, axis2=-1)).copy()


def lmmse_error_variance_simplified(G, n0, es=1.0):
    """N0 * diag((G + rho I)^{-1}).

    With rho = N0/E_s one has W G - I = -rho W, so the Section III-A variance
    collapses to N0 * diag(W (G + rho I) W^H) = N0 * diag(W).  Kept separate so
    the tests can show the two agree (and differ once rho != N0/E_s).
    """
    U = G.shape[-1]
    rho = float(n0) / float(es)
    Wm = np.linalg.inv(G + rho * np.eye(U))
    return float(n0) * np.real(np.diagonal(Wm, axis1=-2, axis2=-1)).copy()


def cond_estimate(A):
    """Upper bound on the 2-norm condition number of an HPD matrix A:
    ||A||_1 * trace(A^{-1}) >= lambda_max / lambda_min, with the 1-norm's
    entry moduli replaced by |Re| + |Im| (at most sqrt(2) larger, so still a
    bound; this is the routing estimate of the FP64 re-solve, which is not
    part of the paper)."""
    A = _c128(A)
    n1 = np.max(np.sum(np.abs(A.real) + np.abs(A.imag), axis=-2), axis=-1)
    tr = np.real(np.trace(np.linalg.inv(A), axis1=-2, axis2=-1))
    return n1 * tr


def eq_pd(H, y, n0, cluster_off, es=1.0):
    """Partially decentralised L-MMSE (Section II-C, Section III-A).

    The feedforward adder tree sums the local statistics (eq. (fullMRC)):
    y^MRC = sum_c y_c^MRC, G = sum_c G_c; the centralised unit then computes
    the L-MMSE estimate and its error variance.
    Returns z [W][U] complex128, sigma2 [W][U] float64.
    """
    Gc, mc = local_statistics(H, y, cluster_off)
    G = Gc.sum(axis=1)
    m = mc.sum(axis=1)
    z = lmmse_estimate(G, m, n0, es)
    s2 = lmmse_error_variance(G, n0, es)
    return z, s2


def eq_centralized(H, y, n0, es=1.0):
    """Centralised L-MMSE on the whole array (one cluster holding all B rows)."""
    B = np.asarray(H).shape[1]
    return eq_pd(H, y, n0, [0, B], es)


def optimal_fusion_weights(s2_c):
    """nu_{c,u} = sigma_{c,u}^{-2} / sum_c' sigma_{c',u}^{-2}  (Lemma 1, eq. (opt_fusion)).

    s2_c has the cluster index on axis -2: [..., C, U]."""
    p = 1.0 / np.asarray(s2_c, np.float64)
    return p / p.sum(axis=-2, keepdims=True)


def eq_fd(H, y, n0, cluster_off, nu=None, es=1.0, return_local=False):
    """Fully decentralised L-MMSE (Section II-D, Section IV).

    Each cluster equalises locally with its own statistics (L-MMSE with the
    same rho = N0/E_s), giving z_c and sigma_c^2.  The fusion tree forms
    z_u = sum_c nu_{c,u} z_{c,u} (eq. (fusionrule)) with the optimal weights of
    Lemma 1 unless `nu` [W][C][U] is given (then used as is, not renormalised),
    and the fused error variance sum_c nu_{c,u}^2 sigma_{c,u}^2 (the
    denominator of eq. (postfusionSINR), uncorrelated cluster errors); for the
    optimal weights this equals (sum_c 1/sigma_{c,u}^2)^{-1} (Theorem 3).
    """
    Gc, mc = local_statistics(H, y, cluster_off)
    z_c = lmmse_estimate(Gc, mc, n0, es)
    s2_c = lmmse_error_variance(Gc, n0, es)
    w = optimal_fusion_weights(s2_c) if nu is None else np.asarray(nu, np.float64)
    z = np.sum(w * z_c, axis=1)
    s2 = np.sum(w * w * s2_c, axis=1)
    if return_local:
        return z, s2, dict(z_c=z_c, s2_c=s2_c, nu=w, G_c=Gc, m_c=mc)
    return z, s2


def eq_pd_symbols(H, Y, n0, cluster_off, es=1.0):
    """PD L-MMSE of N_sym receive vectors per channel matrix (Section VI-B:
    the Gram matrices are formed once per subcarrier and reused over the OFDM
    symbols of the coherence time; the matched filter is formed for every
    symbol).

    H [W][B][U], Y [W][S][B]; returns Z [W][S][U] and sigma2 [W][U] (the error
    variance does not depend on the receive vector).
    """
    H = _c128(H)
    Y = _c128(Y)
    off = [int(v) for v in cluster_off]
    W, B, U = H.shape
    G = np.zeros((W, U, U), np.complex128)
    M = np.zeros((W, U, Y.shape[1]), np.complex128)
    for c in range(len(off) - 1):
        Hc = H[:, off[c]:off[c + 1], :]
        G += _herm(Hc) @ Hc
        # H_c^H [y_1 ... y_S] restricted to the cluster's rows
        M += _herm(Hc) @ np.swapaxes(Y[:, :, off[c]:off[c + 1]], 1, 2)
    A = G + (float(n0) / float(es)) * np.eye(U)
    Z = np.swapaxes(np.linalg.solve(A, M), 1, 2)
    s2 = lmmse_error_variance(G, n0, es)
    return Z, s2


def eq_fd_symbols(H, Y, n0, cluster_off, nu=None, es=1.0):
    """FD L-MMSE of N_sym receive vectors per channel matrix: local estimates
    z_{c,s} = (G_c + rho I)^{-1} H_c^H y_{c,s} for every symbol, fused with the
    weights of Lemma 1 (which depend on the local error variances only, so
    they are the same for every symbol) or the given `nu` [W][C][U].
    Returns Z [W][S][U] and sigma2 [W][U].
    """
    H = _c128(H)
    Y = _c128(Y)
    off = [int(v) for v in cluster_off]
    W, B, U = H.shape
    S = Y.shape[1]
    C = len(off) - 1
    rho = float(n0) / float(es)
    z_c = np.empty((W, C, S, U), np.complex128)
    s2_c = np.empty((W, C, U), np.float64)
    for c in range(C):
        Hc = H[:, off[c]:off[c + 1], :]
        Gc = _herm(Hc) @ Hc
        Mc = _herm(Hc) @ np.swapaxes(Y[:, :, off[c]:off[c + 1]], 1, 2)
        z_c[:, c] = np.swapaxes(np.linalg.solve(Gc + rho * np.eye(U), Mc), 1, 2)
        s2_c[:, c] = lmmse_error_variance(Gc, n0, es)
    w = optimal_fusion_weights(s2_c) if nu is None else np.asarray(nu, np.float64)
    Z = np.sum(w[:, :, None, :] * z_c, axis=1)
    s2 = np.sum(w * w * s2_c, axis=1)
    return Z, s2
