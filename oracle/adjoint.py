"""Analytic adjoints of the PD and FD L-MMSE equalisers (test oracle only).

The paper defines no gradient; these are derived here from its forward maps
and pinned against central finite differences of ``oracle.lmmse``.

Convention (as PyTorch uses for complex tensors): for a real loss L and a
complex variable x, grad_x = dL/dRe(x) + i dL/dIm(x), so dL = Re(sum conj(grad_x) dx).

With A = H^H H + rho I, rho = N0/E_s, z = A^{-1} H^H y and
sigma2_u = N0 [A^{-1}]_uu (the Section III-A variance at rho = N0/E_s),
given upstream grads gz (complex, [U]) and gs (real, [U]):
  lambda = A^{-1} gz,   Q = A^{-1} diag(gs) A^{-1}
  grad_H  = (y - H z) lambda^H - H lambda z^H - 2 N0 H Q
  grad_y  = H lambda
  grad_N0 = -Re(z^H lambda)/E_s + sum_u gs_u [A^{-1}]_uu - N0 tr(Q)/E_s
"""
from __future__ import annotations

import numpy as np

from .lmmse import local_statistics


def _herm(a):
    return np.conj(np.swapaxes(a, -1, -2))


def _system_backward(Hc, yc, G, m, n0, es, gz, gs):
    """Backward of (z, sigma2) = L-MMSE(G, m) for a batch of systems built from
    rows Hc [W][b][U], yc [W][b].  Returns grad_H, grad_y, grad_N0 per system."""
    U = G.shape[-1]
    rho = float(n0) / float(es)
    Ainv = np.linalg.inv(G + rho * np.eye(U))
    z = (Ainv @ m[..., None])[..., 0]
    d = np.real(np.diagonal(Ainv, axis1=-2, axis2=-1))
    lam = (Ainv @ gz[..., None])[..., 0]
    Q = Ainv @ (gs[..., :, None] * Ainv)
    Hz = (Hc @ z[..., None])[..., 0]
    Hl = (Hc @ lam[..., None])[..., 0]
    gH = ((yc - Hz)[..., :, None] * np.conj(lam)[..., None, :]
          - Hl[..., :, None] * np.conj(z)[..., None, :]
          - 2.0 * float(n0) * (Hc @ Q))
    gy = Hl
    gn0 = (-np.real(np.sum(np.conj(z) * lam, axis=-1)) / float(es)
           + np.sum(gs * d, axis=-1)
           - float(n0) * np.real(np.trace(Q, axis1=-2, axis2=-1)) / float(es))
    return gH, gy, gn0


def pd_backward(H, y, n0, cluster_off, gz, gs=None, es=1.0):
    """Gradients of the PD equaliser w.r.t. H [W][B][U], y [W][B] and N0 (scalar)."""
    H = np.asarray(H).astype(np.complex128)
    y = np.asarray(y).astype(np.complex128)
    gz = np.asarray(gz).astype(np.complex128)
    gs = np.zeros(gz.shape, np.float64) if gs is None else np.asarray(gs, np.float64)
    Gc, mc = local_statistics(H, y, cluster_off)
    gH, gy, gn0 = _system_backward(H, y, Gc.sum(axis=1), mc.sum(axis=1), n0, es, gz, gs)
    return gH, gy, float(np.sum(gn0))


def fd_backward(H, y, n0, cluster_off, gz, gs=None, nu=None, es=1.0):
    """Gradients of the FD equaliser w.r.t. H, y, N0 and (when given) nu [W][C][U].

    Fusion (Lemma 1 / eq. (fusionrule)): z = sum_c nu_c z_c,
    sigma2 = sum_c nu_c^2 sigma2_c.  With the optimal weights nu_c = p_c / S,
    p_c = 1/sigma2_c, S = sum_c p_c, the weights themselves depend on sigma2_c:
      dL/dp_c = (g_nu_c - sum_c' nu_c' g_nu_c') / S,
      dL/dsigma2_c += -p_c^2 dL/dp_c.
    Returns grad_H, grad_y, grad_N0 and grad_nu (None when nu is computed).
    """
    H = np.asarray(H).astype(np.complex128)
    y = np.asarray(y).astype(np.complex128)
    gz = np.asarray(gz).astype(np.complex128)
    gs = np.zeros(gz.shape, np.float64) if gs is None else np.asarray(gs, np.float64)
    off = [int(v) for v in cluster_off]
    C = len(off) - 1
    U = H.shape[-1]
    rho = float(n0) / float(es)
    Gc, mc = local_statistics(H, y, off)
    Ainv = np.linalg.inv(Gc + rho * np.eye(U))
    z_c = (Ainv @ mc[..., None])[..., 0]                     # [W][C][U]
    s2_c = float(n0) * np.real(np.diagonal(Ainv, axis1=-2, axis2=-1))
    optimal = nu is None
    if optimal:
        p = 1.0 / s2_c
        S = p.sum(axis=1, keepdims=True)
        w = p / S
    else:
        w = np.asarray(nu, np.float64)
    # partials with the weights treated as free variables
    g_nu = np.real(np.conj(gz)[:, None, :] * z_c) + 2.0 * gs[:, None, :] * w * s2_c
    g_s2c = gs[:, None, :] * w * w
    if optimal:
        g_p = (g_nu - np.sum(w * g_nu, axis=1, keepdims=True)) / S
        g_s2c = g_s2c - p * p * g_p
    g_zc = w * gz[:, None, :]
    gH = np.zeros_like(H)
    gy = np.zeros_like(y)
    gn0 = 0.0
    for c in range(C):
        Hc = H[:, off[c]:off[c + 1], :]
        yc = y[:, off[c]:off[c + 1]]
        gHc, gyc, gn0c = _system_backward(Hc, yc, Gc[:, c], mc[:, c], n0, es,
                                           g_zc[:, c], g_s2c[:, c])
        gH[:, off[c]:off[c + 1], :] = gHc
        gy[:, off[c]:off[c + 1]] = gyc
        gn0 += float(np.sum(gn0c))
    return gH, gy, gn0, (None if optimal else g_nu)
