"""Large-system SINR of L-MMSE in the PD and FD architectures (test oracle only).

Used as statistical sanity pins: in a finite Rayleigh-fading system the
empirical (unbiased) SINR of the exact equaliser must come close to these.
"""
from __future__ import annotations

import math


def sinr_pd_lmmse(beta: float, es_over_n0: float) -> float:
    """Corollary 1 (L-MMSE): centralised / PD post-equalisation SINR."""
    a = 1.0 - es_over_n0 * (1.0 - beta)
    return 0.5 * (math.sqrt(a * a + 4.0 * es_over_n0) - a)


def sinr_fd_lmmse(beta: float, es_over_n0: float, w) -> float:
    """Lemma 5: FD post-fusion SINR for cluster fractions w_c (sum w_c = 1)."""
    C = len(w)
    root = sum(math.sqrt((1.0 - es_over_n0 * (wc - beta)) ** 2 + 4.0 * es_over_n0 * wc)
               for wc in w)
    return 0.5 * root - 0.5 * (C - es_over_n0 * (1.0 - C * beta))


def tse_hanly_lmmse_sigma2(beta: float, n0: float, es: float = 1.0, w: float = 1.0,
                           iters: int = 10000) -> float:
    """Fixed point w*sigma^2 = N0 + beta*Psi(sigma^2), Psi = E_s sigma^2/(E_s + sigma^2)
    (Theorem 1; Lemma 2 for a cluster holding the fraction w), by plain iteration."""
    s = (n0 + beta * es) / w
    for _ in range(iters):
        s_new = (n0 + beta * es * s / (es + s)) / w
        if abs(s_new - s) <= 1e-15 * s:
            return s_new
        s = s_new
    return s
