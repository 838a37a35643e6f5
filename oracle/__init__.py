"""FP64 CPU oracle for decentralized feedforward L-MMSE equalisation.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test-suite, the smoke check of the
graft entry point and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, obviously-correct restatement of what the paper
defines (Jeon, Li, Cavallaro, Studer, "Decentralized Equalization with
Feedforward Architectures for Massive MU-MIMO"), computed in complex128 from
the very complex64 inputs the GPU receives.  It shares no code with the HIP
path: it uses NumPy library primitives (matmul, solve, inv) as steps and does
no blocking, fusion or reordering beyond what the formulas state.

Modules
-------
lmmse        forward PD / FD L-MMSE (Sections II-C, III-A, IV-A, IV-B), also with
             several receive vectors per channel matrix (Section VI-B)
linear       PD / FD MRC and ZF (Section III-A, Section IV-A)
lama         LAMA-PD and LAMA-FD (Algorithm 1; Section IV with the Lemma 2 normalisation)
adjoint      analytic gradients of both equalisers (derived, not in the paper)
asymptotics  large-system SINR closed forms (Theorem 1, Corollary 1, Lemma 5)

Pins: every function is checked in ``tests/test_oracle_*.py`` against values
the paper's mathematics fixes (identities, closed forms, worked examples,
finite differences, Monte-Carlo error variances).  Nothing here is "parity
unpinned".
"""
from .lmmse import (local_statistics, lmmse_estimate, lmmse_error_variance,
                    lmmse_error_variance_simplified, cond_estimate, eq_pd, eq_fd,
                    optimal_fusion_weights, eq_centralized, eq_pd_symbols, eq_fd_symbols)
from .linear import (mrc_estimate, mrc_error_variance, zf_estimate, zf_error_variance,
                     lmmse_unbiased_gain, lmmse_unbiased_estimate, lmmse_unbiased_error_variance,
                     eq_pd_linear, eq_fd_linear)
from .lama import (qam_points, posterior_mean_var, lama_pd, lama_original, eq_pd_lama,
                   eq_fd_lama)
from .adjoint import pd_backward, fd_backward
from .asymptotics import (sinr_pd_lmmse, sinr_fd_lmmse, tse_hanly_lmmse_sigma2)

__all__ = [
    "local_statistics", "lmmse_estimate", "lmmse_error_variance",
    "lmmse_error_variance_simplified", "cond_estimate", "eq_pd", "eq_fd",
    "optimal_fusion_weights", "eq_centralized", "eq_pd_symbols", "eq_fd_symbols",
    "mrc_estimate", "mrc_error_variance", "zf_estimate", "zf_error_variance",
    "eq_pd_linear", "eq_fd_linear",
    "qam_points", "posterior_mean_var", "lama_pd", "lama_original", "eq_pd_lama", "eq_fd_lama",
    "pd_backward", "fd_backward",
    "sinr_pd_lmmse", "sinr_fd_lmmse", "tse_hanly_lmmse_sigma2",
]
