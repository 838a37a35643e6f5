"""GPU parity of the ZF, MRC and unbiased L-MMSE equalisers (Section III-A;
Section IV-A for FD) against the FP64 oracle, element by element on the same seeded inputs:
max over systems of ||z - z_ref||_inf / ||z_ref||_inf within the form's
gate, post-equalisation SINR within 0.05 dB.  Plus the degenerate cases:
noise-free ZF recovery, a user with no channel (MRC) and a rank-deficient
Gram (ZF with B < U)."""
import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth
from gpu_util import (TOL_DB, TOL_Z, dev, expect_refused, host, max_db_err, max_rel_err, need_gpu,
                      refused, torch)

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def run(mode, kind, b, prec, nu=None, info=False):
    from paper_1808_04473_amd import api
    H, y = dev(b.H), dev(b.y)
    if mode == "pd":
        out = api.eq_pd(H, y, b.n0, b.cluster_off, precision=prec, return_info=info, equalizer=kind)
    else:
        out = api.eq_fd(H, y, b.n0, b.cluster_off, precision=prec, return_info=info, equalizer=kind,
                        nu=None if nu is None else dev(nu.astype(np.float32)))
    torch.cuda.synchronize()
    return [host(t) for t in out]


def ref(mode, kind, b, nu=None):
    if mode == "pd":
        return oracle.eq_pd_linear(b.H, b.y, b.n0, b.cluster_off, kind)
    return oracle.eq_fd_linear(b.H, b.y, b.n0, b.cluster_off, kind, nu=nu)


SHAPES = [  # (W, B, U, C or offsets); every cluster has B_c >= U (ZF FD)
    (64, 32, 4, 2),
    (200, 256, 16, 8),
    (24, 1024, 32, 16),
    (13, 37, 5, [0, 5, 20, 37]),
    (9, 100, 16, [0, 40, 100]),
    (5, 130, 24, [0, 60, 130]),
]
CASES = [("zf", p) for p in ("fp32", "bf16x3", "bf16_refine", "bf16x3_refine")] + \
        [("mrc", p) for p in ("fp32", "bf16x3")] + [("lmmse_unbiased", p) for p in ("fp32", "bf16x3")]


def _batch(shape, seed, snr=10.0):
    W, B, U, C = shape
    off = C if isinstance(C, list) else None
    nc = len(C) - 1 if isinstance(C, list) else C
    return synth.make_batch(W, B, U, nc, snr, "16qam", seed=seed, cluster_off=off)


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("kind,prec", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"W{s[0]}B{s[1]}U{s[2]}")
def test_linear_matches_oracle(mode, kind, prec, shape):
    b = _batch(shape, seed=shape[0] * 7 + shape[1])
    if refused(mode, prec):
        expect_refused(lambda: run(mode, kind, b, prec, info=True))
        return
    z, s2, info = run(mode, kind, b, prec, info=True)
    zr, sr = ref(mode, kind, b)
    ez, es = max_rel_err(z, zr), max_db_err(s2, sr)
    print(f"{kind} {mode} {prec} W={b.W} B={b.B} U={b.U} C={b.C}: z err {ez:.2e}, sigma2 {es:.4f} dB", flush=True)
    assert ez <= TOL_Z[prec], ez
    assert es <= TOL_DB, es
    assert ((info & ~(1 << 30)) == 0).all()


@pytest.mark.parametrize("kind", ["zf", "mrc", "lmmse_unbiased"])
def test_fd_given_weights(kind):
    b = _batch((31, 96, 8, 3), seed=3)
    nu = np.random.default_rng(4).uniform(0.1, 1.0, size=(31, 3, 8))
    z, s2 = run("fd", kind, b, "fp32", nu=nu)
    zr, sr = ref("fd", kind, b, nu=nu)
    assert max_rel_err(z, zr) <= TOL_Z["fp32"]
    assert max_db_err(s2, sr) <= TOL_DB


@pytest.mark.parametrize("mode", ["pd", "fd"])
def test_zf_noise_free_recovers_symbols(mode):
    b = _batch((50, 256, 16, 8), seed=5)
    b.y = (b.H.astype(np.complex128) @ b.s.astype(np.complex128)[..., None])[..., 0].astype(np.complex64)
    z, _ = run(mode, "zf", b, "fp32")
    assert np.max(np.abs(z - b.s)) < 1e-4


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("U", [4, 12, 24])
def test_zf_padded_users_stay_on_the_fp32_path(mode, U):
    """Well-conditioned ZF systems with U below the lane-group width (padded
    users) are solved in FP32: nothing is routed to the FP64 re-solve."""
    b = synth.make_batch(40, 256, U, 4, 10.0, "16qam", seed=U)
    z, s2, info = run(mode, "zf", b, "fp32", info=True)
    assert (info == 0).all(), np.unique(info)
    zr, sr = ref(mode, "zf", b)
    assert max_rel_err(z, zr) <= TOL_Z["fp32"]
    assert max_db_err(s2, sr) <= TOL_DB


@pytest.mark.filterwarnings("ignore::RuntimeWarning")  # the oracle divides by the zero G_uu
def test_mrc_user_without_channel():
    """A zero column of H makes G_uu = 0: info = u + 1 and NaN outputs for
    that system only."""
    b = _batch((6, 64, 8, 2), seed=6)
    b.H[3, :, 2] = 0
    z, s2, info = run("pd", "mrc", b, "fp32", info=True)
    assert info[3] == 3 and np.isnan(z[3]).all() and np.isnan(s2[3]).all()
    keep = np.arange(6) != 3
    zr, sr = ref("pd", "mrc", b)
    assert (info[keep] == 0).all()
    assert max_rel_err(z[keep], zr[keep]) <= TOL_Z["fp32"]


def test_zf_rank_deficient_gram():
    """B < U: G is singular.  Every system fails an FP32 pivot or the
    condition check and is re-solved in FP64 (flag set); where the FP64
    factorisation fails too (a pivot <= 0, not guaranteed in rounded
    arithmetic) info holds that pivot and the outputs are NaN."""
    b = synth.make_batch(16, 6, 8, 1, 10.0, "qpsk", seed=7)
    z, s2, info = run("pd", "zf", b, "fp32", info=True)
    assert ((info & (1 << 30)) != 0).all()
    piv = info & ~(1 << 30)
    assert ((piv == 0) | (piv >= 7)).all(), piv
    assert (piv > 0).any()
    assert np.isnan(z[piv > 0]).all() and np.isnan(s2[piv > 0]).all()


@pytest.mark.parametrize("mode", ["pd", "fd"])
def test_unbiased_is_scaled_lmmse(mode):
    """PD: the unbiased outputs are the L-MMSE outputs divided by
    mu = 1 - sigma2 / E_s (both from the GPU); FD: unit-gain local estimates
    give a fused estimate whose regression on the symbols has slope near 1,
    where the biased one is below 1."""
    b = _batch((1000, 256, 16, 8), seed=21, snr=0.0)
    zu, su = run(mode, "lmmse_unbiased", b, "fp32")
    zb, sb = run(mode, "lmmse", b, "fp32")
    if mode == "pd":
        mu = 1.0 - sb.astype(np.float64)
        assert max_rel_err(zu, zb / mu) <= 1e-5
        np.testing.assert_allclose(su, sb / mu, rtol=1e-5)
    s = b.s
    slope_u = np.real(np.sum(np.conj(s) * zu) / np.sum(np.abs(s) ** 2))
    slope_b = np.real(np.sum(np.conj(s) * zb) / np.sum(np.abs(s) ** 2))
    print(f"{mode}: slope unbiased {slope_u:.4f}, biased {slope_b:.4f}", flush=True)
    assert abs(slope_u - 1.0) < 0.01 and slope_b < 0.97
