"""Parity at the full sizes and in the launch configuration that bench.py
times, on sampled outputs the oracle computes one by one, plus properties
that hold at any size; maximum shapes; a large FP64 re-solve queue.

- B=256, C=8 x 32, U=16: 32 frames x 1200 = 38,400 systems in one call.
- B=1024, C=16 x 64, U=32: 4 frames x 1200 = 4,800 systems in one call.
"""
import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth
from gpu_util import (TOL_DB, TOL_Z, dev, expect_refused, host, max_db_err, max_rel_err, need_gpu,
                      refused, torch)

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3", "bf16_refine", "bf16x3_refine"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _frames(cfg, nframes, snr):
    bs = [synth.config_batch(cfg, snr, frame=f) for f in range(nframes)]
    H = np.concatenate([b.H for b in bs])
    y = np.concatenate([b.y for b in bs])
    return H, y, bs[0].n0, bs[0].cluster_off


@pytest.fixture(scope="module")
def c2_full():
    H, y, n0, off = _frames(2, 32, 10.0)
    return H, y, n0, off, dev(H), dev(y)


@pytest.fixture(scope="module")
def c3_full():
    H, y, n0, off = _frames(3, 4, 10.0)
    return H, y, n0, off, dev(H), dev(y)


def _sample(W, n, seed):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, W - 1], rng.choice(W, size=n, replace=False)]))
    return idx


def _run_and_check(data, mode, prec, nsample, seed):
    from paper_1808_04473_amd import api
    Hn, yn, n0, off, H, y = data
    W = Hn.shape[0]
    fn = api.eq_pd if mode == "pd" else api.eq_fd
    if refused(mode, prec):
        expect_refused(lambda: fn(H, y, n0, off, precision=prec, return_info=True))
        return
    z, s2, info = fn(H, y, n0, off, precision=prec, return_info=True)
    torch.cuda.synchronize()
    # properties over every system
    assert int(info.ne(0).sum().item()) == 0
    assert bool(torch.isfinite(torch.view_as_real(z)).all().item())
    assert bool((s2 > 0).all().item()) and bool(torch.isfinite(s2).all().item())
    # element-wise parity on sampled systems
    idx = _sample(W, nsample, seed)
    sel = torch.from_numpy(idx).to(H.device)
    zr, sr = (oracle.eq_pd if mode == "pd" else oracle.eq_fd)(Hn[idx], yn[idx], n0, off)
    ez, es = max_rel_err(host(z[sel]), zr), max_db_err(host(s2[sel]), sr)
    print(f"{mode} {prec} W={W}: {len(idx)} sampled systems, z err {ez:.2e}, sigma2 {es:.4f} dB", flush=True)
    assert ez <= TOL_Z[prec] and es <= TOL_DB


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("prec", PRECS)
def test_b256_38400_systems(c2_full, mode, prec):
    _run_and_check(c2_full, mode, prec, 384, 1)


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("prec", PRECS)
def test_b1024_4800_systems(c3_full, mode, prec):
    _run_and_check(c3_full, mode, prec, 48, 2)


def test_largest_b_and_most_clusters():
    """B = 65535 (the largest B) in 3 clusters, and B = 2048 in 1024 clusters
    (the most clusters, B_c = 2 < U = 32) for FD."""
    from paper_1808_04473_amd import api
    cases = [(2, 65535, 8, [0, 20000, 45000, 65535]),
             (2, 2048, 32, list(range(0, 2049, 2)))]
    for W, B, U, off in cases:
        b = synth.make_batch(W, B, U, len(off) - 1, 10.0, "qpsk", seed=B, cluster_off=off)
        for mode in ("pd", "fd"):
            fn = api.eq_pd if mode == "pd" else api.eq_fd
            z, s2 = fn(dev(b.H), dev(b.y), b.n0, b.cluster_off)
            torch.cuda.synchronize()
            zr, sr = (oracle.eq_pd if mode == "pd" else oracle.eq_fd)(b.H, b.y, b.n0, b.cluster_off)
            assert max_rel_err(host(z), zr) <= TOL_Z["fp32"], (W, B, U, mode)
            assert max_db_err(host(s2), sr) <= TOL_DB


def test_large_fp64_queue():
    """3,000 subcarriers, all with nearly collinear users and a tiny N0: every
    one is queued for the FP64 re-solve (the queue drains over the re-solve
    grid several times) and all meet the gate."""
    from paper_1808_04473_amd import api
    rng = np.random.default_rng(21)
    W, B, U, C = 3000, 48, 4, 2
    b = synth.make_batch(W, B, U, C, 10.0, "qpsk", seed=22)
    H = b.H.astype(np.complex128)
    H[:, :, 1] = H[:, :, 0] + 1e-4 * (rng.standard_normal((W, B)) + 1j * rng.standard_normal((W, B)))
    H = H.astype(np.complex64)
    y = (H.astype(np.complex128) @ b.s.astype(np.complex128)[..., None])[..., 0].astype(np.complex64)
    for mode in ("pd", "fd"):
        fn = api.eq_pd if mode == "pd" else api.eq_fd
        z, s2, info = fn(dev(H), dev(y), 1e-9, b.cluster_off, return_info=True)
        torch.cuda.synchronize()
        flags = (host(info) & (1 << 30)) != 0
        routed = flags if mode == "pd" else flags.any(axis=1)
        assert routed.all(), (mode, int(routed.sum()))
        idx = _sample(W, 200, 3)
        zr, sr = (oracle.eq_pd if mode == "pd" else oracle.eq_fd)(H[idx], y[idx], np.float32(1e-9), b.cluster_off)
        assert max_rel_err(host(z)[idx], zr) <= TOL_Z["fp32"]
        assert max_db_err(host(s2)[idx], sr) <= TOL_DB


def _sampled(data, fn, ref, tol, nsample, seed, **kw):
    Hn, yn, n0, off, H, y = data
    W = Hn.shape[0]
    z, s2, info = fn(H, y, n0, off, return_info=True, **kw)
    torch.cuda.synchronize()
    assert int((info & ~(1 << 30)).ne(0).sum().item()) == 0
    assert bool(torch.isfinite(torch.view_as_real(z)).all().item())
    assert bool((s2 > 0).all().item())
    idx = _sample(W, nsample, seed)
    sel = torch.from_numpy(idx).to(H.device)
    zr, sr = ref(Hn[idx], yn[idx], n0, off)
    ez, es = max_rel_err(host(z[sel]), zr), max_db_err(host(s2[sel]), sr)
    print(f"{fn.__name__} {kw} W={W}: {len(idx)} sampled, z err {ez:.2e}, sigma2 {es:.4f} dB", flush=True)
    assert ez <= tol and es <= TOL_DB


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("kind", ["zf", "mrc", "lmmse_unbiased"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_linear_equalisers_at_launch_size(c2_full, c3_full, mode, kind, prec):
    """ZF, MRC and the unbiased L-MMSE at 38,400 (B=256) and 4,800 (B=1024)
    systems, sampled."""
    from paper_1808_04473_amd import api
    fn = api.eq_pd if mode == "pd" else api.eq_fd
    rf = oracle.eq_pd_linear if mode == "pd" else oracle.eq_fd_linear
    for data, n, seed in ((c2_full, 256, 7), (c3_full, 48, 8)):
        _sampled(data, fn, lambda H, y, n0, off: rf(H, y, n0, off, kind), TOL_Z[prec], n, seed,
                 precision=prec, equalizer=kind)


@pytest.mark.parametrize("mode", ["pd", "fd"])
@pytest.mark.parametrize("t_max", [1, 3])
def test_lama_at_launch_size(c2_full, c3_full, mode, t_max):
    """LAMA (16-QAM) at 38,400 (B=256) and 4,800 (B=1024) systems, sampled."""
    from paper_1808_04473_amd import api
    fn = api.eq_pd_lama if mode == "pd" else api.eq_fd_lama
    rf = oracle.eq_pd_lama if mode == "pd" else oracle.eq_fd_lama
    for data, n, seed in ((c2_full, 256, 9), (c3_full, 48, 10)):
        _sampled(data, fn, lambda H, y, n0, off: rf(H, y, n0, off, t_max, 16), TOL_Z["fp32"], n, seed,
                 t_max=t_max, qam=16)
