"""eq_pd_noalloc (the partially decentralised L-MMSE with the library's own
device array as workspace) against eq_pd with a caller workspace: the same
kernels on the same inputs, so the outputs must be bit-identical, and both
meet the oracle's 1e-4 / 0.05 dB gate.  Two calls in a row, the second on a
smaller batch, with systems routed to the FP64 re-solve in each, so that the
queue in the array is used, left behind and cleared between calls."""
import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth
from gpu_util import TOL_DB, TOL_Z, dev, host, max_db_err, max_rel_err, need_gpu, torch

pytestmark = pytest.mark.gpu


def _with_bad_systems(b, bad, seed):
    """b with user 1 of systems `bad` nearly collinear with user 0 and a tiny
    N0, so that their condition estimate routes them to the FP64 re-solve."""
    rng = np.random.default_rng(seed)
    H = b.H.astype(np.complex128).copy()
    for w in bad:
        H[w, :, 1] = H[w, :, 0] + 1e-4 * (rng.standard_normal(b.B) + 1j * rng.standard_normal(b.B))
    H = H.astype(np.complex64)
    y = (H.astype(np.complex128) @ b.s.astype(np.complex128)[..., None])[..., 0].astype(np.complex64)
    return synth.Batch(H, y, b.s, 1e-9, b.cluster_off)


def _batches():
    big = synth.config_batch(2, 10.0)                               # W=1200, B=256, C=8, U=16
    small = synth.make_batch(24, 64, 4, 2, 10.0, "qpsk", seed=11)  # W=24, B=64, C=2, U=4
    return [(_with_bad_systems(big, [3, 600, 1199], 5), {3, 600, 1199}),
            (_with_bad_systems(small, [1, 7, 20], 9), {1, 7, 20})]


def test_noalloc_matches_eq_pd_on_two_calls():
    need_gpu()
    from paper_1808_04473_amd import api
    for k, (b, bad) in enumerate(_batches()):
        print(f"call {k}: W={b.W} B={b.B} U={b.U} C={b.C}", flush=True)
        H, y = dev(b.H), dev(b.y)
        z1, s1, i1 = api.eq_pd_noalloc(H, y, b.n0, b.cluster_off, return_info=True)
        prob, _keep = api.make_problem(b.W, b.B, b.U, b.cluster_off, b.n0)
        ws = api.workspace(prob, H.device)
        z2, s2, i2 = api.eq_pd(H, y, b.n0, b.cluster_off, return_info=True, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(z1, z2) and torch.equal(s1, s2) and torch.equal(i1, i2)
        routed = set(np.nonzero((host(i1) & (1 << 30)) != 0)[0])
        assert routed == bad, routed
        zr, sr = oracle.eq_pd(b.H, b.y, b.n0, b.cluster_off)
        assert max_rel_err(host(z1), zr) <= TOL_Z["fp32"]
        assert max_db_err(host(s1), sr) <= TOL_DB


def test_noalloc_refuses_oversized_batch():
    """W above the array's capacity is refused before any launch."""
    need_gpu()
    from paper_1808_04473_amd import api
    W = api.NOALLOC_MAX_W + 1
    H = torch.zeros((W, 2, 1), dtype=torch.complex64, device="cuda")
    y = torch.zeros((W, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(api.EqError) as e:
        api.eq_pd_noalloc(H, y, 0.1, [0, 2])
    assert e.value.status == -2
