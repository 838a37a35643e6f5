"""Ragged batches (eq_plan_*): 4096 independent systems of uneven B_c, U, C
in one persistent, graph-captured launch with autotuned launch shape; parity
of every system against the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1808_04473_amd import synth
from gpu_util import TOL_DB, TOL_Z, dev, expect_refused, host, need_gpu, refused, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def rb():
    return synth.make_ragged(4096)


def oracle_ragged(rb, fd, subset=None):
    ks = range(rb.nsys) if subset is None else subset
    z, s2 = {}, {}
    for k in ks:
        H, y, n0, off = rb.system(k)
        f = oracle.eq_fd if fd else oracle.eq_pd
        zz, ss = f(H[None], y[None], n0, off)
        z[k], s2[k] = zz[0], ss[0]
    return z, s2


def errors(rb, z, s2, zr, sr):
    ez, es = 0.0, 0.0
    for k, zk in zr.items():
        U, o = int(rb.U[k]), int(rb.z_off[k])
        zg, sg = z[o:o + U], s2[o:o + U]
        ez = max(ez, float(np.max(np.abs(zg - zk)) / np.max(np.abs(zk))))
        es = max(es, float(np.max(np.abs(10 * np.log10(sg / sr[k])))))
    return ez, es


@pytest.mark.parametrize("fd", [False, True], ids=["pd", "fd"])
def test_ragged_4096_fp32(rb, fd, tmp_path):
    from paper_1808_04473_amd import api
    cache = tmp_path / "tune.json"
    plan = api.Plan.from_ragged(rb, fd=fd, precision="fp32", tune_cache=cache)
    H, y = dev(rb.H_pool), dev(rb.y_pool)
    z, s2, info = plan.execute(H, y)
    torch.cuda.synchronize()
    zr, sr = oracle_ragged(rb, fd)
    ez, es = errors(rb, host(z), host(s2), zr, sr)
    print(f"ragged {'fd' if fd else 'pd'} fp32: z err {ez:.2e}, sigma2 {es:.4f} dB, {plan.describe()}", flush=True)
    assert ez <= TOL_Z["fp32"] and es <= TOL_DB
    assert np.all(host(info) == 0)
    # the autotune cache holds this plan's launch shape; a second plan reuses it
    c = json.load(open(cache))
    assert len(c) == 1
    (entry,) = c.values()
    d = plan.describe()
    assert entry["grid"] == d["grid"] and entry["half"] == d["half_items"]
    plan2 = api.Plan.from_ragged(rb, fd=fd, precision="fp32", tune_cache=cache)
    assert plan2.describe()["grid"] == d["grid"]
    # graph replays: same pools twice, then new pools (recapture)
    z1, _, _ = plan2.execute(H, y)
    z2, _, _ = plan2.execute(H, y)
    H2, y2 = H.clone(), y.clone()
    z3, _, _ = plan2.execute(H2, y2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z) and torch.equal(z2, z) and torch.equal(z3, z)


@pytest.mark.parametrize("fd", [False, True], ids=["pd", "fd"])
@pytest.mark.parametrize("prec", ["bf16_refine", "bf16x3_refine", "bf16x3"])
def test_ragged_precisions(rb, fd, prec, tmp_path):
    from paper_1808_04473_amd import api
    if refused("fd" if fd else "pd", prec):
        expect_refused(lambda: api.Plan.from_ragged(rb, fd=fd, precision=prec, tune_cache=tmp_path / "t.json"))
        return
    plan = api.Plan.from_ragged(rb, fd=fd, precision=prec, tune_cache=tmp_path / "t.json")
    z, s2, info = plan.execute(dev(rb.H_pool), dev(rb.y_pool))
    torch.cuda.synchronize()
    subset = list(range(0, rb.nsys, 7))
    zr, sr = oracle_ragged(rb, fd, subset)
    ez, es = errors(rb, host(z), host(s2), zr, sr)
    print(f"ragged {'fd' if fd else 'pd'} {prec}: z err {ez:.2e}, sigma2 {es:.4f} dB", flush=True)
    assert ez <= TOL_Z[prec] and es <= TOL_DB


def test_ragged_small_mixed_and_ill_conditioned(tmp_path):
    """A handful of systems including one with nearly collinear users and a
    tiny N0: that system is routed to the FP64 re-solve and still matches."""
    from paper_1808_04473_amd import api
    rb = synth.make_ragged(37, seed=5)
    k = 3
    B, U = int(rb.B[k]), int(rb.U[k])
    H = rb.H_pool[rb.h_off[k]:rb.h_off[k] + B * U].reshape(B, U).astype(np.complex128)
    rng = np.random.default_rng(1)
    H[:, 1] = H[:, 0] + 1e-4 * (rng.standard_normal(B) + 1j * rng.standard_normal(B))
    rb.H_pool[rb.h_off[k]:rb.h_off[k] + B * U] = H.astype(np.complex64).reshape(-1)
    rb.n0[k] = np.float32(1e-9)
    for fd in (False, True):
        plan = api.Plan.from_ragged(rb, fd=fd, precision="fp32", tune_cache=tmp_path / "t.json")
        z, s2, info = plan.execute(dev(rb.H_pool), dev(rb.y_pool))
        torch.cuda.synchronize()
        info = host(info)
        assert (info[k] & (1 << 30)) != 0
        zr, sr = oracle_ragged(rb, fd)
        ez, es = errors(rb, host(z), host(s2), zr, sr)
        assert ez <= 1e-4 and es <= TOL_DB
