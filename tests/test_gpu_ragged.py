"""Ragged batches (eq_plan_*): 4096 independent systems of uneven B_c, U, C
in one persistent, graph-captured launch with autotuned launch shape (waves
per CU, PD piece rows per tile class); parity of every system against the
FP64 oracle."""
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
    # the autotune cache holds the launch entry (waves per CU) and, for PD,
    # the piece rows of each tile class of the batch, keyed by device, mode,
    # precision and class; a plan for another batch drawn from the same
    # distribution takes its shape from the cache
    mode = "fd" if fd else "pd"
    c = json.load(open(cache))
    d = plan.describe()
    assert sum(v["systems"] for v in d["classes"].values()) == rb.nsys
    assert c[f"gfx950/{mode}/p0/launch"]["wpc"] in (4, 6, 8)
    if fd:
        assert len(c) == 1
        assert sum(v["clusters"] for v in d["classes"].values()) == int(np.sum(rb.C))
        assert all(v["piece_rows"] == 0 for v in d["classes"].values())
    else:
        assert len(c) == 1 + len(d["classes"])
        for name, v in d["classes"].items():
            assert c[f"gfx950/pd/p0/{name}"]["piece_rows"] == v["piece_rows"] in (0, 256, 384, 512, 768)
    other = synth.make_ragged(4096, seed=synth.BASE_SEED + 99)
    plan_o = api.Plan.from_ragged(other, fd=fd, precision="fp32", tune_cache=cache)
    do = plan_o.describe()
    wpc = c[f"gfx950/{mode}/p0/launch"]["wpc"]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert d["grid"] == min(cus * wpc, d["tasks"]) and do["grid"] == min(cus * wpc, do["tasks"])
    for name, v in do["classes"].items():
        if not fd:
            assert c[f"gfx950/pd/p0/{name}"]["piece_rows"] == v["piece_rows"]
    mtime = os.path.getmtime(cache)
    zo, _, _ = plan_o.execute(dev(other.H_pool), dev(other.y_pool))
    torch.cuda.synchronize()
    assert os.path.getmtime(cache) == mtime  # no tuning run: everything was cached
    zro, _ = oracle_ragged(other, fd, list(range(0, other.nsys, 11)))
    zo_h = host(zo)
    ez_o = max(float(np.max(np.abs(zo_h[int(other.z_off[k]):int(other.z_off[k]) + int(other.U[k])] - zk))
                     / np.max(np.abs(zk))) for k, zk in zro.items())
    assert ez_o <= TOL_Z["fp32"], ez_o
    plan_o.close()
    plan2 = api.Plan.from_ragged(rb, fd=fd, precision="fp32", tune_cache=cache)
    # graph replays: same pools twice, then new pools (recapture)
    z1, _, _ = plan2.execute(H, y)
    z2, _, _ = plan2.execute(H, y)
    H2, y2 = H.clone(), y.clone()
    z3, _, _ = plan2.execute(H2, y2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z) and torch.equal(z2, z) and torch.equal(z3, z)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_ragged_pd_row_pieces(rb, prec, tmp_path):
    """PD systems cut into row pieces of 32 rows (a cached shape): the
    partial Grams of the pieces are summed by the system's last piece in
    piece order, so every system matches the oracle, and two executions give
    identical bits whichever wave finishes a system."""
    from paper_1808_04473_amd import api
    p = api.PRECISIONS[prec]
    cache = tmp_path / "pieces.json"
    cache.write_text("{\n"
                     f'  "gfx950/pd/p{p}/launch": {{"wpc": 8}},\n'
                     f'  "gfx950/pd/p{p}/ut16": {{"piece_rows": 32}},\n'
                     f'  "gfx950/pd/p{p}/ut32": {{"piece_rows": 32}}\n'
                     "}\n")
    plan = api.Plan.from_ragged(rb, fd=False, precision=prec, tune_cache=cache)
    d = plan.describe()
    assert all(v["piece_rows"] == 32 for v in d["classes"].values())
    # every system of more than 32 rows is cut (16-row blocks for UT = 32,
    # 32-row blocks for UT = 16)
    npieces = 0
    for k in range(rb.nsys):
        B, rpb = int(rb.B[k]), (32 if int(rb.U[k]) <= 16 else 16)
        if B > 32:
            nb = -(-B // rpb)
            per = max(1, 32 // rpb)
            npieces += -(-nb // per)
    assert sum(v["pieces"] for v in d["classes"].values()) == npieces > 0
    H, y = dev(rb.H_pool), dev(rb.y_pool)
    z, s2, info = plan.execute(H, y)
    z2, s22, _ = plan.execute(H, y, out=(torch.empty_like(z), torch.empty_like(s2), torch.empty_like(info)))
    torch.cuda.synchronize()
    assert torch.equal(z, z2) and torch.equal(s2, s22)
    subset = list(range(0, rb.nsys, 5))
    zr, sr = oracle_ragged(rb, False, subset)
    ez, es = errors(rb, host(z), host(s2), zr, sr)
    print(f"ragged pd {prec} pieces of 32 rows: z err {ez:.2e}, sigma2 {es:.4f} dB", flush=True)
    assert ez <= TOL_Z[prec] and es <= TOL_DB
    assert np.all(host(info) == 0)
    plan.close()


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
        Hd, yd = dev(rb.H_pool), dev(rb.y_pool)
        zr, sr = oracle_ragged(rb, fd)
        # three executions of the captured graph: the queue heads, arrival
        # counters and FP64 queue must start each execution at zero
        for rep in range(3):
            z, s2, info = plan.execute(Hd, yd)
            torch.cuda.synchronize()
            info = host(info)
            assert (info[k] & (1 << 30)) != 0
            assert np.all((info & ~(1 << 30)) == 0)
            ez, es = errors(rb, host(z), host(s2), zr, sr)
            assert ez <= 1e-4 and es <= TOL_DB, rep


def _custom_batch(specs, seed=11):
    """A ragged batch of the given systems: specs = [(U, [cluster sizes])],
    i.i.d. Rayleigh H, 16-QAM symbols, SNR 10 dB."""
    rng = np.random.default_rng(seed)
    pts = synth.constellation("16qam")
    Us = np.array([u for u, _ in specs], np.int64)
    Cs = np.array([len(c) for _, c in specs], np.int64)
    Bs = np.array([int(sum(c)) for _, c in specs], np.int64)
    h_off = np.concatenate([[0], np.cumsum(Bs * Us)[:-1]]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(Bs)[:-1]]).astype(np.int64)
    z_off = np.concatenate([[0], np.cumsum(Us)[:-1]]).astype(np.int64)
    clus_first = np.concatenate([[0], np.cumsum(Cs)[:-1]]).astype(np.int64)
    H_pool = np.empty(int((Bs * Us).sum()), np.complex64)
    y_pool = np.empty(int(Bs.sum()), np.complex64)
    n0 = np.empty(len(specs), np.float32)
    for k in range(len(specs)):
        B, U = int(Bs[k]), int(Us[k])
        H = (rng.standard_normal((B, U)) + 1j * rng.standard_normal((B, U))) / np.sqrt(2 * B)
        s = pts[rng.integers(0, len(pts), size=U)]
        n0[k] = synth.noise_variance(U, B, 10.0)
        y = H @ s + (rng.standard_normal(B) + 1j * rng.standard_normal(B)) * np.sqrt(n0[k] / 2)
        H_pool[h_off[k]:h_off[k] + B * U] = H.reshape(-1).astype(np.complex64)
        y_pool[y_off[k]:y_off[k] + B] = y.astype(np.complex64)
    return synth.RaggedBatch(H_pool=H_pool, y_pool=y_pool, s_pool=np.zeros(int(Us.sum()), np.complex64),
                             B=Bs.astype(np.int32), U=Us.astype(np.int32), C=Cs.astype(np.int32), n0=n0,
                             h_off=h_off, y_off=y_off, z_off=z_off, clus_first=clus_first,
                             cluster_sizes=np.concatenate([np.array(c, np.int32) for _, c in specs]))


EXTREME = [
    (8, [40]), (16, [64]), (24, [48]), (32, [96]),         # FD with one cluster
    (8, [16] * 64), (16, [32] * 40), (32, [40] * 24),      # clusters over many rounds
    (1, [3, 5]), (17, [20, 18, 30]), (2, [1, 1, 1]),       # U = 1, 17, one-row clusters
    (32, [64] * 60), (16, [256] * 4),                      # B = 3840 and 1024: many pieces
    (7, [12, 20]), (9, [20, 24]), (23, [30, 26]), (25, [40, 36]),  # either side of the short
                                                           # FD solves (U <= 8 of 16, U <= 24 of 32)
]


@pytest.mark.parametrize("fd", [False, True], ids=["pd", "fd"])
@pytest.mark.parametrize("rows", [None, 32], ids=["tuned", "pieces32"])
def test_ragged_extreme_shapes(fd, rows, tmp_path):
    """Single-cluster FD systems, systems whose 24-64 clusters span many
    rounds, U = 1 and 17, one-row clusters, systems cut into up to 120 row
    pieces, and U = 7, 9, 23, 25 around the widths where FD leaves out the
    padded users' steps: every system against the oracle."""
    from paper_1808_04473_amd import api
    rb = _custom_batch(EXTREME)
    cache = tmp_path / "t.json"
    if rows is not None:
        mode = "fd" if fd else "pd"
        cache.write_text("{\n" + f'  "gfx950/{mode}/p0/launch": {{"wpc": 8}},\n'
                         f'  "gfx950/{mode}/p0/ut16": {{"piece_rows": {rows}}},\n'
                         f'  "gfx950/{mode}/p0/ut32": {{"piece_rows": {rows}}}\n' + "}\n")
    plan = api.Plan.from_ragged(rb, fd=fd, precision="fp32", tune_cache=cache)
    z, s2, info = plan.execute(dev(rb.H_pool), dev(rb.y_pool))
    torch.cuda.synchronize()
    zr, sr = oracle_ragged(rb, fd)
    ez, es = errors(rb, host(z), host(s2), zr, sr)
    print(f"ragged extreme {'fd' if fd else 'pd'} rows={rows}: z err {ez:.2e}, sigma2 {es:.4f} dB, "
          f"{plan.describe()}", flush=True)
    assert ez <= 1e-4 and es <= TOL_DB
    assert np.all((host(info) & ~(1 << 30)) == 0)
    plan.close()
