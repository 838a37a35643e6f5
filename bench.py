#!/usr/bin/env python3
"""Throughput of decentralized feedforward L-MMSE equalisation on one MI355X.

Workload: B = 256 antennas in C = 8 clusters of 32, U = 16 users, 16-QAM,
SNR 10 dB, i.i.d. Rayleigh H; one step equalises F frames x 1200 subcarriers
(default F = 32: 38,400 independent systems, 1.34 GB of H and y, so the
inputs stream from HBM rather than from the 256 MB Infinity Cache).  The
headline `value` is partially-decentralised (PD) L-MMSE in FP32; every other
form (FD fusion; split-BF16 MFMA Gram; BF16 / split-BF16 MFMA Gram with one
refinement step) is timed the same way under "variants", and the split-BF16
MFMA form is set against FP32 under "bf16_mfma_vs_fp32".  Inputs are resident in HBM before timing starts,
and about 0.2 s of untimed calls of each form (`settle_s`) precede its warmup steps, so that the timed
steps run at the device's loaded clocks.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--frames F]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B, C, U, W_FRAME, SNR_DB = 256, 8, 16, 1200, 10.0
HBM_PEAK_GBS = 8000.0
CPU_MIN_SECONDS = 10.0
SETTLE_S = 0.2  # untimed load before each timed form (see settle)
_SETTLE_S = [SETTLE_S]  # the run's value (--settle-s)


def bytes_per_system(B=B, U=U):
    """Algorithmic HBM bytes of one system: read H and y once, write z and sigma2."""
    return B * U * 8 + B * 8 + U * 8 + U * 4


def kernel_source_sha(files=None):
    """sha256[:16] over the kernel sources `files` (names under csrc/; all of
    them when None)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1808_04473_amd", "csrc")
    names = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".h", ".cpp"))) if files is None \
        else list(files)
    for f in names:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(variant):
    """HBM traffic per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current sources of that kernel (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except (OSError, ValueError):
        return None
    e = t.get(variant)
    if not e or e.get("source_sha") != kernel_source_sha(e.get("sources")):
        return None
    return e.get("bytes_per_launch")


def make_inputs(frames):
    from paper_1808_04473_amd import synth
    Hs, ys = [], []
    n0 = None
    for f in range(frames):
        b = synth.config_batch(2, SNR_DB, frame=f)
        Hs.append(b.H)
        ys.append(b.y)
        n0 = b.n0
        off = b.cluster_off
    return np.concatenate(Hs), np.concatenate(ys), n0, off


def cpu_cores():
    """Host threads the oracle baseline may use: the CPUs this process may run
    on, capped at 16 (the host share of one GPU) or at OMP_NUM_THREADS when set."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = 16
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        cap = min(cap, int(env))
    return max(1, min(n, cap))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_worker_init():
    # one BLAS / OpenMP thread per worker process: the parallelism is the pool
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _cpu_worker(task):
    """Generates its frames of the step (not timed), then runs the FP64 PD
    oracle over them, frame by frame, until `seconds` of wall time have passed."""
    frames, seconds = task
    import oracle
    from paper_1808_04473_amd import synth
    batches = [synth.config_batch(2, SNR_DB, frame=f) for f in frames]
    n, t0, c0 = 0, time.time(), time.process_time()
    while True:
        for b in batches:
            oracle.eq_pd(b.H, b.y, b.n0, b.cluster_off)
            n += b.H.shape[0]
        if time.time() - t0 >= seconds:
            break
    return n, t0, time.time(), time.process_time() - c0


class CpuBaseline:
    """The FP64 oracle (as it stands) on the host cores, one process per core.

    The pool is forked before anything touches the GPU; each worker equalises
    its share of the step's frames (generated from the same seeds as the GPU
    inputs) repeatedly for about `seconds` of wall time.  Throughput is the
    systems done over the span from the first worker's start to the last
    worker's end."""

    def __init__(self, frames, seconds=CPU_MIN_SECONDS, cores=None):
        import multiprocessing as mp
        self.cores = cores or cpu_cores()
        self.frames = frames
        self.seconds = seconds
        self.pool = mp.get_context("fork").Pool(self.cores, initializer=_cpu_worker_init)

    def run(self):
        shares = [list(range(k, self.frames, self.cores)) for k in range(self.cores)]
        shares = [sh for sh in shares if sh]
        try:
            res = self.pool.map(_cpu_worker, [(sh, self.seconds) for sh in shares])
        finally:
            self.pool.close()
            self.pool.join()
        n = sum(r[0] for r in res)
        span = max(r[2] for r in res) - min(r[1] for r in res)
        cpu = sum(r[3] for r in res)
        return {"value": n / span, "unit": "subcarriers/s", "cores": len(shares), "kind": "oracle",
                "cpu_model": cpu_model(),
                "sample": f"PD L-MMSE complex128 NumPy oracle, {len(shares)} processes x 1 thread over the "
                          f"step's {self.frames} x {W_FRAME} subcarriers, ~{self.seconds:g} s each: {n} "
                          f"systems in {span:.1f} s wall, {cpu:.1f} s CPU"}

    def close(self):
        self.pool.terminate()
        self.pool.join()


COMPACT_VARIANT_KEYS = ("call_ms_mean", "hbm_frac")
COMPACT_BF16_KEYS = ("form", "speedup", "hbm_frac", "parity_max_rel_err_z")
COMPACT_DROP_ROOFLINE = ("alg_bytes_per_system", "call_GBps")


def compact_record(out, full_path=None):
    """The driver-facing last line: the headline, its roofline and the CPU
    baseline, the BF16-MFMA comparison and one short entry per timed form
    (the full record, with every other workload, goes to `full_path`)."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "settle_s", "ms_per_step", "higher_is_better",
            "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline",
            "bf16_mfma_vs_fp32")
    rec = {k: out[k] for k in keys if k in out}
    if "roofline" in rec:
        rec["roofline"] = {k: v for k, v in rec["roofline"].items() if k not in COMPACT_DROP_ROOFLINE}
    if "bf16_mfma_vs_fp32" in rec:
        rec["bf16_mfma_vs_fp32"] = {m: {k: v for k, v in c.items() if k in COMPACT_BF16_KEYS}
                                    for m, c in rec["bf16_mfma_vs_fp32"].items()}
    rec["forms_fields"] = list(COMPACT_VARIANT_KEYS)
    rec["forms"] = {k: [v.get(kk) for kk in COMPACT_VARIANT_KEYS] for k, v in out.get("variants", {}).items()}
    if full_path:
        rec["full_record"] = os.path.relpath(full_path, ROOT) if full_path.startswith(ROOT) else full_path
    return _round_floats(rec)


def _round_floats(x, sig=5):
    """Floats to `sig` significant digits (the compact line stays under 2 KB,
    the driver keeps only the end of the output)."""
    if isinstance(x, float):
        return float(f"{x:.{sig}g}")
    if isinstance(x, dict):
        return {k: _round_floats(v, sig) for k, v in x.items()}
    if isinstance(x, list):
        return [_round_floats(v, sig) for v in x]
    return x


VARIANTS = [("pd", "fp32"), ("pd", "bf16x3"), ("pd", "bf16_refine"), ("pd", "bf16x3_refine"),
            ("fd", "fp32"), ("fd", "bf16x3"), ("fd", "bf16x3_refine")]
# FD with the single-BF16 Gram is refused by the library (EQ_ENOTSUP): its
# fusion weights come from diag(A_c^-1) of the rounded Gram and miss the
# 2e-4 gate after refinement.


def _per_call(fn, steps):
    """Per-call HIP-event times (ms) of `steps` calls, each bracketed by its
    own event pair (the pairs add a gap of their own between calls, so these
    describe the spread, not the throughput)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    return np.array([e0.elapsed_time(e1) for e0, e1 in ev])


def settle(fn, seconds):
    """Untimed calls of `fn` for about `seconds` of wall time, before a form is
    timed.  The GPU raises its clocks only after several milliseconds of
    sustained load; after host-side work (input generation, the previous
    form's oracle check: the device idle for up to seconds) a form's few
    warmup steps and short timed region would otherwise run at the idle
    clocks (about 15% slower for PD FP32, which a second pass of the same
    calls does not show)."""
    import torch
    t0 = time.perf_counter()
    n = 0
    while True:
        for _ in range(16):
            fn()
        n += 16
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return n


def _timed(fn, steps, warmup):
    """Mean time per call (ms) of `steps` back-to-back calls between one pair
    of HIP events on the current stream, plus median / p10 / p90 of calls
    timed one by one."""
    import torch
    if _SETTLE_S[0] > 0:
        settle(fn, _SETTLE_S[0])
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    per = _per_call(fn, steps)
    return {"call_ms_mean": e0.elapsed_time(e1) / steps, "call_ms_median": float(np.median(per)),
            "call_ms_p10": float(np.percentile(per, 10)), "call_ms_p90": float(np.percentile(per, 90))}


def _rel_err(zg, zr):
    return float(np.max(np.max(np.abs(zg - zr), -1) / np.max(np.abs(zr), -1)))


NSYM = 14  # OFDM symbols per coherence interval (Section VI-B)


def bytes_per_system_sym(B, U, S):
    """Algorithmic HBM bytes of one channel matrix with S receive vectors."""
    return B * U * 8 + S * B * 8 + S * U * 8 + U * 4


def symbol_inputs(Hn, S, seed=11):
    from paper_1808_04473_amd import synth
    Yn, _ = synth.symbols_for_channels(Hn, S, SNR_DB, "16qam", seed)
    return Yn


def symbol_measurements(Hn, n0, off, H, steps, S, tag):
    """eq_pd_sym / eq_fd_sym with S receive vectors per channel matrix, both
    one-pass forms, against S single-vector calls of the same form."""
    import torch
    import oracle
    from paper_1808_04473_amd import api
    dev = torch.device("cuda:0")
    W, Bs, Us = Hn.shape
    Hd = torch.from_numpy(Hn).to(dev) if H is None else H
    Yn = symbol_inputs(Hn, S)
    Y = torch.from_numpy(Yn).to(dev)
    y1 = Y[:, 0, :].contiguous()
    samp = np.arange(0, W, max(1, W // 48))
    sel = torch.from_numpy(samp).to(dev)
    nb = W * bytes_per_system_sym(Bs, Us, S)
    out = {}
    # LAMA (T_max = 2, 16-QAM) over the same vectors, against 14 single-vector LAMA calls
    for mode in ("pd", "fd"):
        fs = api.eq_pd_lama_sym if mode == "pd" else api.eq_fd_lama_sym
        f1 = api.eq_pd_lama if mode == "pd" else api.eq_fd_lama
        rf = oracle.eq_pd_lama if mode == "pd" else oracle.eq_fd_lama
        t = _timed(lambda: fs(Hd, Y, n0, off, t_max=2, qam=16), steps, 3)
        t1 = _timed(lambda: f1(Hd, y1, n0, off, t_max=2, qam=16), steps, 3)
        z, s2 = fs(Hd, Y, n0, off, t_max=2, qam=16)
        zs = z[sel].cpu().numpy()
        errs = [_rel_err(zs[:, s], rf(Hn[samp], Yn[samp, s], n0, off, 2, 16)[0]) for s in range(0, S, 5)]
        t.update({"subcarriers_per_s": W / (t["call_ms_mean"] * 1e-3),
                  "vectors_per_s": W * S / (t["call_ms_mean"] * 1e-3),
                  "alg_GBps": (nb + W * S * Us * 4) / (t["call_ms_mean"] * 1e-3) / 1e9,
                  "single_vector_call_ms_mean": t1["call_ms_mean"],
                  "speedup_vs_single_vector_calls": S * t1["call_ms_mean"] / t["call_ms_mean"],
                  "parity_max_rel_err_z": float(max(errs))})
        t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
        out[f"symbols{S}_{tag}_{mode}_lama_T2_fp32"] = t
        del z, s2
    for mode in ("pd", "fd"):
        fs = api.eq_pd_sym if mode == "pd" else api.eq_fd_sym
        f1 = api.eq_pd if mode == "pd" else api.eq_fd
        zr, sr = (oracle.eq_pd_symbols if mode == "pd" else oracle.eq_fd_symbols)(Hn[samp], Yn[samp], n0, off)
        for prec in ("fp32", "bf16x3"):
            t = _timed(lambda: fs(Hd, Y, n0, off, precision=prec), steps, 3)
            t1 = _timed(lambda: f1(Hd, y1, n0, off, precision=prec), steps, 3)
            z, s2 = fs(Hd, Y, n0, off, precision=prec)
            t.update({"subcarriers_per_s": W / (t["call_ms_mean"] * 1e-3),
                      "vectors_per_s": W * S / (t["call_ms_mean"] * 1e-3),
                      "alg_GBps": nb / (t["call_ms_mean"] * 1e-3) / 1e9,
                      "single_vector_call_ms_mean": t1["call_ms_mean"],
                      "speedup_vs_single_vector_calls": S * t1["call_ms_mean"] / t["call_ms_mean"],
                      "parity_max_rel_err_z": _rel_err(z[sel].cpu().numpy(), zr),
                      "parity_max_sigma2_db": float(np.max(np.abs(10 * np.log10(s2[sel].cpu().numpy() / sr))))})
            t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
            out[f"symbols{S}_{tag}_{mode}_{prec}"] = t
            del z, s2
    del Y, y1
    return out


def extra_measurements(Hn, yn, n0, off, H, y, steps):
    """The other rows of the path, each timed the same way and parity-sampled
    against the oracle: single-frame latency (W = 1200), the headline sweep
    replayed from a HIP graph, the B = 1024 / U = 32
    workload in every precision form, ragged batches of 4096 systems, ZF,
    MRC and LAMA on the headline systems, 14 receive vectors per channel
    matrix, and the FD forward + adjoint of the differentiation workload."""
    import torch
    import oracle
    from paper_1808_04473_amd import api, synth
    dev = H.device
    out = {}
    # single frame of the headline workload
    H1, y1 = H[:W_FRAME].contiguous(), y[:W_FRAME].contiguous()
    for mode, fn in (("pd", api.eq_pd), ("fd", api.eq_fd)):
        out[f"latency_w{W_FRAME}_{mode}_fp32"] = _timed(lambda: fn(H1, y1, n0, off), steps, 3)

    # one sweep of the headline workload captured in a HIP graph and replayed:
    # the same launches without the host side of a call; each replay must
    # reproduce the eager result exactly
    W, B, U = H.shape
    for mode, fn in (("pd", api.eq_pd), ("fd", api.eq_fd)):
        zg = torch.empty((W, U), dtype=torch.complex64, device=dev)
        sg = torch.empty((W, U), dtype=torch.float32, device=dev)
        ig = torch.empty((W,) if mode == "pd" else (W, len(off) - 1), dtype=torch.int32, device=dev)
        prob, _o = api.make_problem(W, B, U, off, n0)
        wsg = api.workspace(prob, dev)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn(H, y, n0, off, out=(zg, sg, ig), ws=wsg)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn(H, y, n0, off, out=(zg, sg, ig), ws=wsg)
        t = _timed(g.replay, steps, 3)
        ze, se = fn(H, y, n0, off)
        torch.cuda.synchronize()
        t.update({"subcarriers_per_s": W / (t["call_ms_mean"] * 1e-3),
                  "alg_GBps": W * bytes_per_system() / (t["call_ms_mean"] * 1e-3) / 1e9,
                  "replay_equals_eager": bool(torch.equal(torch.view_as_real(zg), torch.view_as_real(ze))
                                              and torch.equal(sg, se))})
        t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
        out[f"graph_replay_B256_U16_{mode}_fp32"] = t
        del g

    # B = 1024 antennas in 16 clusters of 64, U = 32, 4 frames x 1200 (1.3 GB of H)
    c3 = [synth.config_batch(3, 10.0, frame=f) for f in range(4)]
    H3n = np.concatenate([b.H for b in c3]); y3n = np.concatenate([b.y for b in c3])
    n03, off3 = c3[0].n0, c3[0].cluster_off
    H3, y3 = torch.from_numpy(H3n).to(dev), torch.from_numpy(y3n).to(dev)
    W3, B3, U3 = H3n.shape
    bps3 = bytes_per_system(B3, U3)
    samp = np.arange(0, W3, W3 // 32)
    ref3 = {"pd": oracle.eq_pd(H3n[samp], y3n[samp], n03, off3), "fd": oracle.eq_fd(H3n[samp], y3n[samp], n03, off3)}
    for mode in ("pd", "fd"):
        fn = api.eq_pd if mode == "pd" else api.eq_fd
        for prec in ("fp32", "bf16x3", "bf16_refine", "bf16x3_refine"):
            if mode == "fd" and prec == "bf16_refine":
                continue
            t = _timed(lambda: fn(H3, y3, n03, off3, precision=prec), steps, 3)
            z, s2, info = fn(H3, y3, n03, off3, precision=prec, return_info=True)
            routed = ((info & (1 << 30)) != 0)
            routed = routed.any(dim=-1) if mode == "fd" else routed
            zr, sr = ref3[mode]
            sel = torch.from_numpy(samp).to(dev)
            t.update({"systems_per_s": W3 / (t["call_ms_mean"] * 1e-3),
                      "alg_GBps": W3 * bps3 / (t["call_ms_mean"] * 1e-3) / 1e9,
                      "fp64_routed": int(routed.sum().item()),
                      "parity_max_rel_err_z": _rel_err(z[sel].cpu().numpy(), zr),
                      "parity_max_sigma2_db": float(np.max(np.abs(10 * np.log10(s2[sel].cpu().numpy() / sr))))})
            out[f"B1024_U32_{mode}_{prec}"] = t
    del H3, y3

    # ragged: 4 independent batches of 4096 systems (beyond the Infinity Cache)
    rbs = [synth.make_ragged(4096, seed=synth.BASE_SEED + 4 + 17 * k) for k in range(4)]
    pools = [(torch.from_numpy(rb.H_pool).to(dev), torch.from_numpy(rb.y_pool).to(dev)) for rb in rbs]
    nbytes = sum(int(np.sum(rb.B.astype(np.int64) * rb.U * 8 + rb.B * 8 + rb.U * 12)) for rb in rbs)
    for fd in (False, True):
        plans = [api.Plan.from_ragged(rb, fd=fd) for rb in rbs]

        def run_all():
            for pl, (hp, yp) in zip(plans, pools):
                pl.execute(hp, yp)
        t = _timed(run_all, steps, 2)
        t.update({"systems_per_s": 4 * 4096 / (t["call_ms_mean"] * 1e-3),
                  "alg_GBps": nbytes / (t["call_ms_mean"] * 1e-3) / 1e9,
                  "plan_shape": plans[0].describe()})
        rb, (hp, yp) = rbs[0], pools[0]
        z, s2, info = plans[0].execute(hp, yp)
        zh = z.cpu().numpy()
        errs = []
        for k in range(0, rb.nsys, 97):
            Bk, Uk = int(rb.B[k]), int(rb.U[k])
            Hk = rb.H_pool[rb.h_off[k]:rb.h_off[k] + Bk * Uk].reshape(1, Bk, Uk)
            yk = rb.y_pool[rb.y_off[k]:rb.y_off[k] + Bk].reshape(1, Bk)
            offk = np.concatenate([[0], np.cumsum(rb.cluster_sizes[rb.clus_first[k]:rb.clus_first[k] + rb.C[k]])])
            zr, _ = (oracle.eq_fd if fd else oracle.eq_pd)(Hk, yk, float(rb.n0[k]), offk)
            errs.append(_rel_err(zh[rb.z_off[k]:rb.z_off[k] + Uk][None], zr))
        t["parity_max_rel_err_z"] = float(max(errs))
        out[f"ragged_4x4096_{'fd' if fd else 'pd'}_fp32"] = t
        for pl in plans:
            pl.close()
    del pools

    # ZF, MRC and unbiased L-MMSE on the headline systems (same Gram pass,
    # different solve or output scaling)
    samp2 = np.arange(0, Hn.shape[0], Hn.shape[0] // 48)
    sel2 = torch.from_numpy(samp2).to(dev)
    for mode in ("pd", "fd"):
        fn = api.eq_pd if mode == "pd" else api.eq_fd
        rf = oracle.eq_pd_linear if mode == "pd" else oracle.eq_fd_linear
        for kind in ("zf", "mrc", "lmmse_unbiased"):
            for prec in ("fp32", "bf16x3"):
                t = _timed(lambda: fn(H, y, n0, off, precision=prec, equalizer=kind), steps, 3)
                z, s2 = fn(H, y, n0, off, precision=prec, equalizer=kind)
                zr, sr = rf(Hn[samp2], yn[samp2], n0, off, kind)
                t.update({"subcarriers_per_s": H.shape[0] / (t["call_ms_mean"] * 1e-3),
                          "alg_GBps": H.shape[0] * bytes_per_system() / (t["call_ms_mean"] * 1e-3) / 1e9,
                          "parity_max_rel_err_z": _rel_err(z[sel2].cpu().numpy(), zr),
                          "parity_max_sigma2_db": float(np.max(np.abs(10 * np.log10(s2[sel2].cpu().numpy() / sr))))})
                t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
                out[f"{kind}_B256_U16_{mode}_{prec}"] = t

    # LAMA-PD / LAMA-FD (Algorithm 1), 16-QAM, on the headline systems
    for mode in ("pd", "fd"):
        fn = api.eq_pd_lama if mode == "pd" else api.eq_fd_lama
        rf = oracle.eq_pd_lama if mode == "pd" else oracle.eq_fd_lama
        for t_max in (1, 2, 3):
            for prec in ("fp32", "bf16x3"):
                t = _timed(lambda: fn(H, y, n0, off, t_max=t_max, qam=16, precision=prec), steps, 3)
                z, s2 = fn(H, y, n0, off, t_max=t_max, qam=16, precision=prec)
                zr, sr = rf(Hn[samp2], yn[samp2], n0, off, t_max, 16)
                t.update({"subcarriers_per_s": H.shape[0] / (t["call_ms_mean"] * 1e-3),
                          "alg_GBps": H.shape[0] * bytes_per_system() / (t["call_ms_mean"] * 1e-3) / 1e9,
                          "parity_max_rel_err_z": _rel_err(z[sel2].cpu().numpy(), zr),
                          "parity_max_sigma2_db": float(np.max(np.abs(10 * np.log10(s2[sel2].cpu().numpy() / sr))))})
                t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
                out[f"lama_T{t_max}_B256_U16_{mode}_{prec}"] = t

    # several receive vectors per channel matrix: 14 OFDM symbols per subcarrier
    # on the headline channels and on the B = 1024 / U = 32 channels
    out.update(symbol_measurements(Hn, n0, off, H, steps, NSYM, "B256_U16"))
    out.update(symbol_measurements(H3n, n03, off3, None, steps, NSYM, "B1024_U32"))

    # differentiation workload: FD forward + adjoint (w.r.t. H, y, N0), 38,400 systems
    gz = torch.randn(H.shape[0], U, dtype=torch.complex64, device=dev)

    def fwd_bwd():
        api.eq_fd(H, y, n0, off)
        api.eq_fd_backward(H, y, n0, off, gz=gz)
    t = _timed(fwd_bwd, max(5, steps // 5), 2)
    W = H.shape[0]
    # forward reads H, y; adjoint reads H, y and writes grad_H, grad_y
    t.update({"systems_per_s": W / (t["call_ms_mean"] * 1e-3),
              "alg_GBps": W * (3 * B * U * 8 + 3 * B * 8) / (t["call_ms_mean"] * 1e-3) / 1e9})
    out["fd_forward_adjoint_fp32"] = t
    return out


def copy_probe(mib, dev):
    """One plain device copy of `mib` MiB: the scale reference of the HBM
    counters (FETCH_SIZE / WRITE_SIZE) in a rocprofv3 --pmc run."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def symbols_main(args, dev):
    """--nsym S: the headline channels with S receive vectors each, timed per
    variant the same way (one JSON line; not the headline metric)."""
    import torch
    Hn, _, n0, off = make_inputs(args.frames)
    W = Hn.shape[0]
    H = torch.from_numpy(Hn).to(dev)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib, dev)
    variants = [("pd", "fp32"), ("pd", "bf16x3"), ("fd", "fp32"), ("fd", "bf16x3")] \
        if args.variants == "all" else [tuple(v.split(":")) for v in args.variants.split(",")]
    r = symbol_measurements(Hn, n0, off, H, args.steps, args.nsym, "B256_U16")
    res = {f"{m}_{p}": r[f"symbols{args.nsym}_B256_U16_{m}_{p}"] for m, p in variants}
    print(json.dumps({"metric": f"equalized receive vectors/s @B={B},U={U},C={C},N_sym={args.nsym}",
                      "unit": "receive vectors/s", "n_gpus": 1, "steps": args.steps,
                      "config": {"workload": f"{W} subcarriers x {args.nsym} OFDM symbols, B={B}, C={C}, U={U}"},
                      "variants": res}), flush=True)
    return 0


def focused_main(args, dev):
    """--workload b1024 | ragged | adjoint: one workload timed alone, for
    focused rocprofv3 runs (one JSON line; not the headline metric).

    b1024:   B = 1024 antennas in 16 clusters of 64, U = 32, 4 frames x 1200
             subcarriers (1.3 GB of H), every form in --variants;
    ragged:  4 independent batches of 4096 ragged systems (--variants modes);
    adjoint: FD forward and adjoint (grad H, y, N0) on the headline systems."""
    import torch
    from paper_1808_04473_amd import api, synth
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib, dev)
    res = {}
    if args.workload == "b1024":
        c3 = [synth.config_batch(3, 10.0, frame=f) for f in range(4)]
        H = torch.from_numpy(np.concatenate([b.H for b in c3])).to(dev)
        y = torch.from_numpy(np.concatenate([b.y for b in c3])).to(dev)
        n0, off = c3[0].n0, c3[0].cluster_off
        W, Bb, Ub = H.shape
        variants = [v for v in VARIANTS] if args.variants == "all" else \
            [tuple(v.split(":")) for v in args.variants.split(",")]
        for mode, prec in variants:
            fn = api.eq_pd if mode == "pd" else api.eq_fd
            t = _timed(lambda: fn(H, y, n0, off, precision=prec), args.steps, args.warmup)
            t["systems_per_s"] = W / (t["call_ms_mean"] * 1e-3)
            t["alg_GBps"] = W * bytes_per_system(Bb, Ub) / (t["call_ms_mean"] * 1e-3) / 1e9
            t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
            res[f"{mode}_{prec}"] = t
        workload = f"B={Bb}, C=16, U={Ub}, {W} systems per call"
    elif args.workload == "ragged":
        rbs = [synth.make_ragged(4096, seed=synth.BASE_SEED + 4 + 17 * k) for k in range(4)]
        pools = [(torch.from_numpy(rb.H_pool).to(dev), torch.from_numpy(rb.y_pool).to(dev)) for rb in rbs]
        nbytes = sum(int(np.sum(rb.B.astype(np.int64) * rb.U * 8 + rb.B * 8 + rb.U * 12)) for rb in rbs)
        modes = ["pd", "fd"] if args.variants == "all" else [v.split(":")[0] for v in args.variants.split(",")]
        for mode in modes:
            plans = [api.Plan.from_ragged(rb, fd=mode == "fd") for rb in rbs]

            def run_all():
                for pl, (hp, yp) in zip(plans, pools):
                    pl.execute(hp, yp)
            t = _timed(run_all, args.steps, args.warmup)
            t["systems_per_s"] = 4 * 4096 / (t["call_ms_mean"] * 1e-3)
            t["alg_GBps"] = nbytes / (t["call_ms_mean"] * 1e-3) / 1e9
            t["hbm_frac"] = t["alg_GBps"] / HBM_PEAK_GBS
            t["alg_bytes_per_call"] = nbytes
            res[f"{mode}_fp32"] = t
            for pl in plans:
                pl.close()
        workload = "4 batches x 4096 ragged systems (B_c in {16,24,32,48,64}, C in 2..16, U in {8,16,24,32})"
    else:  # adjoint
        Hn, yn, n0, off = make_inputs(args.frames)
        H, y = torch.from_numpy(Hn).to(dev), torch.from_numpy(yn).to(dev)
        W = H.shape[0]
        gz = torch.randn(W, U, dtype=torch.complex64, device=dev)
        tf = _timed(lambda: api.eq_fd(H, y, n0, off), args.steps, args.warmup)
        tb = _timed(lambda: api.eq_fd_backward(H, y, n0, off, gz=gz), args.steps, args.warmup)
        # the adjoint reads H, y and grad_z and writes grad_H and grad_y
        bb = W * (2 * B * U * 8 + 2 * B * 8 + U * 8)
        tb.update({"systems_per_s": W / (tb["call_ms_mean"] * 1e-3),
                   "alg_GBps": bb / (tb["call_ms_mean"] * 1e-3) / 1e9, "alg_bytes_per_call": bb})
        tb["hbm_frac"] = tb["alg_GBps"] / HBM_PEAK_GBS
        res = {"fd_forward_fp32": tf, "fd_backward_fp32": tb}
        workload = f"FD B={B}, C={C}, U={U}, {W} systems per call"
    print(json.dumps({"workload": args.workload, "config": {"workload": workload}, "steps": args.steps,
                      "results": res}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=32)
    ap.add_argument("--variants", default="all",
                    help="comma list of mode:prec (e.g. pd:fp32,fd:bf16x3_refine) or 'all'")
    ap.add_argument("--cpu-seconds", type=float, default=CPU_MIN_SECONDS,
                    help="wall time of each oracle worker process in the CPU baseline")
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="oracle worker processes (default: the host CPUs, at most 16)")
    ap.add_argument("--full-out", default=os.path.join(ROOT, "gpurun_out", "bench_full.json"),
                    help="where the full record (every workload) is written; '' = nowhere")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (B=1024/U=32, ragged, adjoint, latency)")
    ap.add_argument("--nsym", type=int, default=1,
                    help="time eq_pd_sym / eq_fd_sym with this many receive vectors per channel "
                         "matrix instead of the headline workload (for focused profiles)")
    ap.add_argument("--workload", choices=["headline", "b1024", "ragged", "adjoint"], default="headline",
                    help="time one other workload alone (focused profiles; not the headline metric)")
    ap.add_argument("--settle-s", type=float, default=SETTLE_S,
                    help="seconds of untimed calls of each form before its warmup steps, so "
                         "that the timed steps run at the device's loaded clocks (0 = none)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (PMC scale reference)")
    args = ap.parse_args(argv)
    _SETTLE_S[0] = args.settle_s

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one MI355X: the equaliser is data-parallel over subcarriers "
              "and this build has no multi-GPU path (--gpus must be 1).", file=sys.stderr)
        return 2

    # the oracle's worker processes are forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline and args.nsym == 1 and args.workload == "headline":
        cpu = CpuBaseline(args.frames, args.cpu_seconds, args.cpu_cores or None)
    try:
        return _gpu_main(args, cpu)
    finally:
        if cpu is not None:
            cpu.close()


def _gpu_main(args, cpu):
    import torch
    from paper_1808_04473_amd import api
    api.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.nsym > 1:
        return symbols_main(args, dev)
    if args.workload != "headline":
        return focused_main(args, dev)

    t_gen = time.perf_counter()
    Hn, yn, n0, off = make_inputs(args.frames)
    gen_s = time.perf_counter() - t_gen
    W = Hn.shape[0]
    H = torch.from_numpy(Hn).to(dev)
    y = torch.from_numpy(yn).to(dev)
    torch.cuda.synchronize()

    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib, dev)

    variants = VARIANTS if args.variants == "all" else [tuple(v.split(":")) for v in args.variants.split(",")]
    bps = bytes_per_system()
    results = {}
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(W, size=min(256, W), replace=False))
    for mode, prec in variants:
        z = torch.empty((W, U), dtype=torch.complex64, device=dev)
        s2 = torch.empty((W, U), dtype=torch.float32, device=dev)
        info = torch.empty((W,) if mode == "pd" else (W, C), dtype=torch.int32, device=dev)
        prob, _k = api.make_problem(W, B, U, off, n0, 1.0, prec)
        ws = api.workspace(prob, dev)
        fn = api.eq_pd if mode == "pd" else api.eq_fd

        def step():
            fn(H, y, n0, off, precision=prec, out=(z, s2, info), ws=ws)

        if args.settle_s > 0:
            settle(step, args.settle_s)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # the timed region: K back-to-back steps between one pair of HIP events
        # on the library's stream, synchronised on both sides
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        call_ms = e0.elapsed_time(e1) / args.steps
        per = _per_call(step, min(args.steps, 20))  # spread of single calls
        ms = wall * 1e3 / args.steps
        r = {"ms_per_step": ms, "subcarriers_per_s": W / (ms * 1e-3), "call_ms_mean": call_ms,
             "call_ms_median_single": float(np.median(per)), "call_ms_p10_single": float(np.percentile(per, 10)),
             "call_ms_p90_single": float(np.percentile(per, 90)),
             "alg_GBps": W * bps / (call_ms * 1e-3) / 1e9}
        r["hbm_frac"] = r["alg_GBps"] / HBM_PEAK_GBS
        # the same K steps again with the library's kernel timer on: HIP events
        # recorded around the Gram + solve launch alone, on the call's stream
        with api.KernelTimer(args.steps) as kt:
            for _ in range(args.steps):
                step()
        r["kernel_ms_mean"] = kt.mean_ms
        r["kernel_launches_timed"] = kt.count
        r["kernel_alg_GBps"] = W * bps / (kt.mean_ms * 1e-3) / 1e9
        r["kernel_hbm_frac"] = r["kernel_alg_GBps"] / HBM_PEAK_GBS
        r["fp64_routed"] = int(((info & (1 << 30)) != 0).any(dim=-1).sum().item()) if mode == "fd" \
            else int(((info & (1 << 30)) != 0).sum().item())
        if not args.no_parity:
            import oracle
            Hs, ys = Hn[sample], yn[sample]
            if mode == "pd":
                zr, sr = oracle.eq_pd(Hs, ys, n0, off)
            else:
                zr, sr = oracle.eq_fd(Hs, ys, n0, off)
            zg = z[torch.from_numpy(sample).to(dev)].cpu().numpy()
            sg = s2[torch.from_numpy(sample).to(dev)].cpu().numpy()
            r["parity_max_rel_err_z"] = float(np.max(np.max(np.abs(zg - zr), -1) / np.max(np.abs(zr), -1)))
            r["parity_max_sigma2_db"] = float(np.max(np.abs(10 * np.log10(sg / sr))))
        results[f"{mode}_{prec}"] = r
        print(f"# {mode} {prec}: {ms:.3f} ms/step, {r['subcarriers_per_s'] / 1e6:.2f} M subcarriers/s, "
              f"{r['alg_GBps']:.0f} GB/s ({100 * r['hbm_frac']:.1f}% of HBM peak)", file=sys.stderr, flush=True)
        del z, s2, info, ws

    # practical read ceiling of this device: one nontemporal read of the same H
    ceiling = None
    if not args.no_extras:
        nb = api.probe_read(H)
        t = _timed(lambda: api.probe_read(H), min(args.steps, 20), 3)
        ceiling = nb / (t["call_ms_mean"] * 1e-3) / 1e9
        for r in results.values():
            r["frac_of_read_ceiling"] = r["alg_GBps"] / ceiling
            r["kernel_frac_of_read_ceiling"] = r["kernel_alg_GBps"] / ceiling

    head_key = "pd_fp32" if "pd_fp32" in results else next(iter(results))
    head = results[head_key]
    launch_bytes = W * bps
    traffic = load_traffic(head_key)
    out = {
        "metric": "equalized subcarriers/s @B=256,U=16,C=8: FP32 vs BF16-MFMA; % HBM roofline",
        "value": head["subcarriers_per_s"],
        "unit": "subcarriers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": args.settle_s,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"PD L-MMSE, B={B} (C={C} x {B // C}), U={U}, {args.frames} x {W_FRAME} = {W} "
                               f"subcarriers per step, 16-QAM, {SNR_DB:g} dB, i.i.d. Rayleigh",
                   "B": B, "C": C, "U": U, "systems_per_step": W, "form": head_key},
        "roofline": {"bound": "hbm", "achieved": head["kernel_alg_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["kernel_hbm_frac"],
                     "traffic": traffic,
                     "kernel": "eq_forward_kernel<16, FP32, PD>",
                     "kernel_us_mean": head["kernel_ms_mean"] * 1e3,
                     "timing": f"kernel-timer HIP events on its stream, {head['kernel_launches_timed']} "
                               f"launches (second pass)",
                     "alg_bytes_per_launch": launch_bytes,
                     "alg_bytes_per_system": bps,
                     "call_GBps": head["alg_GBps"], "call_frac": head["hbm_frac"],
                     "read_ceiling_GBps": ceiling,
                     "frac_of_read_ceiling": None if ceiling is None else head["kernel_alg_GBps"] / ceiling},
        "variants": results,
        "input_generation_s": gen_s,
    }
    # the BF16-MFMA form against plain FP32 on the same systems
    for mode in ("pd", "fd"):
        a, b = results.get(f"{mode}_bf16x3"), results.get(f"{mode}_fp32")
        if a and b:
            out.setdefault("bf16_mfma_vs_fp32", {})[mode] = {
                "form": f"{mode}_bf16x3", "speedup": a["subcarriers_per_s"] / b["subcarriers_per_s"],
                "hbm_frac": a["hbm_frac"], "frac_of_read_ceiling": a.get("frac_of_read_ceiling"),
                "parity_max_rel_err_z": a.get("parity_max_rel_err_z"),
                "fp32_parity_max_rel_err_z": b.get("parity_max_rel_err_z")}
    if not args.no_extras:
        out["other_workloads"] = extra_measurements(Hn, yn, n0, off, H, y, min(args.steps, 20))
    if cpu is not None:
        out["cpu_baseline"] = cpu.run()
    full_path = args.full_out or None
    if full_path:
        try:
            os.makedirs(os.path.dirname(full_path), exist_ok=True)
            with open(full_path, "w") as f:
                json.dump(out, f, indent=1)
            print(f"# full record: {full_path}", file=sys.stderr, flush=True)
        except OSError as e:
            print(f"# full record not written ({e})", file=sys.stderr, flush=True)
            full_path = None
    print(json.dumps(compact_record(out, full_path)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
