"""Thin Python binding of libdbpeq.so (ctypes; argument marshalling only).

Every step of the equaliser runs in the library's HIP kernels; this module
checks tensor placement / dtype / shape, allocates outputs and workspace with
PyTorch (device memory and streams only) and calls the C ABI declared in
include/dbpeq.h on the current HIP stream.  If the library is not built the
calls raise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbpeq.so")

PRECISIONS = {"fp32": 0, "bf16_refine": 1, "bf16x3_refine": 2, "bf16x3": 3}
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported problem size",
          -3: "HIP runtime error", -4: "workspace missing or too small",
          -5: "device allocation failed"}
INFO_FP64 = 1 << 30


class EqError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({status})")
        self.status = status


class EqProblem(ctypes.Structure):
    _fields_ = [("W", c_int32), ("B", c_int32), ("U", c_int32), ("C", c_int32),
                ("cluster_off", POINTER(c_int32)), ("n0", c_float), ("es", c_float),
                ("precision", c_int32), ("equalizer", c_int32)]


class EqSys(ctypes.Structure):
    _fields_ = [("h_off", c_int64), ("y_off", c_int64), ("z_off", c_int64),
                ("B", c_int32), ("U", c_int32), ("C", c_int32), ("clus_first", c_int32),
                ("n0", c_float), ("_reserved", c_int32)]


_lib = None

# (name, restype, argtypes) of every exported entry point of include/dbpeq.h
SIGNATURES = [
    ("eq_abi_version", c_int32, []),
    ("eq_status_string", c_char_p, [c_int32]),
    ("eq_workspace_size", c_size_t, [POINTER(EqProblem)]),
    ("eq_backward_workspace_size", c_size_t, [POINTER(EqProblem)]),
    ("eq_pd", c_int32, [POINTER(EqProblem), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                        c_void_p, c_size_t, c_void_p]),
    ("eq_fd", c_int32, [POINTER(EqProblem), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                        c_void_p, c_void_p, c_size_t, c_void_p]),
    ("eq_pd_noalloc", c_int32, [POINTER(EqProblem), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p]),
    ("eq_pd_sym", c_int32, [POINTER(EqProblem), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p, c_size_t, c_void_p]),
    ("eq_fd_sym", c_int32, [POINTER(EqProblem), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("eq_pd_lama", c_int32, [POINTER(EqProblem), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p]),
    ("eq_fd_lama", c_int32, [POINTER(EqProblem), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p]),
    ("eq_pd_lama_sym", c_int32, [POINTER(EqProblem), c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p]),
    ("eq_fd_lama_sym", c_int32, [POINTER(EqProblem), c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("eq_pd_backward", c_int32, [POINTER(EqProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("eq_fd_backward", c_int32, [POINTER(EqProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_size_t, c_void_p]),
    ("eq_plan_create", c_int32, [POINTER(c_void_p), POINTER(EqSys), c_int32, POINTER(c_int32),
                                 c_int32, c_int32, c_int32, c_float, c_char_p]),
    ("eq_plan_execute", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p]),
    ("eq_plan_describe", c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    ("eq_plan_destroy", c_int32, [c_void_p]),
    ("eq_probe_read", c_int32, [c_void_p, c_size_t, c_void_p, c_void_p]),
    ("eq_kernel_timer_start", c_int32, [c_int32]),
    ("eq_kernel_timer_stop", c_int32, [POINTER(c_int32), POINTER(ctypes.c_double)]),
]


def load_library(path: str = LIB_PATH):
    """Load libdbpeq.so (built in-tree by paper_1808_04473_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1808_04473_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check(fn: str, st: int):
    if st != 0:
        raise EqError(fn, st)


EQUALIZERS = {"lmmse": 0, "zf": 1, "mrc": 2, "lmmse_unbiased": 3}


def make_problem(W, B, U, cluster_off, n0, es=1.0, precision="fp32", equalizer="lmmse"):
    """EqProblem plus the host offset array that must outlive the call."""
    off = np.ascontiguousarray(np.asarray(cluster_off, dtype=np.int32))
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    eqz = EQUALIZERS[equalizer] if isinstance(equalizer, str) else int(equalizer)
    p = EqProblem(int(W), int(B), int(U), int(len(off) - 1),
                  off.ctypes.data_as(POINTER(c_int32)), float(n0), float(es), prec, eqz)
    return p, off


def _check_inputs(H, y):
    if not (isinstance(H, torch.Tensor) and isinstance(y, torch.Tensor)):
        raise TypeError("H and y must be torch tensors")
    if H.device.type != "cuda" or y.device.type != "cuda":
        raise ValueError("H and y must be on a HIP device (no CPU fallback)")
    if H.dtype != torch.complex64 or y.dtype != torch.complex64:
        raise TypeError("H and y must be complex64")
    if H.device != y.device:
        raise ValueError("H and y must be on the same device")
    if H.dim() != 3 or y.dim() != 2 or H.shape[0] != y.shape[0] or H.shape[1] != y.shape[1]:
        raise ValueError(f"shapes H {tuple(H.shape)} / y {tuple(y.shape)} are not [W][B][U] / [W][B]")
    return H.contiguous(), y.contiguous()


def _check_tensor(name, t, shape, dtype, device):
    """A caller-supplied output or weight tensor: its pointer goes to the
    kernels, which trust its extent, so it must match exactly."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, not {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, not {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _outputs(out, zshape, s2shape, infoshape, device):
    """Output tensors: allocated here, or the caller's (z, sigma2, info)
    checked against the shapes the call writes (sigma2 and info may be None)."""
    if out is None:
        return (torch.empty(zshape, dtype=torch.complex64, device=device),
                torch.empty(s2shape, dtype=torch.float32, device=device),
                torch.empty(infoshape, dtype=torch.int32, device=device))
    if not isinstance(out, (tuple, list)) or len(out) != 3:
        raise ValueError("out must be a tuple (z, sigma2, info)")
    z, s2, info = out
    _check_tensor("out z", z, zshape, torch.complex64, device)
    if s2 is not None:
        _check_tensor("out sigma2", s2, s2shape, torch.float32, device)
    if info is not None:
        _check_tensor("out info", info, infoshape, torch.int32, device)
    return z, s2, info


def _check_nu(nu, W, C, U, device):
    if nu is None:
        return None
    if not isinstance(nu, torch.Tensor) or nu.dtype != torch.float32 or tuple(nu.shape) != (W, C, U) \
            or nu.device != device:
        raise ValueError("nu must be float32 [W][C][U] on the same device")
    return nu.contiguous()


def _check_ws(ws, device):
    if ws is None:
        return None
    if not isinstance(ws, torch.Tensor) or ws.device != device or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 tensor on the same device")
    return ws


def workspace(prob: EqProblem, device) -> torch.Tensor:
    lib = load_library()
    n = lib.eq_workspace_size(ctypes.byref(prob))
    # zero-filled once; every call leaves it zero-filled
    return torch.zeros(max(int(n), 256), dtype=torch.uint8, device=device)


# Forward workspaces kept per (device, stream): each call leaves its workspace
# zero-filled and calls on one stream are ordered, so one zero-fill serves
# every later call on that stream.
_WS_CACHE: dict = {}


def _cached_workspace(prob: EqProblem, device) -> torch.Tensor:
    lib = load_library()
    need = max(int(lib.eq_workspace_size(ctypes.byref(prob))), 256)
    key = (device.index if device.index is not None else torch.cuda.current_device(), _stream())
    ws = _WS_CACHE.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.zeros(need, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def eq_pd(H, y, n0, cluster_off, precision="fp32", es=1.0, return_info=False, out=None,
          ws=None, equalizer="lmmse"):
    """Partially decentralised equalisation of W systems (L-MMSE by default,
    or equalizer="zf" / "mrc" / "lmmse_unbiased"): (z [W][U] c64, sigma2 [W][U] f32).

    `out` = (z, sigma2, info) and `ws` (uint8 workspace) may be preallocated."""
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision, equalizer)
    z, s2, info = _outputs(out, (W, U), (W, U), (W,), H.device)
    ws = _cached_workspace(prob, H.device) if ws is None else _check_ws(ws, H.device)
    st = lib.eq_pd(ctypes.byref(prob), _ptr(H), _ptr(y), _ptr(z), _ptr(s2), _ptr(info),
                   _ptr(ws), ws.numel(), _stream())
    _check("eq_pd", st)
    return (z, s2, info) if return_info else (z, s2)


NOALLOC_MAX_W = 262144  # EQ_NOALLOC_MAX_W


def eq_pd_noalloc(H, y, n0, cluster_off, precision="fp32", es=1.0, return_info=False, out=None,
                  equalizer="lmmse"):
    """eq_pd with the library's own device array as its workspace (W at most
    NOALLOC_MAX_W).  The C call allocates nothing; pass `out` = (z, sigma2,
    info) to keep this wrapper from allocating the outputs."""
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision, equalizer)
    z, s2, info = _outputs(out, (W, U), (W, U), (W,), H.device)
    st = lib.eq_pd_noalloc(ctypes.byref(prob), _ptr(H), _ptr(y), _ptr(z), _ptr(s2), _ptr(info), _stream())
    _check("eq_pd_noalloc", st)
    return (z, s2, info) if return_info else (z, s2)


def eq_fd(H, y, n0, cluster_off, nu=None, precision="fp32", es=1.0, return_info=False,
          out=None, ws=None, equalizer="lmmse"):
    """Fully decentralised equalisation (L-MMSE, "zf", "mrc" or "lmmse_unbiased" per cluster);
    nu [W][C][U] float32 user weights or None (optimal)."""
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision, equalizer)
    C = prob.C
    nu = _check_nu(nu, W, C, U, H.device)
    z, s2, info = _outputs(out, (W, U), (W, U), (W, C), H.device)
    ws = _cached_workspace(prob, H.device) if ws is None else _check_ws(ws, H.device)
    st = lib.eq_fd(ctypes.byref(prob), _ptr(H), _ptr(y), _ptr(nu), _ptr(z), _ptr(s2), _ptr(info),
                   _ptr(ws), ws.numel(), _stream())
    _check("eq_fd", st)
    return (z, s2, info) if return_info else (z, s2)


def _check_sym_inputs(H, Y):
    if not (isinstance(H, torch.Tensor) and isinstance(Y, torch.Tensor)):
        raise TypeError("H and Y must be torch tensors")
    if H.device.type != "cuda" or Y.device.type != "cuda":
        raise ValueError("H and Y must be on a HIP device (no CPU fallback)")
    if H.dtype != torch.complex64 or Y.dtype != torch.complex64:
        raise TypeError("H and Y must be complex64")
    if H.device != Y.device:
        raise ValueError("H and Y must be on the same device")
    if H.dim() != 3 or Y.dim() != 3 or H.shape[0] != Y.shape[0] or H.shape[1] != Y.shape[2]:
        raise ValueError(f"shapes H {tuple(H.shape)} / Y {tuple(Y.shape)} are not [W][B][U] / [W][S][B]")
    return H.contiguous(), Y.contiguous()


def _sym_call(fd, H, Y, n0, cluster_off, nu, precision, es, return_info, out, ws, equalizer):
    lib = load_library()
    H, Y = _check_sym_inputs(H, Y)
    W, B, U = H.shape
    S = Y.shape[1]
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision, equalizer)
    C = prob.C
    if nu is not None and not fd:
        raise ValueError("nu applies to FD only")
    nu = _check_nu(nu, W, C, U, H.device)
    z, s2, info = _outputs(out, (W, S, U), (W, U), (W, C) if fd else (W,), H.device)
    ws = _cached_workspace(prob, H.device) if ws is None else _check_ws(ws, H.device)
    if fd:
        st = lib.eq_fd_sym(ctypes.byref(prob), S, _ptr(H), _ptr(Y), _ptr(nu), _ptr(z), _ptr(s2),
                           _ptr(info), _ptr(ws), ws.numel(), _stream())
    else:
        st = lib.eq_pd_sym(ctypes.byref(prob), S, _ptr(H), _ptr(Y), _ptr(z), _ptr(s2), _ptr(info),
                           _ptr(ws), ws.numel(), _stream())
    _check("eq_fd_sym" if fd else "eq_pd_sym", st)
    return (z, s2, info) if return_info else (z, s2)


def eq_pd_sym(H, Y, n0, cluster_off, precision="fp32", es=1.0, return_info=False, out=None,
              ws=None, equalizer="lmmse"):
    """PD L-MMSE (or "zf" / "mrc" / "lmmse_unbiased") of S receive vectors per channel matrix: H [W][B][U],
    Y [W][S][B] -> (Z [W][S][U] c64, sigma2 [W][U] f32).  Precision "fp32" or "bf16x3"."""
    return _sym_call(False, H, Y, n0, cluster_off, None, precision, es, return_info, out, ws, equalizer)


def eq_fd_sym(H, Y, n0, cluster_off, nu=None, precision="fp32", es=1.0, return_info=False,
              out=None, ws=None, equalizer="lmmse"):
    """FD L-MMSE (or "zf" / "mrc" / "lmmse_unbiased") of S receive vectors per channel matrix (weights as eq_fd)."""
    return _sym_call(True, H, Y, n0, cluster_off, nu, precision, es, return_info, out, ws, equalizer)


def _lama_call(fd, H, y, n0, cluster_off, t_max, qam, nu, precision, es, return_info):
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision)
    C = prob.C
    if nu is not None and not fd:
        raise ValueError("nu applies to FD only")
    nu = _check_nu(nu, W, C, U, H.device)
    z = torch.empty((W, U), dtype=torch.complex64, device=H.device)
    s2 = torch.empty((W, U), dtype=torch.float32, device=H.device)
    info = torch.empty((W, C) if fd else (W,), dtype=torch.int32, device=H.device)
    if fd:
        st = lib.eq_fd_lama(ctypes.byref(prob), int(t_max), int(qam), _ptr(H), _ptr(y), _ptr(nu), _ptr(z),
                            _ptr(s2), _ptr(info), _stream())
    else:
        st = lib.eq_pd_lama(ctypes.byref(prob), int(t_max), int(qam), _ptr(H), _ptr(y), _ptr(z), _ptr(s2),
                            _ptr(info), _stream())
    _check("eq_fd_lama" if fd else "eq_pd_lama", st)
    return (z, s2, info) if return_info else (z, s2)


def eq_pd_lama(H, y, n0, cluster_off, t_max=2, qam=16, precision="fp32", es=1.0, return_info=False):
    """LAMA-PD (Algorithm 1) with t_max iterations for square QAM of `qam`
    points: (z [W][U] c64, sigma2 [W][U] f32)."""
    return _lama_call(False, H, y, n0, cluster_off, t_max, qam, None, precision, es, return_info)


def eq_fd_lama(H, y, n0, cluster_off, t_max=2, qam=16, nu=None, precision="fp32", es=1.0,
               return_info=False):
    """LAMA-FD: Algorithm 1 per normalised cluster, fused with Lemma 1's weights (or nu)."""
    return _lama_call(True, H, y, n0, cluster_off, t_max, qam, nu, precision, es, return_info)


def _lama_sym_call(fd, H, Y, n0, cluster_off, t_max, qam, nu, precision, es, return_info):
    lib = load_library()
    H, Y = _check_sym_inputs(H, Y)
    W, B, U = H.shape
    S = Y.shape[1]
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, precision)
    C = prob.C
    if nu is not None and not fd:
        raise ValueError("nu applies to FD only")
    nu = _check_nu(nu, W, C, U, H.device)
    z = torch.empty((W, S, U), dtype=torch.complex64, device=H.device)
    s2 = torch.empty((W, S, U), dtype=torch.float32, device=H.device)
    info = torch.empty((W, C) if fd else (W,), dtype=torch.int32, device=H.device)
    if fd:
        st = lib.eq_fd_lama_sym(ctypes.byref(prob), S, int(t_max), int(qam), _ptr(H), _ptr(Y), _ptr(nu),
                                _ptr(z), _ptr(s2), _ptr(info), _stream())
    else:
        st = lib.eq_pd_lama_sym(ctypes.byref(prob), S, int(t_max), int(qam), _ptr(H), _ptr(Y), _ptr(z),
                                _ptr(s2), _ptr(info), _stream())
    _check("eq_fd_lama_sym" if fd else "eq_pd_lama_sym", st)
    return (z, s2, info) if return_info else (z, s2)


def eq_pd_lama_sym(H, Y, n0, cluster_off, t_max=2, qam=16, precision="fp32", es=1.0, return_info=False):
    """LAMA-PD of S receive vectors per channel matrix: (Z [W][S][U], sigma2 [W][S][U])."""
    return _lama_sym_call(False, H, Y, n0, cluster_off, t_max, qam, None, precision, es, return_info)


def eq_fd_lama_sym(H, Y, n0, cluster_off, t_max=2, qam=16, nu=None, precision="fp32", es=1.0,
                   return_info=False):
    """LAMA-FD of S receive vectors per channel matrix (weights as eq_fd_lama)."""
    return _lama_sym_call(True, H, Y, n0, cluster_off, t_max, qam, nu, precision, es, return_info)


def _bwd_workspace(prob: EqProblem, device) -> torch.Tensor:
    lib = load_library()
    n = lib.eq_backward_workspace_size(ctypes.byref(prob))
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device=device)


def _grad_inputs(gz, gs, W, U, device):
    if gz is not None:
        if gz.dtype != torch.complex64 or tuple(gz.shape) != (W, U) or gz.device != device:
            raise ValueError("gz must be complex64 [W][U] on the device")
        gz = gz.contiguous()
    if gs is not None:
        if gs.dtype != torch.float32 or tuple(gs.shape) != (W, U) or gs.device != device:
            raise ValueError("gs must be float32 [W][U] on the device")
        gs = gs.contiguous()
    return gz, gs


def eq_pd_backward(H, y, n0, cluster_off, gz=None, gs=None, es=1.0):
    """Adjoint of eq_pd: (grad_H [W][B][U], grad_y [W][B], grad_N0 0-dim float32)."""
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, "fp32")
    gz, gs = _grad_inputs(gz, gs, W, U, H.device)
    gH = torch.empty_like(H)
    gy = torch.empty_like(y)
    gn0 = torch.zeros((), dtype=torch.float32, device=H.device)
    ws = _bwd_workspace(prob, H.device)
    st = lib.eq_pd_backward(ctypes.byref(prob), _ptr(H), _ptr(y), _ptr(gz), _ptr(gs), _ptr(gH),
                            _ptr(gy), _ptr(gn0), _ptr(ws), ws.numel(), _stream())
    _check("eq_pd_backward", st)
    return gH, gy, gn0


def eq_fd_backward(H, y, n0, cluster_off, gz=None, gs=None, nu=None, es=1.0):
    """Adjoint of eq_fd: (grad_H, grad_y, grad_N0, grad_nu or None)."""
    lib = load_library()
    H, y = _check_inputs(H, y)
    W, B, U = H.shape
    prob, _off = make_problem(W, B, U, cluster_off, n0, es, "fp32")
    gz, gs = _grad_inputs(gz, gs, W, U, H.device)
    nu = _check_nu(nu, W, prob.C, U, H.device)
    gnu = None if nu is None else torch.empty_like(nu)
    gH = torch.empty_like(H)
    gy = torch.empty_like(y)
    gn0 = torch.zeros((), dtype=torch.float32, device=H.device)
    ws = _bwd_workspace(prob, H.device)
    st = lib.eq_fd_backward(ctypes.byref(prob), _ptr(H), _ptr(y), _ptr(nu), _ptr(gz), _ptr(gs),
                            _ptr(gH), _ptr(gy), _ptr(gn0), _ptr(gnu), _ptr(ws), ws.numel(), _stream())
    _check("eq_fd_backward", st)
    return gH, gy, gn0, gnu


PLAN_CLASSES = 2        # EQ_PLAN_CLASSES
PLAN_CLASS_NAMES = ("ut16", "ut32")


class Plan:
    """A ragged batch of independent systems (eq_plan_* of the C ABI).

    desc arrays (numpy, length nsys): B, U, C, n0, h_off, y_off, z_off,
    clus_first; cluster_sizes (int32) holds every system's cluster sizes.
    Offsets are in complex elements of the pools passed to execute()."""

    def __init__(self, B, U, C, n0, h_off, y_off, z_off, clus_first, cluster_sizes, fd=False,
                 precision="fp32", es=1.0, tune_cache=None):
        lib = load_library()
        n = len(B)
        self.nsys = n
        self.fd = bool(fd)
        desc = (EqSys * n)()
        for k in range(n):
            desc[k] = EqSys(int(h_off[k]), int(y_off[k]), int(z_off[k]), int(B[k]), int(U[k]), int(C[k]),
                            int(clus_first[k]), float(n0[k]), 0)
        sizes = np.ascontiguousarray(np.asarray(cluster_sizes, dtype=np.int32))
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = c_void_p()
        st = lib.eq_plan_create(ctypes.byref(h), desc, n, sizes.ctypes.data_as(POINTER(c_int32)),
                                len(sizes), int(bool(fd)), prec, float(es),
                                None if tune_cache is None else str(tune_cache).encode())
        _check("eq_plan_create", st)
        self._h = h
        self._lib = lib
        Bn, Un = np.asarray(B, np.int64), np.asarray(U, np.int64)
        # elements of each pool that the descriptors address
        self.nh = int(max(np.asarray(h_off, np.int64) + Bn * Un)) if n else 0
        self.ny = int(max(np.asarray(y_off, np.int64) + Bn)) if n else 0
        self.nz = int(max(np.asarray(z_off, np.int64) + Un)) if n else 0

    @classmethod
    def from_ragged(cls, rb, fd=False, precision="fp32", tune_cache=None):
        return cls(rb.B, rb.U, rb.C, rb.n0, rb.h_off, rb.y_off, rb.z_off, rb.clus_first,
                   rb.cluster_sizes, fd=fd, precision=precision, es=rb.es, tune_cache=tune_cache)

    def execute(self, Hpool, ypool, out=None):
        """Equalises every system: (z pool, sigma2 pool, info [nsys]).  The
        pools must cover every descriptor's extent (checked here: the kernels
        trust the offsets)."""
        for name, t, need in (("Hpool", Hpool, self.nh), ("ypool", ypool, self.ny)):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.complex64 \
                    or not t.is_contiguous() or t.dim() != 1:
                raise ValueError(f"{name} must be a contiguous 1-D complex64 device tensor")
            if t.numel() < need:
                raise ValueError(f"{name} holds {t.numel()} elements; the descriptors address {need}")
        if ypool.device != Hpool.device:
            raise ValueError("Hpool and ypool must be on the same device")
        if out is None:
            z = torch.empty(self.nz, dtype=torch.complex64, device=Hpool.device)
            s2 = torch.empty(self.nz, dtype=torch.float32, device=Hpool.device)
            info = torch.empty(self.nsys, dtype=torch.int32, device=Hpool.device)
        else:
            if not isinstance(out, (tuple, list)) or len(out) != 3:
                raise ValueError("out must be a tuple (z, sigma2, info)")
            z, s2, info = out
            for name, t, dt, need in (("out z", z, torch.complex64, self.nz), ("out sigma2", s2, torch.float32, self.nz),
                                      ("out info", info, torch.int32, self.nsys)):
                if t is None and name != "out z":
                    continue
                if not isinstance(t, torch.Tensor) or t.device != Hpool.device or t.dtype != dt \
                        or not t.is_contiguous() or t.numel() < need:
                    raise ValueError(f"{name} must be a contiguous {dt} tensor of at least {need} elements "
                                     f"on {Hpool.device}")
        st = self._lib.eq_plan_execute(self._h, _ptr(Hpool), _ptr(ypool), _ptr(z), _ptr(s2), _ptr(info),
                                       _stream())
        _check("eq_plan_execute", st)
        return z, s2, info

    def describe(self):
        """Launch shape per tile class (padded users 16 / 32): systems, work
        items, PD row pieces (FD: clusters) and PD piece rows (0 = systems
        are not cut); the persistent waves of the launch and the total number
        of work items."""
        shape = (c_int32 * (5 * PLAN_CLASSES))()
        nt = c_int32()
        _check("eq_plan_describe", self._lib.eq_plan_describe(self._h, shape, ctypes.byref(nt)))
        classes = {}
        for k, name in enumerate(PLAN_CLASS_NAMES):
            v = shape[5 * k:5 * k + 5]
            if v[0]:
                key = "clusters" if self.fd else "pieces"
                classes[name] = {"systems": v[0], "items": v[1], key: v[2], "piece_rows": v[3]}
        return {"classes": classes, "grid": shape[4], "tasks": nt.value}

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check("eq_plan_destroy", self._lib.eq_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


KERNEL_TIMER_MAX = 65536  # EQ_KERNEL_TIMER_MAX


class KernelTimer:
    """Device time of the main kernel of the forward calls made inside the
    `with` block (eq_kernel_timer_*): on exit, `count` launches were timed
    and `mean_ms` is their average duration.  A measurement aid."""

    def __init__(self, capacity):
        self.capacity = int(capacity)
        self.count, self.total_ms = 0, 0.0

    def __enter__(self):
        _check("eq_kernel_timer_start", load_library().eq_kernel_timer_start(self.capacity))
        return self

    def __exit__(self, *exc):
        n, ms = c_int32(), ctypes.c_double()
        _check("eq_kernel_timer_stop", load_library().eq_kernel_timer_stop(ctypes.byref(n), ctypes.byref(ms)))
        self.count, self.total_ms = n.value, ms.value
        return False

    @property
    def mean_ms(self):
        return self.total_ms / self.count if self.count else float("nan")


def probe_read(t, sink=None):
    """Reads every byte of device tensor t once (eq_probe_read); time it on
    the current stream to obtain the practical HBM read ceiling."""
    lib = load_library()
    if t.device.type != "cuda" or not t.is_contiguous():
        raise ValueError("probe_read takes a contiguous device tensor")
    nbytes = t.numel() * t.element_size() // 16 * 16
    if sink is None:
        sink = torch.empty(1, dtype=torch.float32, device=t.device)
    _check("eq_probe_read", lib.eq_probe_read(_ptr(t), nbytes, _ptr(sink), _stream()))
    return nbytes
