"""The C ABI (no GPU needed): the library loads, exports every entry point the
header declares, and rejects invalid arguments on the host before any HIP
call (EQ_EINVAL / EQ_ENOTSUP / EQ_EWORKSPACE, no device side effects)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1808_04473_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbpeq.h")

EINVAL, ENOTSUP, EWORKSPACE = -1, -2, -4


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libdbpeq.so not built (run python -m paper_1808_04473_amd.build)")
    return api.load_library()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eq_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("eq_pd", "eq_fd", "eq_pd_backward", "eq_fd_backward", "eq_plan_create",
              "eq_plan_execute", "eq_plan_destroy", "eq_workspace_size", "eq_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == {s[0] for s in api.SIGNATURES}


def test_abi_version_and_status_strings(lib):
    assert lib.eq_abi_version() == 3
    for st, txt in api.STATUS.items():
        assert lib.eq_status_string(st).decode() == txt


def _prob(W=4, B=8, U=2, off=(0, 4, 8), n0=0.1, es=1.0, prec=0, eqz=0):
    return api.make_problem(W, B, U, list(off), n0, es, prec, eqz)


# dummy, suitably aligned host addresses: validation must reject before any use
FAKE = ctypes.create_string_buffer(1 << 16)
A = (ctypes.addressof(FAKE) + 255) // 256 * 256


def _call_pd(lib, prob, H=A, y=A, z=A, s2=A, info=A, ws=A, wsb=1 << 12):
    return lib.eq_pd(ctypes.byref(prob), H, y, z, s2, info, ws, wsb, None)


def _call_fd(lib, prob, nu=None, H=A, y=A, z=A, ws=A, wsb=1 << 12):
    return lib.eq_fd(ctypes.byref(prob), H, y, nu, z, A, A, ws, wsb, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(n0=0.0), EINVAL), (dict(n0=-1.0), EINVAL), (dict(n0=float("nan")), EINVAL),
    (dict(n0=float("inf")), EINVAL), (dict(es=0.0), EINVAL), (dict(es=float("nan")), EINVAL),
    (dict(off=(0, 4, 7)), EINVAL), (dict(off=(1, 4, 8)), EINVAL), (dict(off=(0, 4, 4, 8)), EINVAL),
    (dict(off=(0, 5, 4, 8)), EINVAL), (dict(U=0), EINVAL), (dict(U=33), ENOTSUP),
    (dict(W=-1), EINVAL), (dict(B=0, off=(0,)), EINVAL), (dict(prec=4), EINVAL), (dict(prec=7), EINVAL),
    (dict(prec=-1), EINVAL),
])
def test_invalid_problem_rejected(lib, kw, expect):
    prob, _keep = _prob(**kw)
    assert _call_pd(lib, prob) == expect
    assert _call_fd(lib, prob) == expect
    assert lib.eq_workspace_size(ctypes.byref(prob)) == 0


def test_too_many_clusters(lib):
    prob, _k = api.make_problem(1, 2000, 2, list(range(0, 2001)), 0.1)
    assert _call_pd(lib, prob) == ENOTSUP
    prob, _k = api.make_problem(1, 70000, 2, [0, 70000], 0.1)
    assert _call_pd(lib, prob) == ENOTSUP


def test_null_and_misaligned_pointers(lib):
    prob, _k = _prob()
    assert _call_pd(lib, prob, H=None) == EINVAL
    assert _call_pd(lib, prob, y=None) == EINVAL
    assert _call_pd(lib, prob, z=None) == EINVAL
    assert _call_pd(lib, prob, H=A + 4) == EINVAL
    assert _call_pd(lib, prob, z=A + 2) == EINVAL
    assert _call_pd(lib, prob, s2=A + 2) == EINVAL
    assert _call_fd(lib, prob, nu=A + 1) == EINVAL
    assert lib.eq_pd(None, A, A, A, A, A, A, 4096, None) == EINVAL


def test_workspace_checked(lib):
    prob, _k = _prob(W=1000)
    need = lib.eq_workspace_size(ctypes.byref(prob))
    assert need >= 256 + 4 * 1000
    assert _call_pd(lib, prob, ws=None) == EWORKSPACE
    assert _call_pd(lib, prob, wsb=need - 1) == EWORKSPACE


def test_zero_systems_is_a_noop(lib):
    prob, _k = _prob(W=0)
    # no HIP call happens for W = 0, so this is safe without a GPU
    assert lib.eq_pd(ctypes.byref(prob), None, None, None, None, None, None, 0, None) == 0
    assert lib.eq_fd(ctypes.byref(prob), None, None, None, None, None, None, None, 0, None) == 0


def test_probe_read_validation(lib):
    # all of these are rejected (or are no-ops) before any HIP call
    assert lib.eq_probe_read(A, 0, A, None) == 0
    assert lib.eq_probe_read(None, 1024, A, None) == EINVAL
    assert lib.eq_probe_read(A, 1024, None, None) == EINVAL
    assert lib.eq_probe_read(A + 8, 1024, A, None) == EINVAL
    assert lib.eq_probe_read(A, 1000, A, None) == EINVAL


def test_python_binding_refuses_cpu_tensors(lib):
    import torch
    H = torch.zeros((2, 4, 2), dtype=torch.complex64)
    y = torch.zeros((2, 4), dtype=torch.complex64)
    with pytest.raises(ValueError):
        api.eq_pd(H, y, 0.1, [0, 4])


def test_plan_validation(lib):
    import ctypes as ct
    desc = (api.EqSys * 2)()
    desc[0] = api.EqSys(0, 0, 0, 8, 2, 2, 0, 0.1, 0)
    desc[1] = api.EqSys(16, 8, 2, 8, 2, 2, 2, 0.1, 0)
    sizes = np.array([4, 4, 3, 5], np.int32)
    ps = sizes.ctypes.data_as(ct.POINTER(ct.c_int32))
    h = ct.c_void_p()
    # wrong cluster sizes sum (3 + 5 = 8 is fine; make it 9)
    bad = np.array([4, 4, 4, 5], np.int32)
    assert lib.eq_plan_create(ct.byref(h), desc, 2, bad.ctypes.data_as(ct.POINTER(ct.c_int32)), 4, 0, 0, 1.0, None) == EINVAL
    assert lib.eq_plan_create(ct.byref(h), desc, 0, ps, 4, 0, 0, 1.0, None) == EINVAL
    assert lib.eq_plan_create(ct.byref(h), desc, 2, ps, 4, 2, 0, 1.0, None) == EINVAL
    assert lib.eq_plan_create(ct.byref(h), desc, 2, ps, 4, 0, 9, 1.0, None) == EINVAL
    assert lib.eq_plan_create(ct.byref(h), desc, 2, ps, 3, 0, 0, 1.0, None) == EINVAL  # clusters past the table
    desc[1].n0 = 0.0
    assert lib.eq_plan_create(ct.byref(h), desc, 2, ps, 4, 0, 0, 1.0, None) == EINVAL
    desc[1].n0 = 0.1
    desc[1].U = 40
    assert lib.eq_plan_create(ct.byref(h), desc, 2, ps, 4, 0, 0, 1.0, None) == ENOTSUP
    assert lib.eq_plan_execute(None, A, A, A, A, A, None) == EINVAL
    assert lib.eq_plan_destroy(None) == 0


def _call_sym(lib, prob, nsym, fd=False, H=A, Y=A, Z=A, ws=A, wsb=1 << 12):
    if fd:
        return lib.eq_fd_sym(ctypes.byref(prob), nsym, H, Y, None, Z, A, A, ws, wsb, None)
    return lib.eq_pd_sym(ctypes.byref(prob), nsym, H, Y, Z, A, A, ws, wsb, None)


@pytest.mark.parametrize("fd", [False, True])
def test_symbols_validation(lib, fd):
    # all rejected (or no-ops) before any HIP call
    prob, _k = _prob()
    assert _call_sym(lib, prob, 0, fd) == EINVAL
    assert _call_sym(lib, prob, -3, fd) == EINVAL
    assert _call_sym(lib, prob, 1025, fd) == ENOTSUP
    assert _call_sym(lib, prob, 4, fd, Y=None) == EINVAL
    assert _call_sym(lib, prob, 4, fd, Z=A + 4) == EINVAL
    assert _call_sym(lib, prob, 4, fd, ws=None) == EWORKSPACE
    for prec in (1, 2):  # refining forms are not offered for several vectors
        p2, _k2 = _prob(prec=prec)
        assert _call_sym(lib, p2, 4, fd) == ENOTSUP
    p3, _k3 = _prob(n0=0.0)
    assert _call_sym(lib, p3, 4, fd) == EINVAL
    p0, _k0 = _prob(W=0)
    assert _call_sym(lib, p0, 4, fd, H=None, Y=None, Z=None, ws=None, wsb=0) == 0


def test_problem_struct_layout():
    # the equaliser field sits in what was the struct's tail padding
    assert ctypes.sizeof(api.EqProblem) == 40
    assert api.EqProblem.equalizer.offset == 36


@pytest.mark.parametrize("fd", [False, True])
def test_equalizer_validation(lib, fd):
    call = _call_fd if fd else _call_pd
    for bad in (-1, 4, 99):
        prob, _k = _prob(eqz=bad)
        assert call(lib, prob) == EINVAL
        assert lib.eq_workspace_size(ctypes.byref(prob)) == 0
    # MRC has no refinement step; the unbiased L-MMSE gain is not refined
    for eqz in (2, 3):
        for prec in (1, 2):
            prob, _k = _prob(eqz=eqz, prec=prec)
            assert call(lib, prob) == ENOTSUP
    # multi-vector calls take every equaliser, but MRC no refining form
    prob, _k = _prob(eqz=2, prec=1)
    assert _call_sym(lib, prob, 4, fd) == ENOTSUP
    # the adjoint is (biased) L-MMSE only
    for eqz in (1, 2, 3):
        prob, _k = _prob(eqz=eqz)
        assert lib.eq_backward_workspace_size(ctypes.byref(prob)) == 0
        if fd:
            st = lib.eq_fd_backward(ctypes.byref(prob), A, A, None, A, None, A, A, None, None, A, 1 << 12, None)
        else:
            st = lib.eq_pd_backward(ctypes.byref(prob), A, A, A, None, A, A, None, A, 1 << 12, None)
        assert st == ENOTSUP


@pytest.mark.parametrize("fd", [False, True])
def test_lama_validation(lib, fd):
    # all rejected (or no-ops) before any HIP call
    def call(prob, t, q, H=A, y=A, z=A):
        if fd:
            return lib.eq_fd_lama(ctypes.byref(prob), t, q, H, y, None, z, A, A, None)
        return lib.eq_pd_lama(ctypes.byref(prob), t, q, H, y, z, A, A, None)
    prob, _k = _prob()
    assert call(prob, 0, 16) == EINVAL
    assert call(prob, 65, 16) == EINVAL
    for q in (2, 8, 32, 256):
        assert call(prob, 2, q) == EINVAL
    assert call(prob, 2, 16, y=None) == EINVAL
    assert call(prob, 2, 16, z=A + 4) == EINVAL
    for prec in (1, 2):
        p2, _k2 = _prob(prec=prec)
        assert call(p2, 2, 16) == ENOTSUP
    p3, _k3 = _prob(n0=-1.0)
    assert call(p3, 2, 16) == EINVAL
    p0, _k0 = _prob(W=0)
    assert call(p0, 2, 16, H=None, y=None, z=None) == 0
    if fd:
        assert lib.eq_fd_lama(None, 2, 16, A, A, None, A, A, A, None) == EINVAL
    else:
        assert lib.eq_pd_lama(None, 2, 16, A, A, A, A, A, None) == EINVAL


@pytest.mark.parametrize("fd", [False, True])
def test_lama_symbols_validation(lib, fd):
    def call(prob, nsym, t, q, Y=A):
        if fd:
            return lib.eq_fd_lama_sym(ctypes.byref(prob), nsym, t, q, A, Y, None, A, A, A, None)
        return lib.eq_pd_lama_sym(ctypes.byref(prob), nsym, t, q, A, Y, A, A, A, None)
    prob, _k = _prob()
    assert call(prob, 0, 2, 16) == EINVAL
    assert call(prob, 1025, 2, 16) == ENOTSUP
    assert call(prob, 4, 0, 16) == EINVAL
    assert call(prob, 4, 2, 32) == EINVAL
    assert call(prob, 4, 2, 16, Y=None) == EINVAL
    p2, _k2 = _prob(prec=1)
    assert call(p2, 4, 2, 16) == ENOTSUP
    p0, _k0 = _prob(W=0)
    assert call(p0, 4, 2, 16) == 0


def test_binding_names_match_header_enums():
    """The binding's precision and equaliser names map to the values that
    include/dbpeq.h gives the enumerators."""
    import re
    from paper_1808_04473_amd import api
    text = open(HEADER).read()

    def enum(name):
        body = re.search(r"typedef enum \{([^}]*)\}\s*" + name + ";", text, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        return {k: int(v) for k, v in re.findall(r"(EQ_\w+)\s*=\s*(\d+)", body)}

    eqz = enum("eq_equalizer")
    assert eqz == {"EQ_LMMSE": 0, "EQ_ZF": 1, "EQ_MRC": 2, "EQ_LMMSE_UNBIASED": 3}
    assert {f"EQ_{k.upper()}": v for k, v in api.EQUALIZERS.items()} == eqz
    prec = enum("eq_precision")
    assert {f"EQ_{k.upper()}": v for k, v in api.PRECISIONS.items()} == prec


def test_fd_single_bf16_refinement_refused(lib):
    """FD's fusion weights come from diag((G_c + rho I)^{-1}), which the
    refinement step does not correct: eq_fd and FD plans refuse the
    single-BF16 Gram (EQ_ENOTSUP, before any HIP call); PD accepts it."""
    import ctypes as ct
    prob, _off = api.make_problem(4, 8, 2, [0, 4, 8], 0.1, 1.0, "bf16_refine")
    ws = 1 << 12
    assert lib.eq_fd(ct.byref(prob), A, A, None, A, A, A, A, ws, None) == ENOTSUP
    for eqz in (0, 1):  # L-MMSE and ZF
        prob.equalizer = eqz
        assert lib.eq_fd(ct.byref(prob), A, A, None, A, A, A, A, ws, None) == ENOTSUP
    # PD with the same problem gets past validation to the workspace check
    prob.equalizer = 0
    assert lib.eq_pd(ct.byref(prob), A, A, A, A, A, None, 0, None) == EWORKSPACE
    desc = (api.EqSys * 1)()
    desc[0] = api.EqSys(0, 0, 0, 8, 2, 2, 0, 0.1, 0)
    sizes = np.array([4, 4], np.int32)
    h = ct.c_void_p()
    assert lib.eq_plan_create(ct.byref(h), desc, 1, sizes.ctypes.data_as(ct.POINTER(ct.c_int32)), 2, 1, 1,
                              1.0, None) == ENOTSUP
    assert not h.value


def test_binding_checks_caller_outputs():
    """Caller-supplied out / nu / ws tensors reach the kernels as raw
    pointers, so the binding checks shape, dtype, device and contiguity."""
    import torch
    cpu = torch.device("cpu")
    W, U, C = 5, 3, 2
    z = torch.empty((W, U), dtype=torch.complex64)
    s2 = torch.empty((W, U), dtype=torch.float32)
    info = torch.empty((W,), dtype=torch.int32)
    assert api._outputs((z, s2, info), (W, U), (W, U), (W,), cpu)[0] is z
    assert api._outputs((z, None, None), (W, U), (W, U), (W,), cpu)[1] is None
    with pytest.raises(ValueError):
        api._outputs((z[:4], s2, info), (W, U), (W, U), (W,), cpu)            # too few systems
    with pytest.raises(ValueError):
        api._outputs((z, s2, torch.empty((W, C), dtype=torch.int32)), (W, U), (W, U), (W,), cpu)
    with pytest.raises(TypeError):
        api._outputs((z, s2.double(), info), (W, U), (W, U), (W,), cpu)
    with pytest.raises(ValueError):
        api._outputs((torch.empty((U, W), dtype=torch.complex64).t(), s2, info), (W, U), (W, U), (W,), cpu)
    with pytest.raises(ValueError):
        api._outputs((z, s2), (W, U), (W, U), (W,), cpu)
    meta = torch.device("meta")
    with pytest.raises(ValueError):
        api._outputs((z, s2, info), (W, U), (W, U), (W,), meta)               # wrong device
    with pytest.raises(ValueError):
        api._check_nu(torch.empty((W, C, U + 1)), W, C, U, cpu)
    assert api._check_nu(None, W, C, U, cpu) is None
    with pytest.raises(ValueError):
        api._check_ws(torch.empty(64, dtype=torch.float32), cpu)


def test_noalloc_validates_before_any_hip_call(lib):
    """eq_pd_noalloc checks its arguments like eq_pd, and refuses W above the
    capacity of its device array (EQ_ENOTSUP), before any HIP call."""
    import ctypes as ct
    bad, _k1 = _prob(n0=0.0)
    assert lib.eq_pd_noalloc(ct.byref(bad), A, A, A, A, A, None) == EINVAL
    ok, _k2 = _prob()
    assert lib.eq_pd_noalloc(ct.byref(ok), None, A, A, A, A, None) == EINVAL
    big, _k3 = _prob(W=api.NOALLOC_MAX_W + 1)
    assert lib.eq_pd_noalloc(ct.byref(big), A, A, A, A, A, None) == ENOTSUP
    txt = open(HEADER).read()
    assert f"#define EQ_NOALLOC_MAX_W {api.NOALLOC_MAX_W}" in txt


def test_plan_class_constants_match_header():
    txt = open(HEADER).read()
    assert f"#define EQ_PLAN_CLASSES {api.PLAN_CLASSES}" in txt
    assert len(api.PLAN_CLASS_NAMES) == api.PLAN_CLASSES


def test_kernel_timer_argument_errors():
    """The kernel timer refuses bad capacities and a stop without a start
    before any HIP call (no device needed)."""
    lib = api.load_library()
    n, ms = ctypes.c_int32(), ctypes.c_double()
    assert lib.eq_kernel_timer_start(0) == EINVAL
    assert lib.eq_kernel_timer_start(api.KERNEL_TIMER_MAX + 1) == EINVAL
    assert lib.eq_kernel_timer_stop(ctypes.byref(n), ctypes.byref(ms)) == EINVAL
    txt = open(HEADER).read()
    assert f"#define EQ_KERNEL_TIMER_MAX {api.KERNEL_TIMER_MAX}" in txt
