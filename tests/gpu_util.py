"""Helpers for the GPU parity tests: device placement, error metrics."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1808_04473_amd import api
    api.load_library()  # raises if the HIP library is missing: no fallback


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def max_rel_err(z, z_ref):
    """max over systems of ||z_w - z_ref_w||_inf / ||z_ref_w||_inf."""
    num = np.max(np.abs(z - z_ref), axis=-1)
    den = np.max(np.abs(z_ref), axis=-1)
    return float(np.max(num / den))


def max_db_err(s2, s2_ref):
    """max |10 log10(sigma2 / sigma2_ref)| (post-equalisation SINR in dB)."""
    return float(np.max(np.abs(10.0 * np.log10(s2 / s2_ref))))


def sinr_db_empirical(z, s):
    es = np.mean(np.abs(s) ** 2)
    return 10 * math.log10(es / np.mean(np.abs(z - s) ** 2))


# gates (error on the equalised symbols; SINR)
TOL_Z = {"fp32": 1e-4, "bf16_refine": 2e-4, "bf16x3_refine": 2e-4, "bf16x3": 1e-4}
TOL_DB = 0.05


def refused(mode, prec):
    """Forms the library refuses with EQ_ENOTSUP: FD with the single-BF16
    Gram (its fusion weights come from diag((G_c + rho I)^{-1}), which the
    refinement step does not correct)."""
    return mode == "fd" and prec == "bf16_refine"


def expect_refused(fn):
    """Calls fn() and checks that the library refuses it with EQ_ENOTSUP."""
    from paper_1808_04473_amd import api
    with pytest.raises(api.EqError) as e:
        fn()
    assert e.value.status == -2, e.value.status
