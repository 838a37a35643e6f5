"""dbpeq: decentralized feedforward L-MMSE equalisation on AMD MI355X.

The equaliser itself lives in libdbpeq.so (hand-written gfx950 HIP kernels
behind the C ABI of include/dbpeq.h).  Import `paper_1808_04473_amd.api`
(or the names re-exported here) for the PyTorch-facing calls, and
`paper_1808_04473_amd.synth` for seeded synthetic workloads.
"""

__all__ = ["eq_pd", "eq_fd", "load_library"]


def __getattr__(name):
    # The binding imports torch; keep `import paper_1808_04473_amd.synth` light.
    if name in ("eq_pd", "eq_fd", "load_library", "EqError"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
