"""MI355X (gfx950) Shield-MPPI sampled-rollout step (arXiv 2302.11719).

The compute path is libsmppi.so (hand-written HIP kernels behind the C ABI of
include/smppi.h); this package binds it (``core``), adds the autograd face of
the adjoint kernel (``autograd``), the plan autotuner (``autotune``), rocprofv3
summaries (``profile_summary``) and the seeded workload generator
(``workloads``)."""
from . import workloads  # noqa: F401

__all__ = ["workloads", "core", "autograd"]


def __getattr__(name):
    # torch-dependent modules load lazily so that the generator imports cheaply
    if name in ("core", "autograd", "autotune"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
