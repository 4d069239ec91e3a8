"""MI355X-native hot path of the mu-diff spectral multiple-scattering method
(arXiv:1409.8186): FP64 HIP kernels for gfx950 behind the C ABI of
include/mudiff.h, with a thin Python binding.

    from paper_1409_8186_amd import Problem
    P = Problem.from_cluster(cluster)             # tables on the device
    rho, flag, relres, iters, _ = P.gmres(betas=[[0.0]], tol=1e-8)
    a = P.farfield(rho, thetas)
    u = P.nearfield(rho, points, betas=[[0.0]])   # total field at points

Other formulations (P.set_operator("cfie"), ...), penetrable disks
(P.set_penetrable(k_int, mu), P.interior_field), point sources (sources=
instead of betas) and the misfit gradient (P.grad, FarFieldMisfit) use the
same handle; the time-reversal operator is built from P.mirror_farfield with
the module functions tro, tro_eigh and herglotz.

Importing the package does not load the library; ``Problem`` loads it and
raises if it was not built (``python -m paper_1409_8186_amd.build``).
"""
from ._lib import GRAPH, NO_PRECOND, OP_A, OP_L, OP_LT, POINT_SOURCE, X0, MudiffError  # noqa: F401


def __getattr__(name):
    if name in ("Problem",):
        from .api import Problem
        return Problem
    if name in ("probe", "tro", "tro_eigh", "herglotz"):
        from . import api
        return getattr(api, name)
    if name == "FarFieldMisfit":
        from .autograd import FarFieldMisfit
        return FarFieldMisfit
    raise AttributeError(name)
