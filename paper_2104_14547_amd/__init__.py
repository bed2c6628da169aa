"""MI355X-native differentiable NURBS surfaces (NURBS-Diff, arXiv 2104.14547).

The hot path -- knot-span search, Cox-de Boor basis, the weighted
homogeneous (p+1)x(q+1) patch sum, the rational divide and the adjoint with
respect to control points, weights and knots -- runs in hand-written HIP
kernels for gfx950 behind the C ABI of ``include/nurbsdiff.h``
(``libnurbsdiff.so``).  This package marshals PyTorch tensors into that ABI.

``workloads`` (seeded synthetic inputs) imports neither torch nor the library.
"""
from ._native import (NURBS_GRAD_ALL, NURBS_GRAD_CTRL, NURBS_GRAD_KU, NURBS_GRAD_KV, NURBS_GRAD_W,
                      NURBS_MAX_DEGREE, NURBS_VALIDATE, NativeLibraryMissing)


def __getattr__(name):
    # the torch-facing API is imported on first use, so that `workloads`
    # and the ABI constants load without torch
    import importlib
    if name.startswith("__"):
        raise AttributeError(name)
    if name in ("api", "fit", "serve", "workloads", "build"):
        return importlib.import_module(__name__ + "." + name)
    api = importlib.import_module(__name__ + ".api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
