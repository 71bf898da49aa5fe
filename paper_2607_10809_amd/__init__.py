"""MI355X (gfx950) explicit step of the compact ADER-HWENO scheme on triangles.

The step itself is hand-written HIP in ``libhwe.so`` (C ABI in ``include/hwe.h``);
this package only loads it and marshals torch tensors into it.
"""
from ._lib import HweError, load_library  # noqa: F401


def __getattr__(name):
    # torch-dependent parts are imported on first use
    if name in ("Mesh", "hwe_mesh_init", "hwe_step", "hwe_step_adjoint", "make_opts"):
        from . import hwe
        return getattr(hwe, name)
    if name in ("rollout", "Rollout"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
