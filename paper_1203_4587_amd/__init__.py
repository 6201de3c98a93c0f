"""MI355X-native ADMM reconstruction for Cartesian dynamic parallel MRI.

The compute path is the HIP library ``libcsmri.so`` (C ABI in include/csmri.h);
``paper_1203_4587_amd.api`` only marshals arguments to it.  The library is
loaded on first use and a missing library raises: there is no CPU fallback.
The seeded input generators live in ``paper_1203_4587_amd.synthetic``.
"""
__all__ = ["api", "synthetic", "build"]


def __getattr__(name):
    if name == "api":
        from . import api
        return api
    raise AttributeError(name)
