"""MI355X-native ADMM reconstruction for Cartesian dynamic parallel MRI.

The compute path is the HIP library ``libcsmri.so`` (C ABI in include/csmri.h);
this package only marshals arguments to it.  The library is loaded lazily on
the first call, and a missing or unloadable library raises immediately: there
is no CPU fallback.
"""
__all__ = ["synthetic"]
