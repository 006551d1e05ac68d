"""mgx: batched underwater-vehicle dynamics (MarineGym's Fossen step) on MI355X.

The compute path is the HIP library ``libmgx.so`` behind the C ABI of include/mgx.h;
``mgx`` is its ctypes binding.
"""
from . import mgx  # noqa: F401
from .mgx import Batch, MgxError  # noqa: F401
