"""MI355X-native matrix-free H.v in a symmetry-adapted basis (spin-1/2 ED).

The compute lives in the HIP library ``libsymed.so`` (C ABI declared in
``include/symed.h``); ``symed`` is its Python binding.
"""
from . import symed  # noqa: F401
from .symed import Basis, EdError, eigenvalues, tables_inspect, version  # noqa: F401
