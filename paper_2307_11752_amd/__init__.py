"""MI355X-native fused BGK collide-and-stream (D2Q9 / D3Q19) with bounce-back,
moving walls, periodic wrap and Guo forcing.

The arithmetic runs in the hand-written gfx950 kernels of ``liblbm_hip.so``
(C ABI in include/lbm.h); this package only binds it.  Method: OpenLB User
Guide, release 1.6 (arXiv:2307.11752).
"""
from ._lib import (D2Q9, D3Q19, STORE_BF16, STORE_F16, STORE_F32, STORE_F64, LBMError)  # noqa: F401

__all__ = ["Lattice", "Batch", "D2Q9", "D3Q19", "STORE_F64", "STORE_F32", "STORE_F16", "STORE_BF16",
           "LBMError"]


def __getattr__(name):
    if name == "Lattice":
        from .lattice import Lattice

        return Lattice
    if name == "Batch":
        from .batch import Batch

        return Batch
    raise AttributeError(name)
