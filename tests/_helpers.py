"""Shared test helpers: storage rounding emulation, state construction and
error metrics.  Inputs are built in numpy (or by the oracle); nothing here reads
a value produced by the GPU path to build an input or an expected value."""
from __future__ import annotations

import numpy as np

STORAGES = ("f64", "f32", "f16", "bf16")
EPS_COMPUTE = {"f64": 2.0**-53, "f32": 2.0**-24, "f16": 2.0**-24, "bf16": 2.0**-24}
# the library's FP16 storage holds the value times 2^12 (include/lbm.h)
F16_SCALE = 4096.0


def _bf16_round(a):
    """float64 -> float32 -> bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round_storage(a, storage):
    """Round float64 values to the storage type and back to float64."""
    a = np.asarray(a, dtype=np.float64)
    if storage == "f64":
        return a.copy()
    if storage == "f32":
        return a.astype(np.float32).astype(np.float64)
    if storage == "f16":
        return (a * F16_SCALE).astype(np.float16).astype(np.float64) / F16_SCALE
    if storage == "bf16":
        return _bf16_round(a)
    raise ValueError(storage)


def ulp_storage(a, storage):
    """Spacing of the storage type at |a| (normal range; subnormal spacing below)."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    scale = F16_SCALE if storage == "f16" else 1.0
    bits = {"f64": 52, "f32": 23, "f16": 10, "bf16": 7}[storage]
    tiny = {"f64": 2.0**-1022, "f32": 2.0**-126, "f16": 2.0**-14, "bf16": 2.0**-126}[storage]
    e = np.floor(np.log2(np.maximum(a * scale, tiny)))
    return 2.0 ** (e - bits) / scale


def encode_decode(f, w, storage, shifted):
    """What set_populations followed by get_populations returns for f."""
    wq = w.reshape((-1,) + (1,) * (f.ndim - 1))
    if shifted:
        return round_storage(f - wq, storage) + wq
    return round_storage(f, storage)


def representable(f, w, storage, shifted, iters=4):
    """A state close to f that survives the encode/decode round trip exactly."""
    fr = encode_decode(f, w, storage, shifted)
    for _ in range(iters):
        again = encode_decode(fr, w, storage, shifted)
        if np.array_equal(again, fr):
            return fr
        fr = again
    raise AssertionError("could not build a representable state")


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
