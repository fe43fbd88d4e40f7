"""Python handle over the C ABI (include/lbm.h).

PyTorch supplies device memory and the stream; every step of the method runs in
the gfx950 kernels of liblbm_hip.so.  Names follow the C calls: ``step(n)`` is
``lbm_step``, ``moments()`` is ``lbm_moments`` and so on.
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, load

_STORAGE = {"f64": _lib.STORE_F64, "f32": _lib.STORE_F32, "f16": _lib.STORE_F16,
            "bf16": _lib.STORE_BF16}


def required_bytes(descriptor, nx, ny, nz, storage):
    lib = load()
    pop = ctypes.c_size_t()
    aux = ctypes.c_size_t()
    check(lib.lbm_required_bytes(descriptor, nx, ny, nz, _STORAGE.get(storage, storage),
                                 ctypes.byref(pop), ctypes.byref(aux)))
    return pop.value, aux.value


def validate_geometry(descriptor, material, periodic):
    """Host-only geometry check; returns the C status (0 = accepted)."""
    lib = load()
    mat = np.ascontiguousarray(material, dtype=np.uint8)
    if mat.ndim == 2:
        mat = mat[None]
    nz, ny, nx = mat.shape
    return lib.lbm_validate_geometry(descriptor, nx, ny, nz,
                                     mat.ctypes.data_as(ctypes.c_void_p), int(periodic))


@contextlib.contextmanager
def stream_order(stream, device):
    """Order a library call on a handle's stream between the caller's work.

    The library launches on the stream its handle was created with.  Work the
    caller queued on its current stream before the call (producing an input,
    staging copies, allocating an output) completes before the call's kernels
    start, and the caller's later work waits for them.  Inputs are staged and
    outputs allocated on the caller's stream, so the caching allocator keeps
    their memory ordered on that stream alone.
    """
    caller = torch.cuda.current_stream(device)
    same = caller.cuda_stream == stream.cuda_stream
    if not same:
        stream.wait_stream(caller)
    try:
        yield
    finally:
        if not same:
            caller.wait_stream(stream)


def _vec3(v):
    out = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    if v is not None:
        v = list(np.asarray(v, dtype=np.float64).ravel())
        for a, val in enumerate(v):
            out[a] = val
    return out


class _Handle:
    """Calls shared by owned lattices and batch members (``self.h`` is the C handle)."""

    def _chk(self, st):
        return check(st, self.h)


class Lattice(_Handle):
    """One lattice (one block) on the current GPU.

    shape = (nx, ny, nz); populations live in a caller-owned uint8 tensor
    ``self.pop`` of ``lbm_required_bytes`` bytes (placement: see include/lbm.h).
    """

    def __init__(self, descriptor, shape, tau, storage="f32", shifted=False, stream=None,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the LBM kernels need a ROCm GPU")
        self.lib = load()
        self.descriptor = descriptor
        self.q = 9 if descriptor == _lib.D2Q9 else 19
        nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.storage = storage
        self.shifted = bool(shifted)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            pop_b, aux_b = required_bytes(descriptor, self.nx, self.ny, self.nz, storage)
            self.pop = torch.empty(pop_b, dtype=torch.uint8, device=self.device)
            self.aux = torch.empty(aux_b, dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            st = self.lib.lbm_lattice_create(
                ctypes.byref(h), descriptor, self.nx, self.ny, self.nz, float(tau),
                _STORAGE.get(storage, storage), _lib.FLAG_SHIFTED if shifted else 0,
                ctypes.c_void_p(self.pop.data_ptr()), pop_b, ctypes.c_void_p(self.aux.data_ptr()),
                aux_b, ctypes.c_void_p(self.stream.cuda_stream))
            check(st, None)
        self.h = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up -------------------------------------------------------------
    def set_geometry(self, material, periodic):
        mat = np.ascontiguousarray(material, dtype=np.uint8)
        if mat.size != self.N:
            raise ValueError(f"material needs {self.N} cells, got {mat.size}")
        self._chk(self.lib.lbm_set_geometry(self.h, mat.ctypes.data_as(ctypes.c_void_p),
                                            int(periodic)))

    def set_wall_velocity(self, u_w):
        self._chk(self.lib.lbm_set_wall_velocity(self.h, _vec3(u_w)))

    def set_body_force(self, g):
        self._chk(self.lib.lbm_set_body_force(self.h, _vec3(g)))

    def set_tau(self, tau):
        self._chk(self.lib.lbm_set_tau(self.h, float(tau)))

    def _dev64(self, a, n):
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64)
        t = t.to(self.device).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    # Inputs are staged and outputs allocated on the caller's stream; each call
    # is ordered after that work and before the caller's next (stream_order).
    def init_equilibrium(self, rho=None, u=None):
        """rho: N values or None (1); u: (dim or 3, N...) values or None (0).
        Device float64 tensors of the full shape ((N...) and (3, N...)) are
        used in place; anything else is staged on the device first."""
        r = self._dev64(rho, self.N)
        uu = None
        if u is not None:
            ut = torch.as_tensor(u, dtype=torch.float64)
            if ut.device == self.device and ut.numel() == 3 * self.N:
                uu = ut.reshape(3, self.N).contiguous()
            else:
                ut = ut.reshape(-1, self.N)
                full = torch.zeros((3, self.N), dtype=torch.float64, device=self.device)
                full[: ut.shape[0]] = ut.to(self.device)
                uu = full
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_init_equilibrium(
                self.h, None if r is None else ctypes.c_void_p(r.data_ptr()),
                None if uu is None else ctypes.c_void_p(uu.data_ptr())))
        self.stream.synchronize()

    def set_populations(self, f):
        t = self._dev64(f, self.q * self.N)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_set_populations(self.h, ctypes.c_void_p(t.data_ptr())))
        self.stream.synchronize()

    # -- hot path -----------------------------------------------------------
    def step(self, n=1):
        self._chk(self.lib.lbm_step(self.h, int(n)))

    def set_graph_steps(self, steps):
        """Replay lbm_step in captured HIP graphs of `steps` steps (0 = off)."""
        self._chk(self.lib.lbm_set_graph_steps(self.h, int(steps)))

    # -- read-back ----------------------------------------------------------
    def get_populations(self):
        """Populations in natural layout, float64 tensor (q, nz, ny, nx) on the GPU."""
        out = torch.empty((self.q, self.nz, self.ny, self.nx), dtype=torch.float64,
                          device=self.device)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_get_populations(self.h, ctypes.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def moments(self):
        """(rho (nz,ny,nx), u (3,nz,ny,nx)) as float64 numpy arrays on the host
        (lbm_moments: decoded in double, sync)."""
        rho = np.empty((self.nz, self.ny, self.nx), dtype=np.float64)
        u = np.empty((3, self.nz, self.ny, self.nx), dtype=np.float64)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_moments(self.h, rho.ctypes.data_as(ctypes.c_void_p),
                                           u.ctypes.data_as(ctypes.c_void_p)))
        return rho, u

    def moments_device(self):
        """(rho (nz,ny,nx), u (3,nz,ny,nx)) as float32 tensors on the GPU
        (lbm_moments_device, ordered on the caller's stream)."""
        rho = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device=self.device)
        u = torch.empty((3, self.nz, self.ny, self.nx), dtype=torch.float32, device=self.device)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_moments_device(self.h, ctypes.c_void_p(rho.data_ptr()),
                                                  ctypes.c_void_p(u.data_ptr())))
        return rho, u

    def totals(self):
        """(mass, momentum[3], stats[avRho, avEnergy, maxU]) reduced on the GPU in FP64."""
        m = ctypes.c_double()
        j = (ctypes.c_double * 3)()
        s = (ctypes.c_double * 3)()
        self._chk(self.lib.lbm_totals(self.h, ctypes.byref(m), j, s))
        return m.value, np.array(list(j)), np.array(list(s))

    def info(self):
        steps = ctypes.c_longlong()
        nf = ctypes.c_longlong()
        self._chk(self.lib.lbm_get_info(self.h, ctypes.byref(steps), ctypes.byref(nf)))
        return steps.value, nf.value
