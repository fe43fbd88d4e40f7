"""Porosity gradients through the hand-written discrete adjoint (C ABI
``lbm_porous_*``), exposed as a ``torch.autograd.Function``.

    prob = PorousChannel(material, periodic, tau=0.7, g=(1e-5, 0, 0), steps=500,
                         checkpoint_every=50)
    d = torch.rand(prob.shape_zyx, device="cuda", requires_grad=True)
    J = porous_objective(d, prob)      # mean outlet x-velocity after `steps`
    J.backward()                       # d.grad = dJ/dd via the adjoint sweep
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check_porous, load
from .lattice import stream_order


def _vec3(v):
    out = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    for a, val in enumerate(np.asarray(v, dtype=np.float64).ravel()[:3]):
        out[a] = val
    return out


class PorousChannel:
    def __init__(self, material, periodic, tau, g, steps, checkpoint_every, plane_x=None,
                 stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the LBM kernels need a ROCm GPU")
        self.lib = load()
        mat = np.ascontiguousarray(material, dtype=np.uint8)
        self.shape_zyx = mat.shape
        self.nz, self.ny, self.nx = mat.shape
        self.N = mat.size
        self.steps = int(steps)
        self.checkpoint_every = int(checkpoint_every)
        self.plane_x = self.nx - 1 if plane_x is None else int(plane_x)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nb = ctypes.c_size_t()
        check_porous(self.lib.lbm_porous_required_bytes(self.nx, self.ny, self.nz, self.steps,
                                                        self.checkpoint_every, ctypes.byref(nb)),
                     None)
        self.work = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check_porous(self.lib.lbm_porous_create(
            ctypes.byref(h), self.nx, self.ny, self.nz, float(tau),
            mat.ctypes.data_as(ctypes.c_void_p), int(periodic), _vec3(g), self.steps,
            self.checkpoint_every, self.plane_x, ctypes.c_void_p(self.work.data_ptr()), nb.value,
            ctypes.c_void_p(self.stream.cuda_stream)), None)
        self.h = h

    def _chk(self, st):
        return check_porous(st, self.h)

    def forward(self, porosity):
        """J for a float32 device tensor of shape (nz, ny, nx)."""
        d = porosity.detach().to(device=self.device, dtype=torch.float32).contiguous()
        J = ctypes.c_double()
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_porous_forward(self.h, ctypes.c_void_p(d.data_ptr()),
                                                  ctypes.byref(J)))
        return J.value

    def generation(self):
        """Number of forward runs completed (lbm_porous_generation)."""
        g = ctypes.c_longlong()
        self._chk(self.lib.lbm_porous_generation(self.h, ctypes.byref(g)))
        return g.value

    def backward(self):
        """dJ/dd of the last forward run, float32 tensor (nz, ny, nx)."""
        grad = torch.empty(self.shape_zyx, dtype=torch.float32, device=self.device)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_porous_backward(self.h, ctypes.c_void_p(grad.data_ptr())))
        return grad

    def final_populations(self):
        f = torch.empty((19,) + tuple(self.shape_zyx), dtype=torch.float64, device=self.device)
        with stream_order(self.stream, self.device):
            self._chk(self.lib.lbm_porous_get_final(self.h, ctypes.c_void_p(f.data_ptr())))
        return f

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_porous_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PorousObjective(torch.autograd.Function):
    """J(d) with dJ/dd from the adjoint sweep (checkpointed recomputation).

    The handle keeps the checkpoints of its latest forward run only.  Each
    node records the porosity it was evaluated at and the handle's forward
    count; if another forward ran on the same handle in between (a line
    search, a finite-difference probe), backward first repeats this node's
    forward run, so the gradient always belongs to this node's porosity."""

    @staticmethod
    def forward(ctx, porosity, problem):
        ctx.problem = problem
        d = porosity.detach().to(dtype=torch.float32).contiguous().clone()
        J = problem.forward(d)
        ctx.porosity = d
        ctx.generation = problem.generation()
        return torch.tensor(J, dtype=torch.float64, device=porosity.device)

    @staticmethod
    def backward(ctx, grad_out):
        problem = ctx.problem
        if problem.generation() != ctx.generation:
            problem.forward(ctx.porosity)
        grad = problem.backward()
        return grad * grad_out.to(grad.dtype), None


def porous_objective(porosity, problem):
    return PorousObjective.apply(porosity, problem)
