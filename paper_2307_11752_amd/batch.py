"""Batched ensembles of periodic lattices (C ABI ``lbm_batch_*``).

Each time step advances every member through the batch's own launches (one
per propagation phase, and per row width class in the second); runs of steps
are replayed from a captured HIP graph; ``autotune()`` picks each phase's launch
shape by measurement (``set_phase_launch`` / ``phase_launch`` set and read one
phase's).  Members are lattice handles: read them with the ``Lattice``
calls (``init_equilibrium``, ``moments``, ``totals``, ``get_populations``).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check_batch, load
from .lattice import _STORAGE, Lattice


class BatchMember(Lattice):
    """A lattice owned by a Batch (no buffers of its own)."""

    def __init__(self, batch, index, handle, shape, tau):
        # deliberately not calling Lattice.__init__: the batch owns the memory
        self.lib = batch.lib
        self.descriptor = batch.descriptor
        self.q = batch.q
        self.nx, self.ny, self.nz = shape
        self.N = self.nx * self.ny * self.nz
        self.storage = batch.storage
        self.shifted = batch.shifted
        self.device = batch.device
        self.stream = batch.stream
        self.tau = tau
        self.index = index
        self.h = handle
        self._batch = batch

    def close(self):
        self.h = None  # released with the batch


class Batch:
    def __init__(self, descriptor, shapes, taus, storage="f32", shifted=False, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the LBM kernels need a ROCm GPU")
        self.lib = load()
        self.descriptor = descriptor
        self.q = 9 if descriptor == _lib.D2Q9 else 19
        self.storage = storage
        self.shifted = bool(shifted)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.taus = [float(t) for t in taus]
        if len(self.shapes) != len(self.taus):
            raise ValueError("one tau per lattice")
        self.count = len(self.shapes)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.Stream()
        dims = (ctypes.c_int * (3 * self.count))(*[v for s in self.shapes for v in s])
        tau = (ctypes.c_double * self.count)(*self.taus)
        st = _STORAGE.get(storage, storage)
        pop_b, aux_b = ctypes.c_size_t(), ctypes.c_size_t()
        check_batch(self.lib.lbm_batch_required_bytes(descriptor, self.count, dims, st,
                                                      ctypes.byref(pop_b), ctypes.byref(aux_b)),
                    None)
        self.pop = torch.empty(pop_b.value, dtype=torch.uint8, device=self.device)
        self.aux = torch.empty(aux_b.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check_batch(self.lib.lbm_batch_create(
            ctypes.byref(h), descriptor, self.count, dims, tau, st,
            _lib.FLAG_SHIFTED if shifted else 0, ctypes.c_void_p(self.pop.data_ptr()),
            pop_b.value, ctypes.c_void_p(self.aux.data_ptr()), aux_b.value,
            ctypes.c_void_p(self.stream.cuda_stream)), None)
        self.h = h
        self.members = []
        for i, (shape, t) in enumerate(zip(self.shapes, self.taus)):
            v = ctypes.c_void_p()
            self._chk(self.lib.lbm_batch_lattice(self.h, i, ctypes.byref(v)))
            self.members.append(BatchMember(self, i, v, shape, t))

    def _chk(self, st):
        return check_batch(st, self.h)

    def __len__(self):
        return self.count

    def __getitem__(self, i):
        return self.members[i]

    def step(self, n=1):
        self._chk(self.lib.lbm_batch_step(self.h, int(n)))

    def set_graph_steps(self, steps):
        self._chk(self.lib.lbm_batch_set_graph_steps(self.h, int(steps)))

    def set_launch(self, threads, blocks_per_cu):
        """Launch shape of both propagation phases (lbm_batch_set_launch)."""
        self._chk(self.lib.lbm_batch_set_launch(self.h, int(threads), int(blocks_per_cu)))

    def set_phase_launch(self, phase, threads, blocks_per_cu):
        """Launch shape of one phase (0 or 1) only (lbm_batch_set_phase_launch)."""
        self._chk(self.lib.lbm_batch_set_phase_launch(self.h, int(phase), int(threads),
                                                      int(blocks_per_cu)))

    def phase_launch(self, phase):
        """(threads, blocks_per_cu) of one phase (lbm_batch_get_phase_launch)."""
        t, b = ctypes.c_int(), ctypes.c_int()
        self._chk(self.lib.lbm_batch_get_phase_launch(self.h, int(phase), ctypes.byref(t),
                                                      ctypes.byref(b)))
        return t.value, b.value

    def autotune(self, trial_steps=20):
        """Measure the built-in launch shapes and keep the fastest of each phase
        (read them with phase_launch).  Returns phase 1's threads and blocks per
        CU and the tuned ms per step.  Advances every member (initialise the
        populations again afterwards)."""
        t, b, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._chk(self.lib.lbm_batch_autotune(self.h, int(trial_steps), ctypes.byref(t),
                                              ctypes.byref(b), ctypes.byref(ms)))
        return t.value, b.value, ms.value

    def info(self):
        c, t, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        cells = ctypes.c_longlong()
        self._chk(self.lib.lbm_batch_get_info(self.h, ctypes.byref(c), ctypes.byref(cells),
                                              ctypes.byref(t), ctypes.byref(b)))
        return {"count": c.value, "cells": cells.value, "threads": t.value,
                "blocks_per_cu": b.value}

    def close(self):
        if getattr(self, "h", None):
            for m in self.members:
                m.h = None
            self.lib.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
