"""FP64 CPU oracle of the fused BGK collide-and-stream step (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library (``paper_2307_11752_amd``) never
imports it and shares no code with it; the C source ``lbm_oracle.c`` carries its
own descriptor tables.

The arithmetic lives in ``lbm_oracle.c`` (plain C, IEEE double, compiled with
``-ffp-contract=off``); this module only builds it with gcc and marshals numpy
arrays through ctypes.  Citations of the OpenLB 1.6 User Guide (arXiv
2307.11752) are in the C source next to each routine.

Parity pins (tests/test_oracle_pins.py) tie every routine here to something
other than itself: the guide's printed D2Q9 listing, exact moment identities,
brute-force path tracking of pure streaming, closed-form Poiseuille and Couette
profiles, Taylor-Green decay and exact conservation laws.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

D2Q9 = 0
D3Q19 = 1

OK = 0
ERR_ARG = -1
ERR_GEOMETRY = -2
ERR_UNSUPPORTED = -3

_lib = None


def build(force: bool = True) -> str:
    """Compile lbm_oracle.c into liblbm_oracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    U = ctypes.c_uint
    sigs = {
        "orc_descriptor": [I, P, P, P, P, P, P],
        "orc_equilibrium": [I, D, P, P],
        "orc_guo_source": [I, D, D, P, P, P],
        "orc_cell_moments": [I, P, P, P, P],
        "orc_collide": [I, D, P, P, P, P],
        "orc_check_geometry": [I, I, I, I, P, U],
        "orc_init_equilibrium": [I, I, I, I, P, P, P, P],
        "orc_step": [I, I, I, I, P, U, D, P, P, P, P, I],
        "orc_run": [I, I, I, I, P, U, D, P, P, I, P, P, I],
        "orc_moments": [I, I, I, I, P, P, P, P, P],
        "orc_totals": [I, I, I, I, P, P, P, P, P, P],
        "orc_num_threads": [],
        "orc_porous_collide": [I, D, P, D, P, P, P],
        "orc_porous_step": [I, I, I, I, P, U, D, P, P, P, P, I],
        "orc_porous_objective": [I, I, I, I, P, P, P, I],
        "orc_porous_gradient": [I, I, I, I, P, U, D, P, P, I, P, I, P, P, I],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name in ("orc_equilibrium", "orc_guo_source",
                                      "orc_cell_moments", "orc_collide",
                                      "orc_porous_collide") else I
    lib.orc_porous_objective.restype = D
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _vec3(v):
    out = np.zeros(3, dtype=np.float64)
    if v is not None:
        v = np.asarray(v, dtype=np.float64).ravel()
        out[: v.size] = v
    return out


def descriptor(d: int):
    """Return (c[q,3] int, w[q] float64, opp[q] int, cs2) of descriptor d."""
    lib = _load()
    q = ctypes.c_int()
    dim = ctypes.c_int()
    lib.orc_descriptor(d, ctypes.byref(q), ctypes.byref(dim), None, None, None, None)
    c = np.zeros((q.value, 3), dtype=np.int32)
    w = np.zeros(q.value, dtype=np.float64)
    opp = np.zeros(q.value, dtype=np.int32)
    cs2 = ctypes.c_double()
    st = lib.orc_descriptor(d, None, None, _p(c), _p(w), _p(opp), ctypes.byref(cs2))
    if st:
        raise ValueError("unknown descriptor")
    return c, w, opp, cs2.value


def q_of(d: int) -> int:
    return 9 if d == D2Q9 else 19


def equilibrium(d, rho, u):
    lib = _load()
    out = np.zeros(q_of(d))
    lib.orc_equilibrium(d, float(rho), _p(_vec3(u)), _p(out))
    return out


def guo_source(d, omega, rho, u, g):
    lib = _load()
    out = np.zeros(q_of(d))
    lib.orc_guo_source(d, float(omega), float(rho), _p(_vec3(u)), _p(_vec3(g)), _p(out))
    return out


def cell_moments(d, f, g=None):
    lib = _load()
    f = _f64(f, q_of(d))
    rho = np.zeros(1)
    u = np.zeros(3)
    lib.orc_cell_moments(d, _p(f), _p(_vec3(g)), _p(rho), _p(u))
    return rho[0], u


def collide(d, omega, f, g=None):
    """Post-collision populations of one cell (BGK + Guo); returns (f*, rho, u)."""
    lib = _load()
    f = _f64(f, q_of(d)).copy()
    rho = np.zeros(1)
    u = np.zeros(3)
    lib.orc_collide(d, float(omega), _p(_vec3(g)), _p(f), _p(rho), _p(u))
    return f, rho[0], u


class Lattice:
    """Host FP64 lattice driven by the oracle's two-lattice push step.

    ``mat`` is a uint8 array of shape (nz, ny, nx) (x fastest in memory);
    populations are ``f`` with shape (q, nz, ny, nx).
    """

    def __init__(self, d, mat, periodic, tau, g=None, u_wall=None, nthreads=0):
        self.d = d
        self.q = q_of(d)
        mat = np.ascontiguousarray(mat, dtype=np.uint8)
        if mat.ndim == 2:
            mat = mat[None]
        self.nz, self.ny, self.nx = mat.shape
        self.N = mat.size
        self.mat = mat
        self.periodic = int(periodic)
        self.omega = 0.0 if tau == float("inf") else 1.0 / float(tau)
        self.g = _vec3(g)
        self.uw = _vec3(u_wall)
        self.nthreads = int(nthreads)
        st = _load().orc_check_geometry(d, self.nx, self.ny, self.nz, _p(self.mat),
                                        self.periodic)
        if st:
            raise ValueError(f"geometry rejected by oracle (status {st})")
        self.f = np.zeros((self.q, self.nz, self.ny, self.nx))
        self._work = np.zeros_like(self.f)

    def init_equilibrium(self, rho=None, u=None):
        rho_a = None if rho is None else _f64(rho, self.N)
        u_a = None
        if u is not None:
            u = np.asarray(u, dtype=np.float64)
            full = np.zeros((3, self.N))
            full[: u.shape[0]] = u.reshape(u.shape[0], self.N)
            u_a = full
        st = _load().orc_init_equilibrium(self.d, self.nx, self.ny, self.nz, _p(self.mat),
                                          _p(rho_a), _p(u_a), _p(self.f))
        if st:
            raise ValueError(st)

    def set_populations(self, f):
        self.f[...] = np.asarray(f, dtype=np.float64).reshape(self.f.shape)

    def step(self, n=1):
        st = _load().orc_run(self.d, self.nx, self.ny, self.nz, _p(self.mat), self.periodic,
                             self.omega, _p(self.g), _p(self.uw), int(n), _p(self.f),
                             _p(self._work), self.nthreads)
        if st:
            raise RuntimeError(f"oracle step failed ({st})")

    def moments(self):
        """(rho[nz,ny,nx], u[3,nz,ny,nx]) with the Guo-shifted velocity."""
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        _load().orc_moments(self.d, self.nx, self.ny, self.nz, _p(self.mat), _p(self.g),
                            _p(self.f), _p(rho), _p(u))
        shp = (self.nz, self.ny, self.nx)
        return rho.reshape(shp), u.reshape((3,) + shp)

    def totals(self):
        """(mass, momentum[3], stats[avRho, avEnergy, maxU])."""
        m = np.zeros(1)
        j = np.zeros(3)
        s = np.zeros(3)
        _load().orc_totals(self.d, self.nx, self.ny, self.nz, _p(self.mat), _p(self.g),
                           _p(self.f), _p(m), _p(j), _p(s))
        return m[0], j, s


def check_geometry(d, mat, periodic) -> int:
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    if mat.ndim == 2:
        mat = mat[None]
    nz, ny, nx = mat.shape
    return _load().orc_check_geometry(d, nx, ny, nz, _p(mat), int(periodic))


def num_threads() -> int:
    return _load().orc_num_threads()


# ---------------------------------------------------------------------------
# Porous BGK (Simulation Models, "Porous Media Model") and its discrete adjoint
# ---------------------------------------------------------------------------
def porous_collide(d, omega, f, por, g=None):
    lib = _load()
    f = _f64(f, q_of(d)).copy()
    rho = np.zeros(1)
    u = np.zeros(3)
    lib.orc_porous_collide(d, float(omega), _p(_vec3(g)), float(por), _p(f), _p(rho), _p(u))
    return f, rho[0], u


class PorousProblem:
    """Channel with a per-cell porosity field d (shape (nz, ny, nx)); forward
    runs of the porous step, the outlet-plane objective and its FP64 adjoint
    gradient with respect to d."""

    def __init__(self, d, mat, periodic, tau, g, plane_x=None, nthreads=0):
        self.d = d
        self.q = q_of(d)
        mat = np.ascontiguousarray(mat, dtype=np.uint8)
        if mat.ndim == 2:
            mat = mat[None]
        self.mat = mat
        self.nz, self.ny, self.nx = mat.shape
        self.N = mat.size
        self.periodic = int(periodic)
        self.omega = 1.0 / float(tau)
        self.g = _vec3(g)
        self.plane_x = self.nx - 1 if plane_x is None else int(plane_x)
        self.nthreads = int(nthreads)

    def initial_state(self):
        lat = Lattice(self.d, self.mat, self.periodic, 1.0 / self.omega, g=self.g)
        lat.init_equilibrium()
        return lat.f.copy()

    def forward(self, por, nsteps, f0=None):
        """(J, f^T) after nsteps porous steps from f0 (default: rest, rho = 1)."""
        lib = _load()
        por = _f64(por, self.N)
        a = self.initial_state() if f0 is None else np.array(f0, dtype=np.float64)
        b = np.empty_like(a)
        for _ in range(nsteps):
            st = lib.orc_porous_step(self.d, self.nx, self.ny, self.nz, _p(self.mat),
                                     self.periodic, self.omega, _p(self.g), _p(por), _p(a),
                                     _p(b), self.nthreads)
            if st:
                raise RuntimeError(f"porous step failed ({st})")
            a, b = b, a
        J = lib.orc_porous_objective(self.d, self.nx, self.ny, self.nz, _p(self.mat),
                                     _p(self.g), _p(a), self.plane_x)
        return J, a

    def gradient(self, por, nsteps, f0=None):
        """(J, dJ/dd) by the discrete adjoint, all in FP64."""
        lib = _load()
        por = _f64(por, self.N)
        f0 = self.initial_state() if f0 is None else _f64(f0)
        J = np.zeros(1)
        grad = np.zeros(self.N)
        st = lib.orc_porous_gradient(self.d, self.nx, self.ny, self.nz, _p(self.mat),
                                     self.periodic, self.omega, _p(self.g), _p(por), int(nsteps),
                                     _p(f0), self.plane_x, _p(J), _p(grad), self.nthreads)
        if st:
            raise RuntimeError(f"oracle adjoint failed ({st})")
        return J[0], grad.reshape(self.mat.shape)
