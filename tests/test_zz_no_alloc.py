"""lbm_totals_noalloc, the totals call for callers that cannot allocate (its
reduction scratch is a library-owned static device array), against lbm_totals
(the lattice's own aux scratch): both run the same reduction kernels with the
same block count, so the FP64 results must be bitwise equal.  Two lattices in a
row, the second smaller, so the shared array's leftovers from the first call
cannot leak into the second."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    import paper_2307_11752_amd as P
    from paper_2307_11752_amd import _lib

    _lib.load()
    return P


def _totals(lib, fn, h):
    m = ctypes.c_double()
    j = (ctypes.c_double * 3)()
    s = (ctypes.c_double * 3)()
    st = fn(h, ctypes.byref(m), j, s)
    assert st == 0, lib.lbm_last_error(h).decode()
    return [m.value] + list(j) + list(s)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_noalloc_totals_equal_lbm_totals(lbm, storage):
    from paper_2307_11752_amd import _lib
    from paper_2307_11752_amd import workloads as W

    lib = _lib.load()
    cases = [(1, (72, 40, 36), W.PERIODIC_X | W.PERIODIC_Z, 11),
             (0, (30, 18, 1), W.PERIODIC_X, 12)]
    for d, shape, periodic, seed in cases:
        print(f"[noalloc] d={d} shape={shape} storage={storage}", flush=True)
        lat = lbm.Lattice(d, shape, 0.7, storage=storage, shifted=True)
        mat = W.random_geometry(d, shape, periodic, seed)
        lat.set_geometry(mat, periodic)
        lat.set_body_force((1e-4, -2e-5, 0.0))
        lat.set_wall_velocity((0.02, 0.0, 0.0))
        lat.init_equilibrium(W.random_density(shape, seed + 1),
                             W.random_velocity(shape, seed + 2, dim=3 if d else 2))
        for n in (0, 5):
            lat.step(n)
            a = _totals(lib, lib.lbm_totals, lat.h)
            b = _totals(lib, lib.lbm_totals_noalloc, lat.h)
            assert a == b, (a, b)
            assert a[0] > 0 and np.all(np.isfinite(a))
        lat.close()
