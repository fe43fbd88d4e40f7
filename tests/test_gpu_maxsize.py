"""Lattices at the size limits of the 32-bit population offsets.

Pure streaming (omega = 0, g = 0) on fully periodic D3Q19 boxes must move
every population by n c_i: the GPU state after n steps is compared exactly
with the initial state rolled by n c_i (computed on the GPU with torch.roll;
the permutation needs no oracle).  The initial populations are w_i + m 2^-16
with small integers m, exact in every storage type.

* 608 x 608 x 600 cells (q N = 4.21e9 elements, just under 2^32): one array
  per population.  FP16 takes the flat phase-0 and LDS-row phase-1 kernels,
  FP64 the per-cell kernel with the largest element offsets.
* 380^3 cells in FP32 and 480^3 cells in FP16: the blocked placement with a
  buffer just under 2^32 bytes, so lane byte offsets reach 4.2e9.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [((608, 608, 600), "f16"), ((608, 608, 600), "f64"),
         ((380, 380, 380), "f32"), ((480, 480, 480), "f16")]
SIZE = {"f64": 8, "f32": 4, "f16": 2}


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    import paper_2307_11752_amd as P
    from paper_2307_11752_amd import _lib

    _lib.load()
    return P


def _placement_bytes(lbm, shape, storage):
    """(bytes the library asks for, bytes of the blocked form, bytes of the arrays form)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    s = SIZE[storage]
    B = 32768 // s
    blocked = 19 * (-(-N // B)) * B * s
    arrays = 19 * (-(-N // 64)) * 64 * s
    from paper_2307_11752_amd.lattice import required_bytes

    got, _ = required_bytes(1, nx, ny, nz, storage)
    return got, blocked, arrays


@pytest.mark.parametrize("shape,storage", CASES)
def test_pure_streaming_at_the_offset_limit(orc, lbm, shape, storage):
    nx, ny, nz = shape
    assert 19 * nx * ny * nz < 2**32
    got, blocked, arrays = _placement_bytes(lbm, shape, storage)
    if blocked < 2**32:
        assert got == blocked and blocked > 0.97 * 2**32  # blocked, offsets near 2^32
    else:
        assert got == arrays
    print(f"[maxsize] D3Q19 {shape} {storage}: geometry", flush=True)
    c, w, _, _ = orc.descriptor(1)
    s = torch.cuda.Stream()
    lat = lbm.Lattice(1, shape, float("inf"), storage=storage, shifted=True, stream=s)
    lat.set_geometry(np.ones((nz, ny, nx), np.uint8), 7)
    dev = torch.device("cuda")
    z = torch.arange(nz, device=dev, dtype=torch.int64).view(nz, 1, 1)
    y = torch.arange(ny, device=dev, dtype=torch.int64).view(1, ny, 1)
    x = torch.arange(nx, device=dev, dtype=torch.int64).view(1, 1, nx)

    def initial(i):
        m = (7 * x + 13 * y + 29 * z + 5 * i) % 64 - 32
        return w[i] + m.to(torch.float64) * 2.0**-16

    print(f"[maxsize] {shape} {storage}: set_populations", flush=True)
    f0 = torch.empty((19, nz, ny, nx), dtype=torch.float64, device=dev)
    for i in range(19):
        f0[i] = initial(i)
    lat.set_populations(f0)
    del f0
    torch.cuda.empty_cache()
    done = 0
    for n in (1, 2):  # both propagation phases, odd and even totals
        lat.step(n)
        done += n
        print(f"[maxsize] {shape} {storage}: after {done} steps, compare", flush=True)
        got_f = lat.get_populations()
        for i in range(19):
            exp = torch.roll(initial(i), shifts=(done * int(c[i][2]), done * int(c[i][1]),
                                                 done * int(c[i][0])), dims=(0, 1, 2))
            assert torch.equal(got_f[i], exp), (storage, done, i)
            del exp
        del got_f
        torch.cuda.empty_cache()
    lat.close()
