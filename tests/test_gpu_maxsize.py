"""Lattices at the size limit of the 32-bit population offsets (q * N < 2^32).

Pure streaming (omega = 0, g = 0) on a fully periodic D3Q19 box of
608 x 608 x 600 cells (q * N = 4.21e9) must move every population by n c_i:
the GPU state after n steps is compared exactly with the initial state rolled
by n c_i (computed on the GPU with torch.roll; the permutation needs no
oracle).  FP16 storage takes the flat phase-0 and LDS-row phase-1 kernels,
FP64 storage the per-cell kernel with the largest byte offsets.  The initial
populations are w_i + m 2^-16 with small integers m, exact in both storages.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPE = (608, 608, 600)  # (nx, ny, nz): 19 * N = 4,213,407,744 < 2^32


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    import paper_2307_11752_amd as P
    from paper_2307_11752_amd import _lib

    _lib.load()
    return P


@pytest.mark.parametrize("storage", ["f16", "f64"])
def test_pure_streaming_at_the_offset_limit(orc, lbm, storage):
    nx, ny, nz = SHAPE
    assert 19 * nx * ny * nz < 2**32
    print(f"[maxsize] D3Q19 {SHAPE} {storage}: geometry", flush=True)
    c, w, _, _ = orc.descriptor(1)
    s = torch.cuda.Stream()
    lat = lbm.Lattice(1, SHAPE, float("inf"), storage=storage, shifted=True, stream=s)
    lat.set_geometry(np.ones((nz, ny, nx), np.uint8), 7)
    dev = torch.device("cuda")
    z = torch.arange(nz, device=dev, dtype=torch.int64).view(nz, 1, 1)
    y = torch.arange(ny, device=dev, dtype=torch.int64).view(1, ny, 1)
    x = torch.arange(nx, device=dev, dtype=torch.int64).view(1, 1, nx)

    def initial(i):
        m = (7 * x + 13 * y + 29 * z + 5 * i) % 64 - 32
        return w[i] + m.to(torch.float64) * 2.0**-16

    print(f"[maxsize] {storage}: set_populations", flush=True)
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
        print(f"[maxsize] {storage}: after {done} steps, compare", flush=True)
        got = lat.get_populations()
        for i in range(19):
            exp = torch.roll(initial(i), shifts=(done * int(c[i][2]), done * int(c[i][1]),
                                                 done * int(c[i][0])), dims=(0, 1, 2))
            assert torch.equal(got[i], exp), (storage, done, i)
            del exp
        del got
        torch.cuda.empty_cache()
    lat.close()
