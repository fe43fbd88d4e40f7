"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/lbm.h declares, sizes buffers as documented, validates
geometry with the same rule as the oracle and rejects bad arguments before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_11752_amd import _lib
from paper_2307_11752_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblbm_hip.so is not built; run __graft_entry__.build()")
    return _lib.load()


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = _declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_required_bytes(lib):
    p, a = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lbm_required_bytes(1, 256, 256, 256, _lib.STORE_F32, ctypes.byref(p), ctypes.byref(a)) == 0
    assert p.value == 19 * 256**3 * 4
    assert a.value >= 8 * 256**3
    assert lib.lbm_required_bytes(0, 64, 64, 1, _lib.STORE_F64, ctypes.byref(p), ctypes.byref(a)) == 0
    assert p.value == 9 * 64 * 64 * 8
    # within one chunk (32 KiB of a population): one array per population,
    # PS = N rounded up to 64 elements apart
    assert lib.lbm_required_bytes(1, 10, 10, 10, _lib.STORE_F16, ctypes.byref(p), None) == 0
    assert p.value == ((19 * 1024 * 2 + 255) // 256) * 256
    # blocked placement: N rounded up to whole chunks of 32 KiB / s cells
    assert lib.lbm_required_bytes(1, 100, 100, 100, _lib.STORE_F32, ctypes.byref(p), None) == 0
    assert p.value == 19 * (-(-10**6 // 8192)) * 8192 * 4
    assert lib.lbm_required_bytes(0, 200, 90, 1, _lib.STORE_F64, ctypes.byref(p), None) == 0
    assert p.value == 9 * 5 * 4096 * 8
    # 2^32 bytes or more: arrays again (32-bit byte offsets inside a blocked buffer)
    assert lib.lbm_required_bytes(1, 608, 608, 600, _lib.STORE_F16, ctypes.byref(p), None) == 0
    assert p.value == 19 * 608 * 608 * 600 * 2
    assert lib.lbm_required_bytes(0, 8, 8, 2, 0, ctypes.byref(p), None) == _lib.ERR_ARG
    assert lib.lbm_required_bytes(1, 0, 8, 8, 0, ctypes.byref(p), None) == _lib.ERR_ARG
    assert lib.lbm_required_bytes(1, 8, 8, 8, 9, ctypes.byref(p), None) == _lib.ERR_ARG
    assert lib.lbm_required_bytes(1, 1024, 1024, 1024, 1, ctypes.byref(p), None) == _lib.ERR_UNSUPPORTED


def test_required_bytes_follows_the_documented_placement(lib):
    """pop_bytes for seeded shapes against the rule stated in include/lbm.h:
    blocked (N rounded up to chunks of B = 32768 / s cells) when N > B and that
    stays below 2^32 bytes, else q arrays of N rounded up to 64; both rounded
    up to 256 bytes."""
    rng = np.random.default_rng(2307)
    size = {_lib.STORE_F64: 8, _lib.STORE_F32: 4, _lib.STORE_F16: 2, _lib.STORE_BF16: 2}
    p = ctypes.c_size_t()
    for _ in range(400):
        d = int(rng.integers(0, 2))
        q = 9 if d == 0 else 19
        st = int(rng.integers(0, 4))
        s = size[st]
        scale = float(rng.choice([1e1, 1e2, 1e3, 8e3]))
        nx, ny = (int(v) for v in rng.integers(1, scale, 2))
        nz = 1 if d == 0 else int(rng.integers(1, scale))
        N = nx * ny * nz
        if q * (-(-N // 64)) * 64 >= 2**32:
            assert lib.lbm_required_bytes(d, nx, ny, nz, st, ctypes.byref(p), None) == \
                _lib.ERR_UNSUPPORTED
            continue
        assert lib.lbm_required_bytes(d, nx, ny, nz, st, ctypes.byref(p), None) == 0
        B = 32768 // s
        blocked = q * (-(-N // B)) * B * s
        nbytes = blocked if (N > B and blocked < 2**32) else q * (-(-N // 64)) * 64 * s
        assert p.value == -(-nbytes // 256) * 256, (d, nx, ny, nz, st)



def test_batch_required_bytes_sums_the_members(lib):
    """A batch's population buffer is its members' buffers back to back, each
    sized as a lattice of its own (lbm_required_bytes, a multiple of 256 bytes);
    with 16-bit storage a member of odd nx stores its rows nx + 1 slots apart
    (include/lbm.h, batched ensembles).  Host only."""
    rng = np.random.default_rng(1107)
    p, a = ctypes.c_size_t(), ctypes.c_size_t()
    for st in (_lib.STORE_F64, _lib.STORE_F32, _lib.STORE_F16, _lib.STORE_BF16):
        for _ in range(20):
            count = int(rng.integers(1, 12))
            dims = [int(v) for v in rng.integers(3, 97, 3 * count)]
            expect = 0
            for k in range(count):
                nx, ny, nz = dims[3 * k: 3 * k + 3]
                px = nx + 1 if (st in (_lib.STORE_F16, _lib.STORE_BF16) and nx % 2) else nx
                assert lib.lbm_required_bytes(1, px, ny, nz, st, ctypes.byref(p), None) == 0
                assert p.value % 256 == 0
                expect += p.value
            arr = (ctypes.c_int * len(dims))(*dims)
            assert lib.lbm_batch_required_bytes(1, count, arr, st, ctypes.byref(p),
                                                ctypes.byref(a)) == 0
            assert p.value == expect, (st, dims)
            assert a.value > 0
    arr = (ctypes.c_int * 3)(8, 8, 8)
    assert lib.lbm_batch_required_bytes(1, 0, arr, _lib.STORE_F32, ctypes.byref(p), None) == \
        _lib.ERR_ARG
    wide = (ctypes.c_int * 3)(1030, 4, 4)  # a 16-bit row of 1030 cells needs 515 lanes > 512
    assert lib.lbm_batch_required_bytes(1, 1, wide, _lib.STORE_F16, ctypes.byref(p), None) == \
        _lib.ERR_UNSUPPORTED

def _create(lib, d=1, n=(8, 8, 8), tau=0.8, storage=1, flags=0, pop=256, pop_b=10**9, aux=512,
            aux_b=10**9):
    h = ctypes.c_void_p()
    st = lib.lbm_lattice_create(ctypes.byref(h), d, *n, tau, storage, flags,
                                ctypes.c_void_p(pop) if pop else None, pop_b,
                                ctypes.c_void_p(aux) if aux else None, aux_b, None)
    return st, h


def test_create_rejects_bad_arguments_before_device_calls(lib):
    # fake, never dereferenced addresses: every case below fails host-side checks
    assert _create(lib, tau=0.5)[0] == _lib.ERR_ARG
    assert _create(lib, tau=0.3)[0] == _lib.ERR_ARG
    assert _create(lib, tau=float("nan"))[0] == _lib.ERR_ARG
    assert _create(lib, tau=-float("inf"))[0] == _lib.ERR_ARG
    assert b"tau" in lib.lbm_last_error(None)
    assert _create(lib, d=0, n=(8, 8, 2))[0] == _lib.ERR_ARG
    assert _create(lib, d=7)[0] == _lib.ERR_ARG
    assert _create(lib, n=(8, -1, 8))[0] == _lib.ERR_ARG
    assert _create(lib, pop=0)[0] == _lib.ERR_ARG
    assert _create(lib, aux=0)[0] == _lib.ERR_ARG
    assert _create(lib, pop_b=100)[0] == _lib.ERR_ARG
    assert _create(lib, aux_b=100)[0] == _lib.ERR_ARG
    assert _create(lib, pop=256 + 4)[0] == _lib.ERR_ARG
    assert _create(lib, flags=8)[0] == _lib.ERR_ARG
    assert _create(lib, storage=11)[0] == _lib.ERR_ARG
    h = ctypes.c_void_p()
    assert lib.lbm_lattice_create(None, 1, 8, 8, 8, 0.8, 1, 0, None, 0, None, 0, None) == _lib.ERR_ARG
    assert h.value is None


def test_null_handle_calls(lib):
    assert lib.lbm_step(None, 1) == _lib.ERR_ARG
    assert lib.lbm_set_tau(None, 0.8) == _lib.ERR_ARG
    assert lib.lbm_lattice_destroy(None) == _lib.ERR_ARG
    assert lib.lbm_status_string(_lib.ERR_GEOMETRY) == b"geometry rejected"
    assert lib.lbm_status_string(-99) == b"unknown status"


@pytest.mark.parametrize("d,shape,periodic", [
    (1, (7, 6, 5), 0), (1, (7, 6, 5), 1), (1, (6, 6, 6), 5), (1, (5, 5, 5), 7),
    (0, (9, 8, 1), 0), (0, (9, 8, 1), 1), (0, (9, 8, 1), 3),
])
def test_geometry_rule_matches_oracle(lib, orc, d, shape, periodic):
    """The library's host check and the oracle's check (written independently)
    agree on valid layouts, on broken ones and on unsupported materials."""
    rng = np.random.default_rng(sum(shape) + periodic)
    for trial in range(40):
        mat = W.random_geometry(d, shape, periodic, seed=trial)
        if trial % 4 == 1:  # punch a material-0 hole
            mat[tuple(rng.integers(0, s) for s in mat.shape)] = 0
        if trial % 4 == 2:  # clear a random face (fluid may touch the box edge)
            mat[:, :, 0] = 1
        if trial % 8 == 3:
            mat[0, 0, 0] = rng.choice([4, 5, 9])
        nz, ny, nx = mat.shape
        a = lib.lbm_validate_geometry(d, nx, ny, nz, mat.ctypes.data_as(ctypes.c_void_p), periodic)
        b = orc.check_geometry(d, mat, periodic)
        assert a == b, (trial, a, b)


def test_channel_workload_is_valid(lib):
    wl = W.channel_spheres(nx=64, ny=32, nz=32, seed=5)
    mat = wl.material
    nz, ny, nx = mat.shape
    assert lib.lbm_validate_geometry(1, nx, ny, nz, mat.ctypes.data_as(ctypes.c_void_p), wl.periodic) == 0
    interior = mat[1:-1, 1:-1, :]
    frac = float(np.mean(interior == 2))
    assert 0.20 <= frac < 0.26


def test_cavity_workload_layout():
    wl = W.cavity2d(64)
    m = wl.material[0]
    assert m.shape == (64, 64)
    assert np.all(m[-1, :] == 3)
    assert np.all(m[0, :] == 2) and np.all(m[:-1, 0] == 2) and np.all(m[:-1, -1] == 2)
    assert np.all(m[1:-1, 1:-1] == 1)


def test_header_is_c_and_links(lib, tmp_path):
    """The public header compiles as strict C99 and a C program linked against
    the library makes the host-only calls (tests/c_abi_check.c)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "c_abi_check")
    libdir = os.path.dirname(_lib.LIB_PATH)
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_check.c"),
           "-L", libdir, "-llbm_hip", f"-Wl,-rpath,{libdir}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "c abi ok" in r.stdout
