"""GPU parity: the gfx950 path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bars, each from the arithmetic of the step:
* pure streaming (omega = 0, g = 0, u_w = 0), any storage, odd and even step
  counts: bit-exact (a permutation of stored values);
* FP64 storage, full steps with forcing and moving walls: max |df| <= 1e-13
  (~30 flops per population per step at 2^-53 on values <= 0.5, FMA
  contraction on the GPU only, <= 20 steps: ~1e-14, with a factor 10 margin);
* one step from an exactly representable state, any storage: every population
  within one storage ulp plus 64 compute-type eps of its weight (rounding to
  storage <= 1/2 ulp, a tie may go either way, ~10 eps * w of collision
  arithmetic);
* FP32 storage, many steps: velocity rel-L2 <= 1e-5 (100 steps);
* moments / totals of a state equal the oracle's of the same state to FP64
  rounding.
"""
import numpy as np
import pytest

from _helpers import EPS_COMPUTE, encode_decode, rel_l2, representable, ulp_storage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    import paper_2307_11752_amd as P
    from paper_2307_11752_amd import _lib

    _lib.load()  # raises loudly if the HIP library was not built
    return P


from paper_2307_11752_amd import workloads as W  # noqa: E402

CASES_3D = [
    ((7, 5, 6), 0b000),
    ((9, 6, 5), 0b001),
    ((6, 7, 8), 0b101),
    ((5, 4, 6), 0b111),
    ((70, 9, 7), 0b011),   # more than one x-block of 64 threads, ragged tail
    ((300, 4, 3), 0b111),  # two 256-wide x-blocks, ragged tail
    ((64, 34, 32), 0b001),  # >= 65536 cells: masked lattices take the flat phase-0 kernel
    # >= 65536 cells, rows not a multiple of 64: flat phase 0 with a ragged tail,
    # per-cell phase 1
    ((66, 33, 31), 0b011),
    ((520, 12, 11), 0b111),
    # >= 65536 cells with walls on the x and y faces and rows of 48 cells
    # (a multiple of every lane width): flat masked phase 0, per-cell phase 1
    ((48, 37, 37), 0b100),
]
CASES_2D = [
    ((9, 7, 1), 0b00),
    ((12, 10, 1), 0b01),
    ((8, 9, 1), 0b11),
    ((130, 5, 1), 0b01),
    ((272, 256, 1), 0b01),  # >= 65536 cells: masked D2Q9 takes the flat phase-0 kernel
]
# Fully fluid periodic boxes take the flat phase-0 kernel always, and the row
# kernels for phase 1 when nx is a multiple of the cells per lane (8 bytes /
# storage size) and a row fits 256 lanes; the shapes cover rows held by part
# of a wave or one wave (16-bit storage), the LDS row tile with one and many
# rows per block, and phase 1 falling back to the per-cell kernel (nx not a
# multiple).
FLUID_3D = [(8, 6, 5), (12, 5, 4), (64, 4, 3), (256, 3, 2), (512, 2, 3), (6, 5, 4),
            (20, 3, 7),  # FP32: 12 rows of 10 lanes per LDS-row block, the last one 9 rows
            (256, 5, 3), (512, 3, 3),
            # more cells than one chunk of the blocked placement (4096 / 8192 /
            # 16384 cells for 8- / 4- / 2-byte storage), rows that straddle
            # chunks, a ragged last chunk
            (300, 30, 4), (96, 40, 9), (64, 32, 9),
            (7, 5, 3)]  # an odd cell count: the last phase-0 lane runs into the padding
FLUID_2D = [(16, 10, 1), (128, 6, 1), (36, 7, 1), (10, 9, 1), (200, 90, 1), (9, 7, 1)]


def _pair(orc, lbm, d, shape, periodic, tau, storage, shifted, seed, g=(0, 0, 0), uw=(0, 0, 0),
          fluid_only=False):
    """GPU lattice + oracle lattice with identical geometry and parameters."""
    if fluid_only:
        nx, ny, nz = shape
        mat = np.ones((nz, ny, nx), np.uint8)
    else:
        mat = W.random_geometry(d, shape, periodic, seed)
    gpu = lbm.Lattice(d, shape, tau, storage=storage, shifted=shifted)
    gpu.set_geometry(mat, periodic)
    gpu.set_body_force(g)
    gpu.set_wall_velocity(uw)
    ref = orc.Lattice(d, mat, periodic, tau, g=g, u_wall=uw)
    return gpu, ref, mat


def _fluid(mat):
    return mat == 1


def _weights(orc, d):
    return orc.descriptor(d)[1]


# ---------------------------------------------------------------------------
# Pure streaming: bit-exact for every storage, both propagation phases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,shifted", [("f64", False), ("f64", True), ("f32", False),
                                             ("f32", True), ("f16", True), ("bf16", True),
                                             ("f16", False)])
@pytest.mark.parametrize("d,case", [(1, c) for c in CASES_3D] + [(0, c) for c in CASES_2D])
def test_pure_streaming_bit_exact(orc, lbm, storage, shifted, d, case):
    shape, periodic = case
    print(f"[pure-streaming] d={d} shape={shape} periodic={periodic} {storage} shifted={shifted}",
          flush=True)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, float("inf"), storage, shifted, seed=17)
    w = _weights(orc, d)
    rng = np.random.default_rng(99)
    q = len(w)
    nx, ny, nz = shape
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.3, 0.3, (q, nz, ny, nx)))
    f0 = representable(f0, w, storage, shifted)
    f0[:, ~_fluid(mat)] = 0.0
    gpu.set_populations(f0)
    back = gpu.get_populations().cpu().numpy()
    assert np.array_equal(back, f0), "set/get round trip is not exact"
    ref.set_populations(f0)
    done = 0
    for n in (1, 1, 2, 3):
        gpu.step(n)
        ref.step(n)
        done += n
        got = gpu.get_populations().cpu().numpy()
        fl = _fluid(mat)
        assert np.array_equal(got[:, fl], ref.f[:, fl]), f"mismatch after {done} steps"


@pytest.mark.parametrize("storage,shifted", [("f64", False), ("f32", False), ("f32", True),
                                             ("f16", True), ("bf16", True)])
@pytest.mark.parametrize("d,shape", [(1, s) for s in FLUID_3D] + [(0, s) for s in FLUID_2D])
def test_pure_streaming_bit_exact_fluid_box(orc, lbm, storage, shifted, d, shape):
    periodic = 0b111 if d == 1 else 0b011
    print(f"[pure-streaming fluid] d={d} shape={shape} {storage} shifted={shifted}", flush=True)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, float("inf"), storage, shifted, seed=1,
                          fluid_only=True)
    w = _weights(orc, d)
    rng = np.random.default_rng(7)
    nx, ny, nz = shape
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.3, 0.3, (len(w), nz, ny, nx)))
    f0 = representable(f0, w, storage, shifted)
    gpu.set_populations(f0)
    ref.set_populations(f0)
    done = 0
    for n in (1, 1, 2, 3):
        gpu.step(n)
        ref.step(n)
        done += n
        got = gpu.get_populations().cpu().numpy()
        assert np.array_equal(got, ref.f), f"mismatch after {done} steps"


# ---------------------------------------------------------------------------
# Initialisation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,shifted", [("f64", False), ("f64", True), ("f32", False),
                                             ("f32", True), ("f16", True), ("bf16", True)])
@pytest.mark.parametrize("d", [0, 1])
def test_init_equilibrium(orc, lbm, storage, shifted, d):
    shape, periodic = (CASES_3D[1] if d == 1 else CASES_2D[1])
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, 0.8, storage, shifted, seed=3)
    rho = W.random_density(shape, 4)
    u = W.random_velocity(shape, 5, dim=3 if d == 1 else 2)
    gpu.init_equilibrium(rho, u)
    ref.init_equilibrium(rho, u[: (3 if d == 1 else 2)])
    got = gpu.get_populations().cpu().numpy()
    w = _weights(orc, d)
    expect = encode_decode(ref.f, w, storage, shifted)
    fl = _fluid(mat)
    tol = ulp_storage(np.abs(ref.f[:, fl]) + w[:, None], storage) + 4e-16
    assert np.all(np.abs(got[:, fl] - expect[:, fl]) <= tol)


# ---------------------------------------------------------------------------
# FP64: full steps with forcing and moving walls
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shifted", [False, True])
@pytest.mark.parametrize("d,case", [(1, c) for c in CASES_3D] + [(0, c) for c in CASES_2D])
def test_fp64_full_steps(orc, lbm, shifted, d, case):
    shape, periodic = case
    print(f"[fp64] d={d} shape={shape} periodic={periodic} shifted={shifted}", flush=True)
    g = (2e-4, -1e-4, 5e-5) if d == 1 else (2e-4, -1e-4, 0.0)
    uw = (0.03, 0.0, -0.02) if d == 1 else (0.03, -0.01, 0.0)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, 0.7, "f64", shifted, seed=21, g=g, uw=uw)
    rho = W.random_density(shape, 8)
    u = W.random_velocity(shape, 9, dim=3 if d == 1 else 2)
    gpu.init_equilibrium(rho, u)
    ref.init_equilibrium(rho, u[: (3 if d == 1 else 2)])
    fl = _fluid(mat)
    worst = 0.0
    for n in (1, 1, 5, 13):
        gpu.step(n)
        ref.step(n)
        got = gpu.get_populations().cpu().numpy()
        err = float(np.max(np.abs(got[:, fl] - ref.f[:, fl])))
        worst = max(worst, err)
        assert err <= 1e-13, err
    print(f"  max|df| = {worst:.3e}")
    # moments and totals of the final state
    rho_g, u_g = gpu.moments()
    rho_o, u_o = ref.moments()
    assert np.max(np.abs(rho_g - rho_o)) <= 1e-13
    assert np.max(np.abs(u_g - u_o)) <= 1e-13
    # the device call decodes the same way and rounds once to float
    rd, ud = gpu.moments_device()
    assert np.array_equal(rd.cpu().numpy(), rho_g.astype(np.float32))
    assert np.array_equal(ud.cpu().numpy(), u_g.astype(np.float32))
    m_g, j_g, s_g = gpu.totals()
    m_o, j_o, s_o = ref.totals()
    assert abs(m_g - m_o) <= 1e-12 * m_o
    # the two sides sum N per-cell momenta (each below 1) in different orders:
    # rounding differs by at most about N * eps
    np.testing.assert_allclose(j_g, j_o, rtol=0, atol=1e-15 * mat.size)
    np.testing.assert_allclose(s_g, s_o, rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_moments_span_several_scratch_chunks(orc, lbm, storage):
    """lbm_moments decodes through a device scratch of 32768 cells per chunk:
    a lattice of 69,120 cells takes three chunks, the last one partial."""
    shape, periodic = (48, 40, 36), W.PERIODIC_X | W.PERIODIC_Z
    print(f"[moments chunks] shape={shape} storage={storage}", flush=True)
    gpu, ref, mat = _pair(orc, lbm, 1, shape, periodic, 0.7, storage, True, seed=31,
                          g=(1e-4, 0.0, 2e-5), uw=(0.02, 0.0, 0.0))
    rho = W.random_density(shape, 4)
    u = W.random_velocity(shape, 5)
    gpu.init_equilibrium(rho, u)
    ref.init_equilibrium(rho, u)
    gpu.step(3)
    ref.step(3)
    rho_g, u_g = gpu.moments()
    rho_o, u_o = ref.moments()
    fl = _fluid(mat)
    bar = 1e-13 if storage == "f64" else 1e-5
    assert np.max(np.abs(rho_g[fl] - rho_o[fl])) <= bar
    assert np.max(np.abs(u_g[:, fl] - u_o[:, fl])) <= bar
    assert not np.any(rho_g[~fl]) and not np.any(u_g[:, ~fl])
    rd, ud = gpu.moments_device()
    assert np.array_equal(rd.cpu().numpy(), rho_g.astype(np.float32))
    assert np.array_equal(ud.cpu().numpy(), u_g.astype(np.float32))


@pytest.mark.parametrize("shifted", [False, True])
@pytest.mark.parametrize("d,shape", [(1, s) for s in FLUID_3D] + [(0, s) for s in FLUID_2D])
def test_fp64_full_steps_fluid_box(orc, lbm, shifted, d, shape):
    periodic = 0b111 if d == 1 else 0b011
    g = (2e-4, -1e-4, 5e-5) if d == 1 else (2e-4, -1e-4, 0.0)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, 0.7, "f64", shifted, seed=2, g=g,
                          fluid_only=True)
    rho = W.random_density(shape, 8)
    u = W.random_velocity(shape, 9, dim=3 if d == 1 else 2)
    gpu.init_equilibrium(rho, u)
    ref.init_equilibrium(rho, u[: (3 if d == 1 else 2)])
    for n in (1, 1, 4, 9):
        gpu.step(n)
        ref.step(n)
        got = gpu.get_populations().cpu().numpy()
        err = float(np.max(np.abs(got - ref.f)))
        assert err <= 1e-13, err


# ---------------------------------------------------------------------------
# One step from an exactly representable state, every storage type
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,shifted", [("f64", True), ("f32", False), ("f32", True),
                                             ("f16", True), ("bf16", True)])
@pytest.mark.parametrize("d,case", [(1, CASES_3D[0]), (1, CASES_3D[3]), (1, CASES_3D[4]),
                                    (1, CASES_3D[6]), (1, CASES_3D[7]), (1, CASES_3D[8]),
                                    (1, CASES_3D[9]),
                                    (0, CASES_2D[0]), (0, CASES_2D[3]), (0, CASES_2D[4]),
                                    (1, ((64, 4, 3), "fluid")), (1, ((12, 5, 4), "fluid")),
                                    (0, ((128, 6, 1), "fluid"))])
@pytest.mark.parametrize("parity", [0, 1])
def test_one_step_within_storage_ulp(orc, lbm, storage, shifted, d, case, parity):
    shape, periodic = case
    fluid_only = periodic == "fluid"
    if fluid_only:
        periodic = 0b111 if d == 1 else 0b011
    g = (3e-4, 1e-4, -2e-4) if d == 1 else (3e-4, 1e-4, 0.0)
    uw = (0.04, 0.0, 0.01) if d == 1 else (0.04, 0.0, 0.0)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, 0.6, storage, shifted, seed=33, g=g, uw=uw,
                          fluid_only=fluid_only)
    w = _weights(orc, d)
    ref.init_equilibrium(W.random_density(shape, 1), W.random_velocity(shape, 2, dim=3 if d else 2)[: 3 if d else 2])
    rng = np.random.default_rng(5)
    f0 = ref.f * (1 + rng.uniform(-0.02, 0.02, ref.f.shape))  # off equilibrium
    f0 = representable(f0, w, storage, shifted)
    fl = _fluid(mat)
    f0[:, ~fl] = 0.0
    gpu.set_populations(f0)
    if parity:  # move the GPU to the swapped layout with a pure-streaming step
        gpu.set_tau(float("inf"))
        ref_stream = orc.Lattice(d, mat, periodic, float("inf"))
        ref_stream.set_populations(f0)
        ref_stream.step(1)
        gpu.set_body_force((0, 0, 0))
        gpu.set_wall_velocity((0, 0, 0))
        gpu.step(1)
        gpu.set_tau(0.6)
        gpu.set_body_force(g)
        gpu.set_wall_velocity(uw)
        f0 = ref_stream.f
    ref.set_populations(f0)
    gpu.step(1)
    ref.step(1)
    got = gpu.get_populations().cpu().numpy()[:, fl]
    exp = ref.f[:, fl]
    wq = np.broadcast_to(w[:, None], exp.shape)
    stored = exp - wq if shifted else exp
    tol = ulp_storage(stored, storage) + 64 * EPS_COMPUTE[storage] * wq
    err = np.abs(got - exp)
    print(f"[one-step] {storage} shifted={shifted} d={d} max err/tol = {np.max(err / tol):.3f}")
    assert np.all(err <= tol)


# ---------------------------------------------------------------------------
# FP32: many steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shifted", [False, True])
@pytest.mark.parametrize("d,case", [(1, CASES_3D[2]), (1, CASES_3D[4]), (1, CASES_3D[7]),
                                    (1, CASES_3D[6]), (1, CASES_3D[9]),
                                    (0, CASES_2D[2]), (0, CASES_2D[4]),
                                    (1, ((64, 6, 5), "fluid")), (0, ((128, 16, 1), "fluid"))])
def test_fp32_many_steps(orc, lbm, shifted, d, case):
    shape, periodic = case
    fluid_only = periodic == "fluid"
    if fluid_only:
        periodic = 0b111 if d == 1 else 0b011
    g = (1e-4, 0.0, 0.0)
    uw = (0.05, 0.0, 0.0)
    gpu, ref, mat = _pair(orc, lbm, d, shape, periodic, 0.8, "f32", shifted, seed=41, g=g, uw=uw,
                          fluid_only=fluid_only)
    u = W.random_velocity(shape, 6, amplitude=0.03, dim=3 if d else 2)
    gpu.init_equilibrium(None, u)
    ref.init_equilibrium(None, u[: 3 if d else 2])
    gpu.step(100)
    ref.step(100)
    fl = _fluid(mat)
    rho_g, u_g = gpu.moments()
    rho_o, u_o = ref.moments()
    e = rel_l2(u_g[:, fl], u_o[:, fl])
    print(f"[fp32-100] d={d} shifted={shifted} u rel-L2 = {e:.3e}, "
          f"rho max err = {np.max(np.abs(rho_g[fl] - rho_o[fl])):.3e}")
    assert e <= 1e-5
    assert np.max(np.abs(rho_g[fl] - rho_o[fl])) <= 1e-5


# ---------------------------------------------------------------------------
# HIP graph replay
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,shape,periodic,storage", [(1, (20, 12, 10), 0b001, "f32"),
                                                      (1, (64, 8, 6), 0b111, "f16"),
                                                      (0, (64, 64, 1), 0b00, "f64"),
                                                      (1, (40, 24, 20), 0b001, "f32"),
                                                      (1, (64, 16, 20), 0b111, "f16"),
                                                      (0, (160, 128, 1), 0b00, "f64")])
def test_graph_replay_matches_direct_launches(orc, lbm, d, shape, periodic, storage):
    """Replays of a captured 10-step graph, interleaved with eager work and
    synchronisation, give bit-identical states to direct launches every time."""
    s = torch.cuda.Stream()
    if periodic == 0b111:
        nx, ny, nz = shape
        mat = np.ones((nz, ny, nx), np.uint8)
    else:
        mat = W.random_geometry(d, shape, periodic, seed=4)
    g = (1e-4, 2e-5, 0.0)
    uw = (0.05, 0.0, 0.0)
    lats = []
    for graph in (True, False):
        lat = lbm.Lattice(d, shape, 0.7, storage=storage, shifted=storage != "f64", stream=s)
        lat.set_geometry(mat, periodic)
        lat.set_body_force(g)
        lat.set_wall_velocity(uw)
        lat.init_equilibrium(None, W.random_velocity(shape, 3, dim=3 if d else 2))
        if graph:
            lat.set_graph_steps(10)
        lats.append(lat)
    a, b = lats
    for n in (10, 23, 7, 31, 10):
        a.step(n)
        b.step(n)
        torch.cuda.synchronize()
        ra, ua = a.moments_device()  # eager work between replays
        rb, ub = b.moments_device()
        assert torch.equal(ua, ub) and torch.equal(ra, rb)
        assert torch.equal(a.get_populations(), b.get_populations())
    # a parameter change rebuilds the graph
    for lat in (a, b):
        lat.set_tau(0.9)
        lat.step(20)
    assert torch.equal(a.get_populations(), b.get_populations())
    assert a.info()[0] == b.info()[0] == 101


# ---------------------------------------------------------------------------
# Stream order between the caller's stream and the lattice's stream
# ---------------------------------------------------------------------------
def test_inputs_from_a_busy_caller_stream(lbm):
    """A lattice on a stream of its own reads an input that the caller's stream
    is still producing (queued behind ~40 GB of unrelated traffic): the library
    call waits for it, and the output is ordered before the caller's next work."""
    shape = (40, 24, 20)
    nx, ny, nz = shape
    s = torch.cuda.Stream()
    lat = lbm.Lattice(1, shape, 0.8, storage="f32", stream=s)
    lat.set_geometry(np.ones((nz, ny, nx), np.uint8), 7)
    rng = np.random.default_rng(5)
    want = torch.from_numpy(rng.integers(1, 1024, size=(19, nz, ny, nx)) / 1024.0).cuda()
    torch.cuda.synchronize()
    busy = torch.ones(2**28, device="cuda")
    f = torch.zeros_like(want)
    for _ in range(20):
        busy.mul_(1.0)
    f.copy_(want)
    lat.set_populations(f)  # f32 holds k / 1024 exactly
    got = lat.get_populations()
    assert torch.equal(got, want)
    lat.close()


# ---------------------------------------------------------------------------
# Call-order and argument errors through the ABI on the GPU
# ---------------------------------------------------------------------------
def test_state_errors(lbm):
    from paper_2307_11752_amd import _lib

    lat = lbm.Lattice(1, (4, 4, 4), 0.8)
    with pytest.raises(_lib.LBMError) as e:
        lat.step(1)
    assert e.value.status == _lib.ERR_STATE
    with pytest.raises(_lib.LBMError) as e:
        lat.set_geometry(np.zeros((4, 4, 4), np.uint8) + 1, 0)
    assert e.value.status == _lib.ERR_GEOMETRY
    lat.set_geometry(np.ones((4, 4, 4), np.uint8), 7)
    with pytest.raises(_lib.LBMError) as e:
        lat.step(1)
    assert e.value.status == _lib.ERR_STATE
    lat.init_equilibrium()
    lat.step(3)
    assert lat.info() == (3, 64)
    with pytest.raises(_lib.LBMError) as e:
        lat.set_tau(0.5)
    assert e.value.status == _lib.ERR_ARG
    nan = np.full((19, 4, 4, 4), np.nan)
    lat.set_populations(nan)
    with pytest.raises(_lib.LBMError) as e:
        lat.totals()
    assert e.value.status == _lib.ERR_NONFINITE
