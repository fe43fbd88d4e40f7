"""Batched ensemble (lbm_batch_*): every member after batch steps equals the
FP64 oracle run of that lattice alone, across storages, propagation phases,
graph replays and autotuned launch shapes."""
import numpy as np
import pytest

from _helpers import EPS_COMPUTE, rel_l2, representable, ulp_storage

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


from paper_2307_11752_amd import workloads as W  # noqa: E402

# Row lanes in phase 1: 16-bit rows take 2 cells (4 bytes) a lane, odd ones
# stored with one padding slot (pitch nx + 1); FP32 rows 2 cells (8 bytes) a
# lane when nx is even, else one; FP64 rows one cell a lane.  (3, 3, 3): 27
# cells, so the last 8-byte phase-0 lane runs into the padding.  (48, 20, 18): more
# cells than one chunk of the blocked placement for every storage type, rows
# straddling chunks.
SHAPES = [(5, 4, 3), (16, 9, 7), (7, 12, 5), (33, 3, 4), (3, 3, 3), (20, 17, 11), (64, 5, 2),
          (48, 20, 18), (18, 7, 5)]
TAUS = [0.56, 0.8, 1.0, 0.62, 0.9, 0.7, 0.55, 0.75, 0.65]


def _oracles(orc, shapes, taus, fields):
    refs = []
    for shape, tau, u in zip(shapes, taus, fields):
        nx, ny, nz = shape
        r = orc.Lattice(1, np.ones((nz, ny, nx), np.uint8), 7, tau)
        r.init_equilibrium(None, u)
        refs.append(r)
    return refs


def _fields(shapes, seed=0):
    rng = np.random.default_rng(seed)
    return [W.tgv3d_velocity(*s, rng.uniform(0.01, 0.08)) for s in shapes]


@pytest.mark.parametrize("storage,shifted", [("f64", True), ("f32", False), ("f32", True),
                                             ("f16", True), ("bf16", True)])
def test_batch_matches_oracle(orc, lbm, storage, shifted):
    fields = _fields(SHAPES)
    batch = lbm.Batch(1, SHAPES, TAUS, storage=storage, shifted=shifted)
    for m, u in zip(batch, fields):
        m.init_equilibrium(None, u)
    refs = _oracles(orc, SHAPES, TAUS, fields)
    w = orc.descriptor(1)[1]
    done = 0
    for n in (1, 2, 3):
        batch.step(n)
        for r in refs:
            r.step(n)
        done += n
        for m, r in zip(batch, refs):
            got = m.get_populations().cpu().numpy()
            wq = w[:, None, None, None]
            stored = r.f - wq if shifted else r.f
            if storage == "f64":
                tol = 1e-13
            else:
                tol = (done + 1) * (4 * ulp_storage(np.max(np.abs(stored)), storage)
                                    + 64 * EPS_COMPUTE[storage] * wq)
            assert np.all(np.abs(got - r.f) <= tol), (m.index, done)
            assert m.info()[0] == done
    batch.close()


SHAPES_2D = [(5, 4, 1), (16, 9, 1), (33, 12, 1), (64, 7, 1), (3, 3, 1), (130, 6, 1)]
TAUS_2D = [0.6, 0.8, 1.0, 0.55, 0.9, 0.7]


@pytest.mark.parametrize("storage,shifted", [("f64", True), ("f32", True), ("f16", True),
                                             ("bf16", True)])
def test_batch_d2q9_matches_oracle(orc, lbm, storage, shifted):
    """D2Q9 members (periodic in x and y) against the oracle: FP64 <= 1e-13;
    other storages |df| <= (n+1)(G ulp_S(max|stored|) + 64 eps w) with G = 6.
    The D3Q19 derivation of G = 4 assumes independent rounding errors; on the
    smallest members (a 3x3 box holds a handful of distinct values) the q
    input errors of a cell share their sign, and D2Q9's rest weight is 4/9:
    the rest population's gain omega w_0 sum_j df_j then reaches
    1.82 * (4/9) * 9 * 1/2 = 3.6 ulp per step for tau >= 0.55, plus the fresh
    half ulp and the carried (1 - omega) share: G = 6."""
    rng = np.random.default_rng(3)
    fields = [W.tgv3d_velocity(*s, rng.uniform(0.01, 0.08)) for s in SHAPES_2D]
    batch = lbm.Batch(0, SHAPES_2D, TAUS_2D, storage=storage, shifted=shifted)
    for m, u in zip(batch, fields):
        m.init_equilibrium(None, u)
    refs = []
    for (nx, ny, nz), tau, u in zip(SHAPES_2D, TAUS_2D, fields):
        r = orc.Lattice(0, np.ones((nz, ny, nx), np.uint8), 3, tau)
        r.init_equilibrium(None, u[:2])
        refs.append(r)
    w = orc.descriptor(0)[1]
    done = 0
    for n in (1, 2, 5):
        batch.step(n)
        for r in refs:
            r.step(n)
        done += n
        for m, r in zip(batch, refs):
            got = m.get_populations().cpu().numpy()
            wq = w[:, None, None, None]
            stored = r.f - wq if shifted else r.f
            if storage == "f64":
                tol = 1e-13
            else:
                tol = (done + 1) * (6 * ulp_storage(np.max(np.abs(stored)), storage)
                                    + 64 * EPS_COMPUTE[storage] * wq)
            assert np.all(np.abs(got - r.f) <= tol), (m.index, done)
    batch.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_batch_pure_streaming_bit_exact(orc, lbm, storage):
    taus = [float("inf")] * len(SHAPES)
    batch = lbm.Batch(1, SHAPES, taus, storage=storage, shifted=True)
    w = orc.descriptor(1)[1]
    rng = np.random.default_rng(3)
    refs = []
    for m, shape in zip(batch, SHAPES):
        nx, ny, nz = shape
        f0 = w[:, None, None, None] * (1 + rng.uniform(-0.3, 0.3, (19, nz, ny, nx)))
        f0 = representable(f0, w, storage, True)
        m.set_populations(f0)
        r = orc.Lattice(1, np.ones((nz, ny, nx), np.uint8), 7, float("inf"))
        r.set_populations(f0)
        refs.append(r)
    for n in (1, 2, 5):
        batch.step(n)
        for m, r in zip(batch, refs):
            r.step(n)
            assert np.array_equal(m.get_populations().cpu().numpy(), r.f)
    batch.close()


def test_batch_graph_and_launch_shapes_agree(lbm):
    """Every launch shape and graph replay gives bit-identical states."""
    fields = _fields(SHAPES, seed=5)
    results = []
    # (phase-0 shape, phase-1 shape, graph length)
    for s0, s1, graph in [((256, 8), (256, 8), 0), ((128, 2), (128, 2), 10),
                          ((512, 16), (512, 16), 10), ((256, 0), (256, 0), 4),
                          ((512, 0), (128, 4), 6), ((128, 0), (512, 0), 0)]:
        batch = lbm.Batch(1, SHAPES, TAUS, storage="f32", shifted=True)
        if s0 == s1:
            batch.set_launch(*s0)
        else:
            batch.set_launch(256, 8)
            batch.set_phase_launch(0, *s0)
            batch.set_phase_launch(1, *s1)
        assert (batch.phase_launch(0), batch.phase_launch(1)) == (s0, s1)
        batch.set_graph_steps(graph)
        for m, u in zip(batch, fields):
            m.init_equilibrium(None, u)
        states = []
        for n in (10, 7, 21):
            batch.step(n)
            torch.cuda.synchronize()
            states.append([m.get_populations() for m in batch])
        results.append(states)
        batch.close()
    for other in results[1:]:
        for sa, sb in zip(results[0], other):
            for a, b in zip(sa, sb):
                assert torch.equal(a, b)



@pytest.mark.parametrize("storage,shifted", [("f32", False), ("f16", True)])
def test_batch_xcd_runs_cover_every_item(lbm, storage, shifted):
    """With one block per phase-1 item the kernel deals runs of consecutive
    items to one XCD (a permutation of the items once there are at least
    8 x 64 of them); the persistent shape walks them in order.  64 members of
    16^3 in 128-thread blocks give 1024 phase-1 items: both must agree bitwise."""
    shapes = [(16, 16, 16)] * 64
    taus = [0.6 + 0.005 * k for k in range(64)]
    fields = _fields(shapes, seed=17)
    states = []
    for bpc in (0, 16):
        batch = lbm.Batch(1, shapes, taus, storage=storage, shifted=shifted)
        batch.set_launch(128, bpc)
        for m, u in zip(batch, fields):
            m.init_equilibrium(None, u)
        batch.step(7)
        torch.cuda.synchronize()
        states.append([m.get_populations() for m in batch])
        batch.close()
    for a, b in zip(*states):
        assert torch.equal(a, b)

def test_batch_autotune_then_parity(orc, lbm):
    fields = _fields(SHAPES, seed=9)
    batch = lbm.Batch(1, SHAPES, TAUS, storage="f64", shifted=True)
    for m, u in zip(batch, fields):  # autotune needs initialised members
        m.init_equilibrium(None, u)
    t, b, ms = batch.autotune(trial_steps=4)
    assert t in (128, 256, 512) and b in (0, 2, 4, 8, 16) and ms > 0
    info = batch.info()
    assert (info["threads"], info["blocks_per_cu"]) == (t, b) == batch.phase_launch(1)
    t0, b0 = batch.phase_launch(0)  # each phase keeps its own fastest shape
    assert t0 in (128, 256, 512) and b0 in (0, 2, 4, 8, 16)
    for m, u in zip(batch, fields):  # start over from the initial state
        m.init_equilibrium(None, u)
    refs = _oracles(orc, SHAPES, TAUS, fields)
    batch.set_graph_steps(6)
    batch.step(13)
    for m, r in zip(batch, refs):
        r.step(13)
        assert np.max(np.abs(m.get_populations().cpu().numpy() - r.f)) <= 1e-13
    batch.close()


def test_batch_call_order_errors(lbm):
    from paper_2307_11752_amd import _lib

    batch = lbm.Batch(1, SHAPES[:3], TAUS[:3], storage="f32")
    with pytest.raises(_lib.LBMError) as e:
        batch.step(1)  # members not initialised
    assert e.value.status == _lib.ERR_STATE
    for m in batch:
        m.init_equilibrium()
    batch.step(1)
    with pytest.raises(_lib.LBMError) as e:
        batch[0].step(1)
    assert e.value.status == _lib.ERR_STATE
    with pytest.raises(_lib.LBMError) as e:
        batch[1].set_tau(0.9)
    assert e.value.status == _lib.ERR_STATE
    batch[0].init_equilibrium()  # back to phase 0 while the others are in phase 1
    with pytest.raises(_lib.LBMError) as e:
        batch.step(1)
    assert e.value.status == _lib.ERR_STATE
    with pytest.raises(_lib.LBMError):
        batch.set_launch(100, 4)
    with pytest.raises(_lib.LBMError):
        batch.set_launch(256, -1)
    with pytest.raises(_lib.LBMError) as e:
        batch.set_phase_launch(2, 256, 0)
    assert e.value.status == _lib.ERR_ARG
    with pytest.raises(_lib.LBMError):
        batch.set_phase_launch(0, 96, 0)
    batch.set_phase_launch(0, 512, 0)  # the other phase keeps its shape
    assert batch.phase_launch(0) == (512, 0)
    for bad in (0, 3, 1002):  # trial lengths must be even, 2..1000
        with pytest.raises(_lib.LBMError) as e:
            batch.autotune(trial_steps=bad)
        assert e.value.status == _lib.ERR_ARG
    batch.close()


def test_ensemble_config_sampled(orc, lbm):
    """The 256-lattice ensemble (edges log-uniform 16-96, u0 in [0.01, 0.08],
    tau in [0.55, 1.0]) in the benchmark's launch configuration: a sample of
    members (smallest, largest, and random ones) equals the oracle after 3 steps."""
    shapes, u0, taus = W.tgv_ensemble()
    batch = lbm.Batch(1, shapes, taus, storage="f32", shifted=True)
    batch.set_graph_steps(100)
    for m, s, a in zip(batch, shapes, u0):
        m.init_equilibrium(None, W.tgv3d_velocity(*s, a))
    batch.step(3)
    sizes = [np.prod(s) for s in shapes]
    rng = np.random.default_rng(0)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(len(shapes), 4, replace=False)})
    w = orc.descriptor(1)[1]
    for l in pick:
        nx, ny, nz = shapes[l]
        u = W.tgv3d_velocity(nx, ny, nz, u0[l])
        r = orc.Lattice(1, np.ones((nz, ny, nx), np.uint8), 7, taus[l])
        r.init_equilibrium(None, u)
        r.step(3)
        got = batch[l].get_populations().cpu().numpy()
        wq = w[:, None, None, None]
        tol = 4 * (4 * ulp_storage(np.max(np.abs(r.f - wq)), "f32") + 64 * 2.0**-24 * wq)
        assert np.all(np.abs(got - r.f) <= tol), l
        rho_g, u_g = batch[l].moments()
        rho_o, u_o = r.moments()
        assert rel_l2(u_g, u_o) < 1e-5
    batch.close()
