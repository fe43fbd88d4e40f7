"""Porosity gradients (lbm_porous_*): the GPU forward model and hand-written
adjoint against the FP64 oracle's forward model and discrete adjoint, the
checkpoint interval's invariance, and the torch.autograd wrapper."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def adj():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    from paper_2307_11752_amd import _lib, adjoint

    _lib.load()
    return adjoint


def _smooth_porosity(shape, seed, lo=0.2, hi=1.0):
    """Seeded smooth noise: box-filtered white noise mapped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(size=shape)
    for ax in range(3):
        a = (np.roll(a, 1, ax) + a + np.roll(a, -1, ax)) / 3.0
    a = (a - a.min()) / (a.max() - a.min())
    return lo + (hi - lo) * a


def _channel(shape, interior_walls=True, seed=0):
    nz, ny, nx = shape
    mat = np.ones(shape, np.uint8)
    mat[:, 0, :] = 2
    mat[:, -1, :] = 2
    mat[0, :, :] = 2
    mat[-1, :, :] = 2
    if interior_walls:
        rng = np.random.default_rng(seed)
        inner = rng.uniform(size=shape) < 0.05
        inner[:, :, -1] = False  # keep the objective plane open
        mat[inner & (mat == 1)] = 2
    return mat


SHAPE = (12, 10, 16)  # (nz, ny, nx)
TAU, G, STEPS = 0.7, (1e-4, 0.0, 0.0), 60


def test_forward_and_gradient_match_oracle(orc, adj):
    mat = _channel(SHAPE)
    por = _smooth_porosity(SHAPE, 3)
    ref = orc.PorousProblem(1, mat, 0b001, TAU, G)
    J_o, grad_o = ref.gradient(por, STEPS)
    _, fT_o = ref.forward(por, STEPS)
    prob = adj.PorousChannel(mat, 0b001, TAU, G, STEPS, 10)
    d = torch.tensor(por, dtype=torch.float32, device="cuda")
    J_g = prob.forward(d)
    grad_g = prob.backward().cpu().numpy().astype(np.float64)
    fT_g = prob.final_populations().cpu().numpy()
    fl = mat == 1
    ferr = float(np.max(np.abs(fT_g[:, fl] - fT_o[:, fl])))
    gerr = float(np.linalg.norm(grad_g[fl] - grad_o[fl]) / np.linalg.norm(grad_o[fl]))
    gmax = float(np.max(np.abs(grad_g[fl] - grad_o[fl])) / np.max(np.abs(grad_o[fl])))
    print(f"[adjoint] J gpu {J_g:.9e} oracle {J_o:.9e} rel {abs(J_g / J_o - 1):.2e}; "
          f"max|df| {ferr:.2e}; grad rel-L2 {gerr:.2e}, rel-max {gmax:.2e}")
    assert np.all(grad_g[~fl] == 0.0)
    # FP32 arithmetic and storage of the deviations f - w (~1e-4 here): relative
    # rounding ~1e-7 per operation, accumulated over 60 forward and 60 adjoint
    # steps (measured: |df| 4e-11, J 8e-8, gradient 5e-7)
    assert ferr <= 1e-9
    assert abs(J_g / J_o - 1.0) <= 1e-6
    assert gerr <= 2e-5 and gmax <= 1e-4
    prob.close()


@pytest.mark.parametrize("shape", [(8, 10, 128), (6, 8, 256)])
def test_long_rows_forward_and_gradient_match_oracle(orc, adj, shape):
    """Plain channels (walls on the y and z faces only, periodic x) with x-rows
    as long as the benchmark's (128) and twice that, so that a block spans
    less than one row; same bars as the default case."""
    mat = _channel(shape, interior_walls=False)
    por = _smooth_porosity(shape, 11)
    steps = 40
    ref = orc.PorousProblem(1, mat, 0b001, TAU, G)
    J_o, grad_o = ref.gradient(por, steps)
    _, fT_o = ref.forward(por, steps)
    print(f"[adjoint long rows] shape {shape}", flush=True)
    prob = adj.PorousChannel(mat, 0b001, TAU, G, steps, 8)
    d = torch.tensor(por, dtype=torch.float32, device="cuda")
    J_g = prob.forward(d)
    grad_g = prob.backward().cpu().numpy().astype(np.float64)
    fT_g = prob.final_populations().cpu().numpy()
    fl = mat == 1
    ferr = float(np.max(np.abs(fT_g[:, fl] - fT_o[:, fl])))
    gerr = float(np.linalg.norm(grad_g[fl] - grad_o[fl]) / np.linalg.norm(grad_o[fl]))
    gmax = float(np.max(np.abs(grad_g[fl] - grad_o[fl])) / np.max(np.abs(grad_o[fl])))
    print(f"  J rel {abs(J_g / J_o - 1):.2e}; max|df| {ferr:.2e}; grad rel-L2 {gerr:.2e}, "
          f"rel-max {gmax:.2e}")
    assert np.all(grad_g[~fl] == 0.0)
    assert ferr <= 1e-9
    assert abs(J_g / J_o - 1.0) <= 1e-6
    assert gerr <= 2e-5 and gmax <= 1e-4
    prob.close()


@pytest.mark.parametrize("every", [1, 7, 60])
def test_checkpoint_interval_does_not_change_the_gradient(adj, every):
    """Recomputation from checkpoints reproduces the stored states exactly, so
    the gradient is bit-identical for every checkpoint interval."""
    mat = _channel(SHAPE)
    d = torch.tensor(_smooth_porosity(SHAPE, 4), dtype=torch.float32, device="cuda")
    base = adj.PorousChannel(mat, 0b001, TAU, G, STEPS, 10)
    Jb = base.forward(d)
    gb = base.backward()
    prob = adj.PorousChannel(mat, 0b001, TAU, G, STEPS, every)
    assert prob.forward(d) == Jb
    assert torch.equal(prob.backward(), gb)
    base.close()
    prob.close()


def test_autograd_function(adj):
    mat = _channel(SHAPE, interior_walls=False)
    prob = adj.PorousChannel(mat, 0b001, TAU, G, 40, 8)
    d = torch.tensor(_smooth_porosity(SHAPE, 5), dtype=torch.float32, device="cuda",
                     requires_grad=True)
    J = adj.porous_objective(d, prob)
    (3.0 * J).backward()
    ref = prob.backward()
    assert torch.allclose(d.grad, 3.0 * ref, rtol=1e-6, atol=0)
    assert J.item() == prob.forward(d)
    prob.close()


def test_autograd_after_another_forward_on_the_same_handle(adj):
    """Two objective evaluations on one handle before the first is
    differentiated (a line search does this): each node's gradient belongs to
    its own porosity, equal to a direct forward + backward at that porosity."""
    mat = _channel(SHAPE, interior_walls=False)
    prob = adj.PorousChannel(mat, 0b001, TAU, G, 30, 6)
    d1 = torch.tensor(_smooth_porosity(SHAPE, 6), dtype=torch.float32, device="cuda",
                      requires_grad=True)
    d2 = torch.tensor(_smooth_porosity(SHAPE, 7, lo=0.5), dtype=torch.float32, device="cuda",
                      requires_grad=True)
    J1 = adj.porous_objective(d1, prob)
    g0 = prob.generation()
    J2 = adj.porous_objective(d2, prob)
    assert prob.generation() == g0 + 1
    J1.backward()  # stale: the handle last ran d2
    J2.backward()
    direct = adj.PorousChannel(mat, 0b001, TAU, G, 30, 6)
    assert direct.forward(d1) == J1.item()
    r1 = direct.backward()
    assert direct.forward(d2) == J2.item()
    r2 = direct.backward()
    assert not torch.equal(r1, r2)
    assert torch.equal(d1.grad, r1)
    assert torch.equal(d2.grad, r2)
    prob.close()
    direct.close()


def test_porous_errors(adj):
    from paper_2307_11752_amd import _lib

    mat = _channel(SHAPE, interior_walls=False)
    prob = adj.PorousChannel(mat, 0b001, TAU, G, 10, 5)
    with pytest.raises(_lib.LBMError) as e:
        prob.backward()
    assert e.value.status == _lib.ERR_STATE
    prob.close()
    bad = mat.copy()
    bad[:, -1, :] = 3
    with pytest.raises(_lib.LBMError) as e:
        adj.PorousChannel(bad, 0b001, TAU, G, 10, 5)
    assert e.value.status == _lib.ERR_UNSUPPORTED
    with pytest.raises(_lib.LBMError) as e:
        adj.PorousChannel(mat, 0b001, TAU, G, 10, 11)
    assert e.value.status == _lib.ERR_ARG
