"""Pins of the FP64 oracle against facts fixed by the OpenLB 1.6 User Guide and by
mathematics -- never against the oracle itself.

Each test names the passage or the identity it checks.  Together they are chosen
so that a plausible slip anywhere in the oracle fails at least one of them:

* a wrong velocity, weight or opposite entry  -> guide listing, exact lattice
  isotropy identities, brute-force streaming path tracking;
* a dropped or mis-signed equilibrium term     -> exact moments of f^eq;
* a wrong Guo term or velocity shift           -> exact Guo moments, collision
  momentum change, Poiseuille exactness at the magic relaxation time;
* a wrong bounce-back slot or moving-wall sign -> path tracking, exact Couette
  profile, mass conservation of the lid-driven cavity;
* a wrong viscosity/relaxation relation        -> Poiseuille and Taylor-Green
  decay rate;
* a wrong periodic wrap                        -> path tracking, translation
  invariance, momentum conservation.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MAGIC_TAU = 0.5 + math.sqrt(3.0 / 16.0)


def _frac(x):
    return Fraction(x).limit_denominator(1000)


# ---------------------------------------------------------------------------
# Descriptor tables
# ---------------------------------------------------------------------------
def test_d2q9_matches_guide_listing(orc):
    """Core Concepts, section Descriptor: listing 'Definition of the D2Q9 descriptor'."""
    gold = json.load(open(os.path.join(GOLDEN, "d2q9_descriptor.json")))
    c, w, opp, cs2 = orc.descriptor(orc.D2Q9)
    assert c.shape[0] == gold["q"]
    assert [list(r[:2]) for r in c] == gold["c"]
    assert np.all(c[:, 2] == 0)
    assert list(opp) == gold["opposite"]
    assert [_frac(v) for v in w] == [Fraction(a, b) for a, b in gold["t"]]
    assert _frac(cs2) == Fraction(*gold["cs2"])
    assert list(c[1][:2]) == gold["api_examples"]["c1"]
    assert _frac(w[0]) == Fraction(*gold["api_examples"]["t0"])
    # weights are the correctly rounded doubles of the printed fractions
    for v, (a, b) in zip(w, gold["t"]):
        assert v == a / b


def test_d3q19_is_the_standard_set(orc):
    """D3Q19 is only drawn in the guide (Introduction, discrete velocity sets):
    brute-force the set {c in {-1,0,1}^3 : |c|^2 <= 2} and its weights by speed."""
    c, w, opp, cs2 = orc.descriptor(orc.D3Q19)
    expect = {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2}
    assert len(expect) == 19
    assert {tuple(r) for r in c} == expect
    by_speed = {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}
    for r, v in zip(c, w):
        assert _frac(v) == by_speed[int(np.dot(r, r))]
        assert v == float(by_speed[int(np.dot(r, r))])
    assert _frac(cs2) == Fraction(1, 3)
    # convention shared with the D2Q9 listing: opposite(i) = i + (q-1)/2
    assert list(opp[1:10]) == list(range(10, 19))


@pytest.mark.parametrize("d", [0, 1])
def test_lattice_isotropy_exact(orc, d):
    """Exact rational moment identities of the weights (the properties the
    second-order equilibrium relies on): sum w = 1, odd moments vanish,
    sum w c c = cs2 I, sum w c c c c = cs2^2 (dd + dd + dd)."""
    c, w, opp, cs2 = orc.descriptor(d)
    dim = 2 if d == 0 else 3
    W = [_frac(v) for v in w]
    cs2f = Fraction(1, 3)
    assert sum(W) == 1
    for a in range(dim):
        assert sum(Wi * ci[a] for Wi, ci in zip(W, c)) == 0
    for a, b in itertools.product(range(dim), repeat=2):
        assert sum(Wi * ci[a] * ci[b] for Wi, ci in zip(W, c)) == (cs2f if a == b else 0)
    for a, b, g in itertools.product(range(dim), repeat=3):
        assert sum(Wi * ci[a] * ci[b] * ci[g] for Wi, ci in zip(W, c)) == 0
    for a, b, g, e in itertools.product(range(dim), repeat=4):
        lhs = sum(Wi * ci[a] * ci[b] * ci[g] * ci[e] for Wi, ci in zip(W, c))
        rhs = cs2f * cs2f * ((a == b) * (g == e) + (a == g) * (b == e) + (a == e) * (b == g))
        assert lhs == rhs
    for i in range(len(w)):
        assert opp[opp[i]] == i
        assert np.all(c[opp[i]] == -c[i])


# ---------------------------------------------------------------------------
# Equilibrium, Guo source, collision
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [0, 1])
def test_equilibrium_moments(orc, d):
    """Second-order equilibrium: sum feq = rho, sum c feq = rho u,
    sum c c feq = rho cs2 I + rho u u (exact in real arithmetic)."""
    rng = np.random.default_rng(11 + d)
    c, w, opp, cs2 = orc.descriptor(d)
    dim = 2 if d == 0 else 3
    for _ in range(50):
        rho = rng.uniform(0.5, 1.5)
        u = np.zeros(3)
        u[:dim] = rng.uniform(-0.2, 0.2, dim)
        feq = orc.equilibrium(d, rho, u)
        assert abs(feq.sum() - rho) < 1e-14
        np.testing.assert_allclose(c.T @ feq, rho * u, atol=1e-15)
        P = np.einsum("ia,ib,i->ab", c, c, feq)
        expect = rho * cs2 * np.eye(3) + rho * np.outer(u, u)
        if dim == 2:
            expect[2, 2] = 0.0
        np.testing.assert_allclose(P, expect, atol=2e-15)


@pytest.mark.parametrize("d", [0, 1])
def test_guo_source_moments(orc, d):
    """Guo term (Simulation Models, coupling of momentum and energy equations):
    sum S = 0, sum c S = (1 - omega/2) F, sum c c S = (1 - omega/2)(F u + u F),
    with F = rho g."""
    rng = np.random.default_rng(23 + d)
    c, w, opp, cs2 = orc.descriptor(d)
    dim = 2 if d == 0 else 3
    for _ in range(50):
        omega = rng.uniform(0.5, 1.9)
        rho = rng.uniform(0.5, 1.5)
        u = np.zeros(3)
        g = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        g[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        S = orc.guo_source(d, omega, rho, u, g)
        F = rho * g
        k = 1.0 - omega / 2.0
        assert abs(S.sum()) < 1e-18
        np.testing.assert_allclose(c.T @ S, k * F, rtol=1e-12, atol=1e-19)
        P = np.einsum("ia,ib,i->ab", c, c, S)
        np.testing.assert_allclose(P, k * (np.outer(F, u) + np.outer(u, F)), atol=1e-18)


@pytest.mark.parametrize("d", [0, 1])
def test_collision_conserves_mass_and_adds_force(orc, d):
    """BGK + Guo on one cell: mass is unchanged and the momentum changes by
    exactly rho g (BGK relaxes towards the shifted velocity, Guo adds the rest)."""
    rng = np.random.default_rng(5 + d)
    c, w, opp, cs2 = orc.descriptor(d)
    dim = 2 if d == 0 else 3
    for _ in range(50):
        f = w * (1.0 + rng.uniform(-0.05, 0.05, len(w)))
        g = np.zeros(3)
        g[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        omega = rng.uniform(0.5, 1.9)
        fs, rho, u = orc.collide(d, omega, f, g)
        assert abs(fs.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(c.T @ fs - c.T @ f, rho * g, atol=2e-16)
        # the reported velocity is the shifted one, j/rho + g/2
        np.testing.assert_allclose(u, (c.T @ f) / rho + g / 2, atol=1e-16)


@pytest.mark.parametrize("d", [0, 1])
def test_collision_special_cases(orc, d):
    """omega = 1 without force lands exactly on feq; omega = 0 without force is the identity."""
    rng = np.random.default_rng(7)
    c, w, opp, cs2 = orc.descriptor(d)
    f = w * (1.0 + rng.uniform(-0.05, 0.05, len(w)))
    fs, rho, u = orc.collide(d, 1.0, f)
    np.testing.assert_allclose(fs, orc.equilibrium(d, f.sum(), (c.T @ f) / f.sum()), atol=1e-16)
    fs0, _, _ = orc.collide(d, 0.0, f)
    assert np.array_equal(fs0, f)


# ---------------------------------------------------------------------------
# Streaming, bounce-back, periodic wrap: brute-force path tracking
# ---------------------------------------------------------------------------
def _brute_force_stream(c, opp, mat, periodic, f0, nsteps):
    """Follow every population of every fluid cell for nsteps of pure streaming:
    it moves to x + c_i (wrapped on periodic axes) when that cell is fluid and
    reverses in place (halfway bounce-back) when it is a wall."""
    q = len(c)
    nz, ny, nx = mat.shape
    dims = (nx, ny, nz)
    out = np.zeros_like(f0)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if mat[z, y, x] != 1:
            continue
        for i in range(q):
            pos = [x, y, z]
            di = i
            for _ in range(nsteps):
                nxt = []
                for a in range(3):
                    v = pos[a] + c[di][a]
                    if periodic >> a & 1:
                        v %= dims[a]
                    nxt.append(v)
                if mat[nxt[2], nxt[1], nxt[0]] == 1:
                    pos = nxt
                else:
                    di = opp[di]
            out[di, pos[2], pos[1], pos[0]] = f0[i, z, y, x]
    return out


@pytest.mark.parametrize("d,shape,periodic", [
    (1, (4, 5, 6), 0b001),
    (1, (5, 4, 6), 0b101),
    (1, (3, 4, 5), 0b111),
    (0, (1, 6, 7), 0b01),
    (0, (1, 5, 6), 0b11),
])
@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_pure_streaming_is_the_tracked_permutation(orc, d, shape, periodic, nsteps):
    """Introduction section 1.1 streaming equation + halfway bounce-back:
    with omega = 0, g = 0, u_w = 0 the oracle must permute values exactly."""
    rng = np.random.default_rng(hash((d, shape, periodic, nsteps)) % 2**32)
    c, w, opp, cs2 = orc.descriptor(d)
    nz, ny, nx = shape
    mat = np.ones(shape, np.uint8)
    dims = (nx, ny, nz)
    for a in range(3 if d == 1 else 2):
        if not periodic >> a & 1:
            sl = [slice(None)] * 3
            sl[2 - a] = 0
            mat[tuple(sl)] = 2
            sl[2 - a] = dims[a] - 1
            mat[tuple(sl)] = 3 if a == 1 else 2
    # an interior obstacle cell
    inner = tuple(s // 2 for s in shape)
    mat[inner] = 2
    lat = orc.Lattice(d, mat, periodic, float("inf"))
    f0 = rng.uniform(0.0, 1.0, lat.f.shape)
    lat.set_populations(f0)
    lat.step(nsteps)
    expect = _brute_force_stream(c, opp, mat, periodic, f0, nsteps)
    fl = mat == 1
    assert np.array_equal(lat.f[:, fl], expect[:, fl])


def test_translation_invariance(orc):
    """A fully periodic lattice has no preferred origin: shifting the initial
    field by one cell along each axis shifts the result exactly."""
    rng = np.random.default_rng(3)
    shape = (4, 5, 6)
    mat = np.ones(shape, np.uint8)
    c, w, opp, cs2 = orc.descriptor(1)
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.05, 0.05, (19,) + shape))
    a = orc.Lattice(1, mat, 7, 0.7, g=[1e-4, -2e-4, 3e-4])
    b = orc.Lattice(1, mat, 7, 0.7, g=[1e-4, -2e-4, 3e-4])
    a.set_populations(f0)
    b.set_populations(np.roll(f0, (1, -2, 3), axis=(1, 2, 3)))
    a.step(7)
    b.step(7)
    assert np.array_equal(np.roll(a.f, (1, -2, 3), axis=(1, 2, 3)), b.f)


# ---------------------------------------------------------------------------
# Conservation laws
# ---------------------------------------------------------------------------
def test_periodic_momentum_conservation_and_force_growth(orc):
    """Fully periodic box: total mass is conserved; with g = 0 the momentum is
    conserved, with g != 0 it grows by exactly M g per step."""
    rng = np.random.default_rng(9)
    shape = (5, 6, 7)
    mat = np.ones(shape, np.uint8)
    c, w, opp, cs2 = orc.descriptor(1)
    f0 = w[:, None, None, None] * (1 + rng.uniform(-0.05, 0.05, (19,) + shape))
    lat = orc.Lattice(1, mat, 7, 0.8)
    lat.set_populations(f0)
    m0, j0, _ = lat.totals()
    lat.step(20)
    m1, j1, _ = lat.totals()
    assert abs(m1 - m0) < 1e-12 * m0
    np.testing.assert_allclose(j1, j0, atol=1e-12)
    g = np.array([1e-4, -3e-5, 2e-5])
    lat = orc.Lattice(1, mat, 7, 0.8, g=g)
    lat.set_populations(f0)
    for _ in range(5):
        m0, j0, _ = lat.totals()
        lat.step(1)
        m1, j1, _ = lat.totals()
        assert abs(m1 - m0) < 1e-12 * m0
        np.testing.assert_allclose(j1 - j0, m0 * g, rtol=1e-9, atol=1e-16)


def test_cavity_mass_conservation_and_mirror_symmetry(orc):
    """Lid-driven cavity (config shape 16x16 here): halfway bounce-back walls and a
    full-row moving lid conserve mass; mirroring x together with the lid velocity
    mirrors the flow (u_x flips sign)."""
    n = 16
    mat = np.full((1, n, n), 2, np.uint8)
    mat[0, 1:-1, 1:-1] = 1
    mat[0, -1, :] = 3
    a = orc.Lattice(0, mat, 0, 0.6, u_wall=[0.05, 0, 0])
    b = orc.Lattice(0, mat, 0, 0.6, u_wall=[-0.05, 0, 0])
    a.init_equilibrium()
    b.init_equilibrium()
    m0 = a.totals()[0]
    a.step(300)
    b.step(300)
    assert abs(a.totals()[0] - m0) < 1e-12 * m0
    ra, ua = a.moments()
    rb, ub = b.moments()
    np.testing.assert_allclose(rb, ra[:, :, ::-1], atol=1e-14)
    np.testing.assert_allclose(ub[0], -ua[0][:, :, ::-1], atol=1e-14)
    np.testing.assert_allclose(ub[1], ua[1][:, :, ::-1], atol=1e-14)
    assert np.max(np.abs(ua[0])) > 1e-3  # the lid actually drives a flow


# ---------------------------------------------------------------------------
# Closed-form flows
# ---------------------------------------------------------------------------
def _channel(d, H, nx=3, nz=3, top=2):
    if d == 0:
        mat = np.ones((1, H + 2, nx), np.uint8)
        per = 0b01
    else:
        mat = np.ones((nz, H + 2, nx), np.uint8)
        per = 0b101
    mat[:, 0, :] = 2
    mat[:, -1, :] = top
    return mat, per


def _run_to_steady(lat, tol, chunk=200, maxit=2000):
    prev = None
    for _ in range(maxit):
        lat.step(chunk)
        ux = lat.moments()[1][0, 0, 1:-1, 1]
        if prev is not None and np.max(np.abs(ux - prev)) < tol * np.max(np.abs(ux)):
            return ux
        prev = ux
    raise AssertionError("no steady state")


@pytest.mark.parametrize("d", [0, 1])
def test_poiseuille_exact_at_magic_tau(orc, d):
    """Force-driven channel, halfway bounce-back walls, Guo forcing: at
    tau = 1/2 + sqrt(3/16) the steady BGK solution is the exact parabola
    u(s) = g s (H - s) / (2 nu), nu = cs2 (tau - 1/2), s = j - 1/2.  The centre-line
    speed obeys the guide's poiseuille2d force relation F = 8 nu u_c / Ly^2."""
    gold = json.load(open(os.path.join(GOLDEN, "poiseuille_force.json")))
    H = 9
    nu = (MAGIC_TAU - 0.5) / 3.0
    uc = 1e-3
    g = gold["force_over_nu_uc_times_Ly2"] * nu * uc / H**2
    mat, per = _channel(d, H)
    lat = orc.Lattice(d, mat, per, MAGIC_TAU, g=[g, 0, 0])
    lat.init_equilibrium()
    ux = _run_to_steady(lat, 1e-13)
    s = np.arange(1, H + 1) - 0.5
    ana = g / (2 * nu) * s * (H - s)
    np.testing.assert_allclose(ux, ana, rtol=0, atol=1e-12 * uc)
    assert abs(ux[H // 2] - uc) < 1e-12 * uc
    u = lat.moments()[1]
    assert np.max(np.abs(u[1:])) < 1e-11 * uc


def test_poiseuille_eoc_is_second_order(orc):
    """Guide example poiseuille2dEOC set-up (tau = 0.8, N = 21, 31, 41, 51, residual
    1e-5 stop criterion replaced by a tighter one) and the EOC definition of the
    particle chapter: the relative L2 velocity error converges with order ~2."""
    errs = []
    Hs = (21, 31, 41, 51)
    for H in Hs:
        nu = 0.3 / 3.0
        g = 8 * nu * 0.01 / H**2
        mat, per = _channel(0, H)
        lat = orc.Lattice(0, mat, per, 0.8, g=[g, 0, 0])
        lat.init_equilibrium()
        ux = _run_to_steady(lat, 1e-10)
        s = np.arange(1, H + 1) - 0.5
        ana = g / (2 * nu) * s * (H - s)
        errs.append(np.linalg.norm(ux - ana) / np.linalg.norm(ana))
    for i in range(len(Hs) - 1):
        eoc = math.log(errs[i] / errs[i + 1]) / math.log(Hs[i + 1] / Hs[i])
        assert 1.9 < eoc < 2.1, (Hs[i], eoc, errs)


@pytest.mark.parametrize("d", [0, 1])
@pytest.mark.parametrize("tau", [0.6, 1.3])
def test_couette_exact(orc, d, tau):
    """Moving-wall bounce-back on top, resting wall below, periodic along x:
    the steady state is the exact linear profile u(s) = u_w s / H for any tau."""
    H = 8
    uw = 0.01
    mat, per = _channel(d, H, top=3)
    lat = orc.Lattice(d, mat, per, tau, u_wall=[uw, 0, 0])
    lat.init_equilibrium()
    ux = _run_to_steady(lat, 1e-13)
    s = np.arange(1, H + 1) - 0.5
    np.testing.assert_allclose(ux, uw * s / H, rtol=0, atol=1e-12 * uw)


def _tgv_deviation(orc, n, tau, u0, steps):
    mat = np.ones((1, n, n), np.uint8)
    k = 2 * np.pi / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = np.zeros((2, 1, n, n))
    u[0, 0] = -u0 * np.cos(k * x) * np.sin(k * y)
    u[1, 0] = u0 * np.sin(k * x) * np.cos(k * y)
    lat = orc.Lattice(0, mat, 0b11, tau)
    lat.init_equilibrium(u=u)
    nu = (tau - 0.5) / 3.0
    ke0 = 0.5 * np.sum(u**2)
    lat.step(steps)
    rho, uu = lat.moments()
    ke = 0.5 * np.sum(rho * np.sum(uu**2, axis=0))
    return ke / ke0 / math.exp(-2 * nu * 2 * k * k * steps) - 1.0


def test_taylor_green_decay_converges(orc):
    """Periodic 2D Taylor-Green vortex (tgv3d example is its 3D relative): the
    kinetic energy decays as exp(-2 nu |k|^2 t) with nu = cs2 (tau - 1/2); the
    deviation shrinks with second order in the resolution."""
    e32 = _tgv_deviation(orc, 32, 0.8, 1e-3, 400)
    e64 = _tgv_deviation(orc, 64, 0.8, 1e-3, 1600)
    assert abs(e64) < 5e-3
    assert 3.0 < e32 / e64 < 5.0, (e32, e64)


# ---------------------------------------------------------------------------
# Geometry validation and statistics
# ---------------------------------------------------------------------------
def test_geometry_check(orc):
    """Material numbers 0..5 (Geometry chapter, Setting Material Numbers): fluid
    next to material 0 or next to a non-periodic domain edge is rejected, and
    pressure (4) / curved (5) boundaries are not supported on this path."""
    mat = np.full((1, 6, 6), 2, np.uint8)
    mat[0, 1:-1, 1:-1] = 1
    assert orc.check_geometry(0, mat, 0) == orc.OK
    bad = mat.copy()
    bad[0, 0, 3] = 0
    assert orc.check_geometry(0, bad, 0) == orc.ERR_GEOMETRY
    edge = np.ones((1, 6, 6), np.uint8)
    assert orc.check_geometry(0, edge, 0b01) == orc.ERR_GEOMETRY
    assert orc.check_geometry(0, edge, 0b11) == orc.OK
    for m in (4, 5, 7):
        bad = mat.copy()
        bad[0, 0, 0] = m
        assert orc.check_geometry(0, bad, 0) == orc.ERR_UNSUPPORTED
    assert orc.check_geometry(0, np.ones((2, 4, 4), np.uint8), 7) == orc.ERR_ARG


def test_statistics_definitions(orc):
    """Lesson 'Extract Data From a Simulation': average density, average energy
    (half the mean squared velocity) and maximum velocity norm over fluid cells."""
    rng = np.random.default_rng(1)
    n = 6
    mat = np.ones((1, n, n), np.uint8)
    lat = orc.Lattice(0, mat, 0b11, 0.9)
    rho = rng.uniform(0.9, 1.1, (1, n, n))
    u = rng.uniform(-0.05, 0.05, (2, 1, n, n))
    lat.init_equilibrium(rho=rho, u=u)
    m, j, s = lat.totals()
    assert abs(s[0] - rho.mean()) < 1e-14
    assert abs(s[1] - 0.5 * np.mean(np.sum(u**2, axis=0))) < 1e-14
    assert abs(s[2] - np.max(np.sqrt(np.sum(u**2, axis=0)))) < 1e-14
    np.testing.assert_allclose(j[:2], np.sum(rho * u, axis=(1, 2, 3)), atol=1e-13)


# ---------------------------------------------------------------------------
# Porous BGK (Simulation Models, "Porous Media Model") and its FP64 adjoint
# ---------------------------------------------------------------------------
def test_porous_step_with_unit_porosity_is_the_plain_step(orc):
    """d = 1 means pure fluid: the porous step must equal the plain BGK + Guo
    step bit for bit (walls, periodic x, body force)."""
    sh = (4, 5, 6)
    mat = np.ones(sh, np.uint8)
    mat[:, 0, :] = 2
    mat[:, -1, :] = 2
    g = [1e-4, 2e-5, -3e-5]
    rng = np.random.default_rng(0)
    lat = orc.Lattice(1, mat, 0b101, 0.7, g=g)
    lat.init_equilibrium(None, rng.uniform(-0.05, 0.05, (3,) + sh))
    f0 = lat.f.copy()
    prob = orc.PorousProblem(1, mat, 0b101, 0.7, g)
    _, fT = prob.forward(np.ones(sh), 6, f0=f0)
    lat.step(6)
    assert np.array_equal(fT[:, mat == 1], lat.f[:, mat == 1])


@pytest.mark.parametrize("K", [0.05, 0.2, 2.0])
def test_porous_darcy_law_with_guide_permeability(orc, K):
    """The guide's discrete porosity of a permeability K is
    d = 1 - h^(dim-1) nu tau / K (lattice units, h = 1).  In a periodic box with
    uniform d and body acceleration g the porous step reaches the uniform
    steady velocity u = g / (omega (1 - d)) = K g / nu: Darcy's law."""
    tau = 0.7
    nu = (tau - 0.5) / 3.0
    d = 1.0 - nu * tau / K
    assert 0.0 <= d < 1.0
    g = 1e-6
    mat = np.ones((2, 3, 4), np.uint8)
    prob = orc.PorousProblem(1, mat, 7, tau, [g, 0, 0])
    J, fT = prob.forward(np.full(mat.shape, d), 4000)
    assert abs(J / (K * g / nu) - 1.0) < 1e-9


def test_porous_adjoint_matches_central_differences(orc):
    """The FP64 discrete adjoint gradient of the outlet-plane mean velocity
    with respect to the porosity of single cells equals the central difference
    quotient of the FP64 forward model (the guide's difference-quotient
    derivative option) to the difference quotient's own accuracy."""
    sh = (5, 6, 8)
    mat = np.ones(sh, np.uint8)
    mat[:, 0, :] = 2
    mat[:, -1, :] = 2
    mat[0, :, :] = 2
    mat[-1, :, :] = 2
    rng = np.random.default_rng(1)
    por = rng.uniform(0.3, 1.0, sh)
    prob = orc.PorousProblem(1, mat, 0b001, 0.7, [1e-4, 0, 0])
    J, grad = prob.gradient(por, 40)
    J2, _ = prob.forward(por, 40)
    assert J == J2
    assert np.all(grad[mat != 1] == 0.0)
    fluid = np.argwhere(mat == 1)
    for c in fluid[rng.choice(len(fluid), 8, replace=False)]:
        c = tuple(c)
        h = 1e-4
        pp = por.copy()
        pp[c] += h
        pm = por.copy()
        pm[c] -= h
        fd = (prob.forward(pp, 40)[0] - prob.forward(pm, 40)[0]) / (2 * h)
        assert abs(grad[c] - fd) <= 1e-6 * abs(fd), (c, grad[c], fd)
