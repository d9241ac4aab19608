"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

The paper names the schemes (Sec. 3.1: the energy-conserving Piacsek-Williams
scheme for momentum, Leonard's positivity-preserving ULTIMATE scheme for
scalars) but prints no formulas or values, so every pin here is a hand-derived
worked example, a closed form, an invariant of the discretisation, or a special
case that reduces to a textbook result.  Each is chosen so that a dropped term,
a wrong sign, a wrong index or a swapped operand in the oracle fails one of
them.
"""
import os

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_12850_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows[key] = np.array([float(x) for x in vals])
    return rows


def unit_geometry(nx, ny, nz, dx=1.0, dy=1.0):
    """Uniform unit spacing, constant density: the textbook special case."""
    one = np.ones(nz)
    zf = np.arange(1, nz + 1, dtype=float)
    return I.Geometry(nx, ny, nz, dx, dy, one.copy(), one.copy(), one.copy(), zf,
                      zf - 0.5)


def filled(*arrs):
    return [O.halo_fill(I.pad(np.ascontiguousarray(a, dtype=np.float64))) for a in arrs]


def random_state(nx=8, ny=6, nz=7, nscal=2, seed=11, dx=50.0, dy=40.0):
    g = I.make_geometry(nx, ny, nz, dx=dx, dy=dy)
    f = I.make_fields(g, nscal, seed)
    names = ["u", "v", "w"] + I.scalar_names(nscal)
    return g, filled(*[f[n] for n in names])


# ---------------------------------------------------------------------------
# Hand-derived worked examples (tests/golden)
# ---------------------------------------------------------------------------
def test_pw_1d_worked_example():
    gold = read_golden("pw_1d_burgers.txt")
    g = unit_geometry(4, 1, 2)
    u = np.repeat(gold["u"][:, None, None], 2, axis=2)
    U, V, W = filled(u, np.zeros_like(u), np.zeros_like(u))
    su, sv, sw = O.pw(U, V, W, g)
    for k in range(2):
        np.testing.assert_array_equal(I.interior(su)[:, 0, k], gold["su"])
    assert np.all(I.interior(sv) == 0) and np.all(I.interior(sw) == 0)


def test_tvd_1d_worked_example_faces_and_tendency():
    gold = read_golden("tvd_1d_ultimate.txt")
    phi = gold["phi"]
    faces = [O.ultimate_face(phi[i - 1], phi[i], phi[(i + 1) % 6], 0.5) for i in range(6)]
    np.testing.assert_array_equal(faces, gold["face"])
    g = unit_geometry(6, 1, 2)
    p = np.repeat(phi[:, None, None], 2, axis=2)
    one = np.ones_like(p)
    U, V, W, P = filled(one, 0 * one, 0 * one, p)
    s = O.tvd(U, V, W, P, g, 0.5)
    for k in range(2):
        np.testing.assert_array_equal(I.interior(s)[:, 0, k], gold["s"])
    nxt = phi + 0.5 * gold["s"]
    np.testing.assert_array_equal(nxt, gold["phi_next"])
    assert nxt.sum() == phi.sum() and nxt.min() >= 1 and nxt.max() <= 5


# ---------------------------------------------------------------------------
# I1: a fluid at rest has no advection tendency
# ---------------------------------------------------------------------------
def test_resting_fluid_gives_zero():
    g, st = random_state()
    z = np.zeros_like(I.interior(st[0]))
    U, V, W = filled(z, z, z)
    su, sv, sw = O.pw(U, V, W, g)
    for s in (su, sv, sw):
        assert np.all(I.interior(s) == 0.0)
    for phi in st[3:]:
        assert np.all(I.interior(O.tvd(U, V, W, phi, g, 0.5)) == 0.0)


# ---------------------------------------------------------------------------
# I3/I4: conservation and the kinetic-energy identity, for ANY flow
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_conservation_and_energy_identity_any_flow(seed):
    g, st = random_state(seed=seed)
    u, v, w = st[:3]
    su, sv, sw = O.pw(u, v, w, g)
    sph = [O.tvd(u, v, w, p, g, 0.5) for p in st[3:]]
    b, sc = O.budgets(u, v, w, su, sv, sw, st[3:], sph, g)
    # flux form + periodic sides + closed lid: momentum is conserved
    assert abs(b["C_u"]) <= 1e-14 * sc["C_u"]
    assert abs(b["C_v"]) <= 1e-14 * sc["C_v"]
    # w-cells exchange momentum with the half-cells next to the ground and lid
    assert abs(b["C_w"] - b["C_w_closed"]) <= 1e-14 * sc["C_w"]
    # summation by parts: sum u.su equals minus the KE times the mass divergence
    for comp in "uvw":
        p, q = b[f"P_{comp}"], b[f"Q_{comp}"]
        assert abs(p - q) <= 1e-13 * (sc[f"P_{comp}"] + sc[f"Q_{comp}"]), comp
    # scalar mass: sum rhon dz s = 0
    for n, p in enumerate(st[3:]):
        scale = np.sum(np.abs(I.interior(sph[n])) * g.rhon / g.rdz)
        assert abs(b[f"C_s{n}"]) <= 1e-14 * scale


def test_energy_identity_is_not_trivially_zero():
    """The identity pins something: P is far from zero for a divergent flow."""
    g, st = random_state(seed=5)
    su, sv, sw = O.pw(*st[:3], g)
    b, sc = O.budgets(*st[:3], su, sv, sw, [], [], g)
    for comp in "uvw":
        assert abs(b[f"P_{comp}"]) > 1e-3 * sc[f"P_{comp}"]


# ---------------------------------------------------------------------------
# I2/I5: non-divergent flow keeps a uniform scalar uniform and does no work
# ---------------------------------------------------------------------------
def test_divergence_free_flow_preserves_uniform_scalar_and_energy():
    g = I.make_geometry(10, 8, 9, dx=50.0, dy=40.0)
    vel = I.make_divfree_velocity(g, seed=3)
    u, v, w = filled(vel["u"], vel["v"], vel["w"])
    d = I.interior(O.divergence(u, v, w, g))
    umax = max(np.abs(vel[c]).max() for c in "uvw")
    assert np.abs(d).max() <= 1e-14 * umax / 40.0
    phi = filled(np.full_like(vel["u"], 300.0))[0]
    s = I.interior(O.tvd(u, v, w, phi, g, 0.5))
    assert np.abs(s).max() <= 1e-13 * 300.0 * umax / 40.0
    su, sv, sw = O.pw(u, v, w, g)
    b, sc = O.budgets(u, v, w, su, sv, sw, [], [], g)
    for comp in "uvw":
        assert abs(b[f"P_{comp}"]) <= 1e-13 * sc[f"P_{comp}"]


# ---------------------------------------------------------------------------
# I6: translation invariance (bitwise)
# ---------------------------------------------------------------------------
def test_translation_invariance_bitwise():
    g, st = random_state(seed=21)
    inner = [I.interior(a).copy() for a in st]
    rolled = filled(*[np.roll(a, (3, -2), axis=(0, 1)) for a in inner])
    a0 = O.pw(*st[:3], g)
    a1 = O.pw(*rolled[:3], g)
    for x, y in zip(a0, a1):
        np.testing.assert_array_equal(np.roll(I.interior(x), (3, -2), axis=(0, 1)),
                                      I.interior(y))
    t0 = O.tvd(*st[:3], st[3], g, 0.5)
    t1 = O.tvd(*rolled[:3], rolled[3], g, 0.5)
    np.testing.assert_array_equal(np.roll(I.interior(t0), (3, -2), axis=(0, 1)),
                                  I.interior(t1))


# ---------------------------------------------------------------------------
# x <-> y mirror: swapping the horizontal axes (u <-> v, dx <-> dy) swaps
# su and sv and transposes everything else.  Pins sv against su.
# ---------------------------------------------------------------------------
def test_xy_transpose_symmetry():
    g, st = random_state(nx=7, ny=9, seed=31, dx=50.0, dy=35.0)
    inner = [I.interior(a) for a in st]
    T = lambda a: np.ascontiguousarray(np.transpose(a, (1, 0, 2)))
    gt = I.Geometry(g.ny, g.nx, g.nz, g.dy, g.dx, g.rdz, g.rho, g.rhon, g.z_face,
                    g.z_centre)
    tr = filled(T(inner[1]), T(inner[0]), T(inner[2]), T(inner[3]))
    su, sv, sw = O.pw(*st[:3], g)
    su2, sv2, sw2 = O.pw(*tr[:3], gt)
    tol = dict(rtol=0, atol=1e-14 * np.abs(I.interior(su)).max())
    np.testing.assert_allclose(T(I.interior(sv)), I.interior(su2), **tol)
    np.testing.assert_allclose(T(I.interior(su)), I.interior(sv2), **tol)
    np.testing.assert_allclose(T(I.interior(sw)), I.interior(sw2), **tol)
    s = O.tvd(*st[:3], st[3], g, 0.5)
    s2 = O.tvd(*tr[:3], tr[3], gt, 0.5)
    np.testing.assert_allclose(T(I.interior(s)), I.interior(s2), rtol=0,
                               atol=1e-13 * np.abs(I.interior(s)).max())


# ---------------------------------------------------------------------------
# I7: affine equivariance and homogeneity of the TVD scheme
# ---------------------------------------------------------------------------
def test_tvd_affine_and_homogeneous():
    g, st = random_state(seed=41)
    u, v, w, th = st[:4]
    s = I.interior(O.tvd(u, v, w, th, g, 0.5))
    d = I.interior(O.divergence(u, v, w, g))
    inner = I.interior(th)
    for const in (250.0, -17.0):
        s_shift = I.interior(O.tvd(u, v, w, filled(inner + const)[0], g, 0.5))
        expect = s - const * d / g.rhon[None, None, :]
        np.testing.assert_allclose(s_shift, expect, rtol=0,
                                   atol=1e-12 * np.abs(s).max())
    for lam in (3.0, -2.5):
        s_scaled = I.interior(O.tvd(u, v, w, filled(lam * inner)[0], g, 0.5))
        np.testing.assert_allclose(s_scaled, lam * s, rtol=0,
                                   atol=1e-13 * abs(lam) * np.abs(s).max())


# ---------------------------------------------------------------------------
# 1-D special cases along each axis
# ---------------------------------------------------------------------------
def line_case(axis, profile, speed, n=16):
    """Put a 1-D profile along one axis with a constant speed on every face."""
    shape = [4, 4, 4]
    shape[axis] = n
    g = unit_geometry(*shape)
    idx = [None, None, None]
    idx[axis] = slice(None)
    phi = np.broadcast_to(profile[tuple(idx)], shape).copy()
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis][...] = speed
    if axis == 2:
        vel[2][:, :, n - 1] = 0.0  # lid
    U, V, W, P = filled(*vel, phi)
    return g, U, V, W, P


def take_line(a, axis):
    a = I.interior(a)
    sl = [1, 1, 1]
    sl[axis] = slice(None)
    return a[tuple(sl)]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_courant_one_is_an_exact_shift(axis):
    """I8: at c = 1 every face takes the upwind value, so a step is a shift."""
    n = 16
    rng = np.random.default_rng(axis)
    prof = rng.uniform(0.0, 1.0, n)
    g, U, V, W, P = line_case(axis, prof, 2.0, n)
    s = take_line(O.tvd(U, V, W, P, g, 0.5), axis)  # c = 2 * 0.5 / 1 = 1
    nxt = prof + 0.5 * s
    inner = slice(2, n - 2)
    np.testing.assert_array_equal(nxt[inner], np.roll(prof, 1)[inner])


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("c", [0.25, 0.6])
def test_quickest_is_exact_for_quadratics(axis, c):
    """I9: in a monotone region the limiter is idle and QUICKEST's face value
    is the exact swept average of a quadratic, so one step reproduces the
    exactly translated cell averages."""
    n = 16
    x = np.arange(n + 1, dtype=float)
    Q = lambda t: 0.5 * t ** 2 + 0.004 * t ** 3 / 3.0  # primitive of t + 0.004 t^2
    avg = lambda lo, hi: (Q(hi) - Q(lo)) / (hi - lo)
    prof = avg(x[:-1], x[1:]) + 3.0
    dt = 0.5
    speed = c / dt
    g, U, V, W, P = line_case(axis, prof, speed, n)
    s = take_line(O.tvd(U, V, W, P, g, dt), axis)
    nxt = prof + dt * s
    exact = avg(x[:-1] - c, x[1:] - c) + 3.0
    inner = slice(3, n - 3)
    np.testing.assert_allclose(nxt[inner], exact[inner], rtol=0, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_directions_agree(axis):
    """The same 1-D problem gives the same interior tendency along x, y, z."""
    n = 16
    rng = np.random.default_rng(7)
    prof = rng.uniform(0.0, 2.0, n)
    ref_g, *ref = line_case(0, prof, 1.3, n)
    s_ref = take_line(O.tvd(*ref, ref_g, 0.4), 0)
    g, U, V, W, P = line_case(axis, prof, 1.3, n)
    s = take_line(O.tvd(U, V, W, P, g, 0.4), axis)
    inner = slice(2, n - 2)
    np.testing.assert_allclose(s[inner], s_ref[inner], rtol=0, atol=1e-14)


def test_boundedness_random_1d():
    """I10: constant speed, 0 < c <= 1, periodic: each new value lies between
    the old values of the cell and its upwind neighbour, so q >= 0 stays >= 0."""
    rng = np.random.default_rng(2024)
    worst = 0.0
    for trial in range(300):
        n = 12
        prof = rng.uniform(0.0, 1.0, n) ** rng.uniform(0.5, 4.0)
        c = rng.uniform(0.01, 1.0)
        sign = 1.0 if trial % 2 == 0 else -1.0
        g, U, V, W, P = line_case(0, prof, sign * c, n)
        s = take_line(O.tvd(U, V, W, P, g, 1.0), 0)
        nxt = prof + s
        up = np.roll(prof, 1) if sign > 0 else np.roll(prof, -1)
        lo, hi = np.minimum(prof, up), np.maximum(prof, up)
        viol = np.maximum(lo - nxt, nxt - hi).max()
        worst = max(worst, viol)
    assert worst <= 4e-16


def test_limiter_is_continuous_at_branch_switch():
    """I12: the branches agree where |kappa| = |delta|, so round-off can never
    flip a face value by an O(1) amount.  The face value is Lipschitz in phiC
    with constant at most 1 + 1/c (the slope of the ULTIMATE bound)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        phiU, phiD = rng.uniform(-1, 1, 2)
        c = rng.uniform(0.0, 1.0)
        for phiC in (phiU, phiD):  # the two ends of the monotone range
            for eps in (1e-12, -1e-12):
                a = O.ultimate_face(phiU, phiC + eps, phiD, c)
                b = O.ultimate_face(phiU, phiC, phiD, c)
                assert abs(a - b) <= 1.01 * (1.0 + 1.0 / c) * abs(eps) + 1e-15


def test_ultimate_face_reduces_to_parabola_when_unlimited():
    """Inside the bounds and as c -> 0 the face value is the value at the face
    of the parabola whose averages over the cells U, C, D are phiU, phiC, phiD:
    (-phiU + 5 phiC + 2 phiD)/6 (cell averages, not point values)."""
    v = O.ultimate_face(1.0, 2.0, 3.2, 1e-9)
    assert abs(v - (-1.0 + 5 * 2.0 + 2 * 3.2) / 6.0) < 1e-8
    # the same parabola, built by hand: p(x) = a x^2 + b x + c0 with averages
    # over [-2,-1], [-1,0], [0,1] equal to 1.0, 2.0, 3.2; face at x = 0... the
    # downwind cell is [0,1] so the C/D face is x = 0.
    A = np.array([[7 / 3, -1.5, 1.0], [1 / 3, -0.5, 1.0], [1 / 3, 0.5, 1.0]])
    a, b, c0 = np.linalg.solve(A, [1.0, 2.0, 3.2])
    assert abs(v - c0) < 1e-8


def test_courant_above_one_is_an_error():
    g, st = random_state(seed=3)
    fast = filled(I.interior(st[0]) * 40.0)[0]  # |u| dt/dx > 1
    with pytest.raises(O.CourantError):
        O.tvd(fast, st[1], st[2], st[3], g, 0.5)


# ---------------------------------------------------------------------------
# Step: mass conservation over many steps, positivity, textbook reduction
# ---------------------------------------------------------------------------
def test_step_conserves_scalar_mass_and_positivity():
    g = I.make_geometry(8, 8, 10)
    f = I.make_fields(g, 2, seed=9)
    st = [I.pad(f[n]) for n in ["u", "v", "w", "th", "q1"]]
    w_dz = (g.rhon / g.rdz)[None, None, :]
    m0 = [np.sum(I.interior(a) * w_dz) for a in st[3:]]
    for _ in range(20):
        st = O.step(st, g, 0.5)
    m1 = [np.sum(I.interior(a) * w_dz) for a in st[3:]]
    for a, b in zip(m0, m1):
        assert abs(a - b) <= 1e-13 * abs(a)
    assert I.interior(st[4]).min() > 0.0
    assert np.all(I.interior(st[2])[:, :, -1] == 0.0)


def test_pw_textbook_form_on_uniform_grid():
    """I11: with constant density and uniform dz the mass-weighted averages in
    sw become plain averages: the textbook C-grid flux form."""
    nx, ny, nz = 5, 4, 6
    g = unit_geometry(nx, ny, nz, dx=2.0, dy=3.0)
    rng = np.random.default_rng(1)
    u, v, w = (rng.standard_normal((nx, ny, nz)) for _ in range(3))
    w[:, :, -1] = 0
    U, V, W = filled(u, v, w)
    _, _, sw = O.pw(U, V, W, g)
    r = lambda a, s, ax: np.roll(a, -s, axis=ax)
    wz = np.concatenate([np.zeros((nx, ny, 1)), w, np.zeros((nx, ny, 1))], axis=2)
    wc, wp, wm = wz[:, :, 1:-1], wz[:, :, 2:], wz[:, :, :-2]
    uk = 0.5 * (u + np.concatenate([u[:, :, 1:], u[:, :, -1:]], axis=2))
    vk = 0.5 * (v + np.concatenate([v[:, :, 1:], v[:, :, -1:]], axis=2))
    fx = uk * (wc + r(wc, 1, 0))
    fy = vk * (wc + r(wc, 1, 1))
    fz = (wc + wp) ** 2
    ex = -((fx - r(fx, -1, 0)) / (2 * 2.0) + (fy - r(fy, -1, 1)) / (2 * 3.0)
           + ((wc + wp) ** 2 - (wm + wc) ** 2) / 4.0)
    got = I.interior(sw)[:, :, :-1]
    np.testing.assert_allclose(got, ex[:, :, :-1], rtol=0, atol=1e-13)
    assert np.all(I.interior(sw)[:, :, -1] == 0)
    del fz


def test_generator_is_seeded_and_sane():
    g = I.make_geometry(32, 32, 32)
    a = I.make_fields(g, 2, seed=1)
    b = I.make_fields(g, 2, seed=1)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    assert np.all(a["w"][:, :, -1] == 0)
    assert a["q1"].min() > 0
    assert abs(a["th"].mean() - 300.0) < 2.0
    assert np.abs(a["u"]).max() < 5.5
    assert np.isclose(np.sum(1.0 / g.rdz), 3000.0)
