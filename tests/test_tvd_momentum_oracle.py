"""Pins of the oracle's TVD advection of momentum (the ULTIMATE scheme of
Sec. 3.1 applied to u, v, w on their C-grid control volumes), CPU only.

None of these retypes the oracle's formula.  Each ties it to something fixed
elsewhere:
* with the centred mean as face value the scheme is the pinned PW scheme
  (mass fluxes, indices, signs, geometry and the ground/lid treatment);
* fields that do not vary along x (y) make su (sv) the pinned scalar TVD
  source term of u (v) as a scalar (the y and z fluxes with their limiter,
  Courant numbers and boundary rules);
* piecewise-constant profiles make every limited face value the upwind one, so
  the scheme is donor cell (upwind choice, incl. next to ground and lid);
* quadratic profiles with the limiter inactive give the QUICKEST face values of
  Leonard (1979) (the Courant numbers of the w faces);
* mirror symmetry in x and, on a uniform column, in z (the negative-flux
  branches and the lid against the ground);
* conservation of u and v momentum, and a uniform u in any flow.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_12850_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def interior(a):
    return a[2:-2, 2:-2, :]


def flow(nx, ny, nz, seed, amp=5.0):
    g = I.make_geometry(nx, ny, nz, 50.0, 50.0)
    f = I.make_fields(g, 0, seed, amp=amp, padded=True)
    return g, [f[n] for n in ("u", "v", "w")]


def padded(a):
    return I.pad(np.ascontiguousarray(a))


def uniform_geometry(nx, ny, nz, dz=40.0, dx=50.0, dy=50.0):
    zf = dz * np.arange(1, nz + 1, dtype=np.float64)
    return I.Geometry(nx, ny, nz, dx, dy, np.full(nz, 1.0 / dz), np.ones(nz), np.ones(nz),
                      zf, zf - dz / 2)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("seed", [0, 1])
def test_centred_face_value_is_pw(seed):
    g, (u, v, w) = flow(12, 10, 16, seed)
    su, sv, sw, _ = O.tvd_momentum(u, v, w, g, 0.5, centred=True)
    hu, hv, hw = (O.halo_fill(x) for x in (u, v, w))
    pu, pv, pw_ = O.pw(hu, hv, hw, g)
    for got, ref in ((su, pu), (sv, pv), (sw, pw_)):
        assert rel(interior(got), interior(ref)) <= 1e-13


def test_limited_differs_from_centred():
    # guards the pins above: the limiter must change the answer
    g, (u, v, w) = flow(12, 10, 16, 2)
    lim = O.tvd_momentum(u, v, w, g, 0.5)
    cen = O.tvd_momentum(u, v, w, g, 0.5, centred=True)
    for f in range(3):
        assert rel(interior(lim[f]), interior(cen[f])) > 1e-3


@pytest.mark.parametrize("seed", [3, 4])
def test_x_independent_fields_give_scalar_tvd_of_u(seed):
    g, (u, v, w) = flow(6, 10, 16, seed, amp=10.0)
    col = lambda a: padded(np.repeat(interior(a)[:1], g.nx, 0))
    u, v, w = col(u), col(v), col(w)
    w[:, :, -1] = 0.0
    su, _, _, _ = O.tvd_momentum(u, v, w, g, 2.0)
    hu, hv, hw = (O.halo_fill(x) for x in (u, v, w))
    ref = O.tvd(hu, hv, hw, hu, g, 2.0)
    assert rel(interior(su), interior(ref)) <= 1e-14


@pytest.mark.parametrize("seed", [5, 6])
def test_y_independent_fields_give_scalar_tvd_of_v(seed):
    g, (u, v, w) = flow(10, 6, 16, seed, amp=10.0)
    row = lambda a: padded(np.repeat(interior(a)[:, :1], g.ny, 1))
    u, v, w = row(u), row(v), row(w)
    w[:, :, -1] = 0.0
    _, sv, _, _ = O.tvd_momentum(u, v, w, g, 2.0)
    hu, hv, hw = (O.halo_fill(x) for x in (u, v, w))
    ref = O.tvd(hu, hv, hw, hv, g, 2.0)
    assert rel(interior(sv), interior(ref)) <= 1e-14


def steps(n, values, length):
    """Piecewise-constant profile: runs of `length` cells cycling `values`."""
    return np.array([values[(i // length) % len(values)] for i in range(n)], dtype=np.float64)


def test_step_profile_in_x_is_donor_cell_for_u():
    nx, ny, nz = 24, 3, 4
    g = I.make_geometry(nx, ny, nz)
    prof = steps(nx, [1.0, 2.5, -0.7, -1.9, 0.4], 3)  # runs of 3, sign changes included
    u = padded(np.broadcast_to(prof[:, None, None], (nx, ny, nz)))
    z = padded(np.zeros((nx, ny, nz)))
    su, sv, sw, _ = O.tvd_momentum(u, z, z.copy(), g, 1.0)
    a = (prof + np.roll(prof, -1)) / 2  # mass flux / rhon through the face east of u_i
    donor = np.where(a >= 0, prof, np.roll(prof, -1))
    F = a * donor
    ref = -(F - np.roll(F, 1)) / g.dx
    for j in range(ny):
        for k in range(nz):
            np.testing.assert_allclose(interior(su)[:, j, k], ref, rtol=0, atol=1e-15)
    assert np.abs(interior(sv)).max() == 0.0 and np.abs(interior(sw)).max() == 0.0


def test_step_profile_in_y_is_donor_cell_for_v():
    nx, ny, nz = 3, 20, 4
    g = I.make_geometry(nx, ny, nz, 50.0, 30.0)
    prof = steps(ny, [-1.2, 0.8, 2.0, -0.3], 2)
    v = padded(np.broadcast_to(prof[None, :, None], (nx, ny, nz)))
    z = padded(np.zeros((nx, ny, nz)))
    _, sv, _, _ = O.tvd_momentum(z, v, z.copy(), g, 1.0)
    a = (prof + np.roll(prof, -1)) / 2
    F = a * np.where(a >= 0, prof, np.roll(prof, -1))
    ref = -(F - np.roll(F, 1)) / g.dy
    for i in range(nx):
        for k in range(nz):
            np.testing.assert_allclose(interior(sv)[i, :, k], ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("values", [[0.3, -0.2, 0.5], [-0.4, 0.6], [0.2, 0.2]])
def test_step_profile_in_z_is_donor_cell_for_w_with_ground_and_lid(values):
    nz = 16
    g = I.make_geometry(2, 2, nz)
    # faces 0..nz-2 in runs of two, the lid (nz-1) and the ground are 0
    col = np.zeros(nz)
    col[:nz - 1] = steps(nz - 1, values, 2)
    col[nz - 3:nz - 1] = col[nz - 3]  # last run before the lid also two long
    w = padded(np.broadcast_to(col[None, None, :], (2, 2, nz)))
    z = padded(np.zeros((2, 2, nz)))
    _, _, sw, cm = O.tvd_momentum(z, z.copy(), w, g, 1.0)
    wf = np.concatenate([[0.0], col[:nz - 1], [0.0]])  # faces -1..nz-1
    rho_f = np.concatenate([[0.0], g.rho[:nz - 1], [0.0]])  # w = 0 there anyway
    # face at the centre of cell q sits between wf[q] (face q-1) and wf[q+1] (face q)
    m = (rho_f[:-1] * wf[:-1] + rho_f[1:] * wf[1:]) / 2
    donor = np.where(m >= 0, wf[:-1], wf[1:])
    F = m * donor
    dz = 1.0 / g.rdz
    rdzn = 2.0 / (dz[:-1] + dz[1:])
    ref = -(1.0 / g.rho[:nz - 1]) * rdzn * (F[1:] - F[:-1])
    for i in range(2):
        for j in range(2):
            got = interior(sw)[i, j]
            np.testing.assert_allclose(got[:nz - 1], ref, rtol=1e-13, atol=1e-16)
            assert got[nz - 1] == 0.0


def quickest(U, C, D, c):
    """Leonard (1979): QUICKEST face value (no limiter)."""
    return (C + D) / 2 - c * (D - C) / 2 - (1 - c * c) / 6 * (D - 2 * C + U)


def test_quadratic_in_x_gives_quickest_for_v():
    # v = alpha i^2 along x (monotone, limiter inactive for i >= 2), u = U0:
    # sv_i = -U0 alpha (2 i - c)/dx with c = U0 dt/dx
    nx, ny, nz = 16, 2, 3
    g = I.make_geometry(nx, ny, nz)
    U0, alpha, dt = 3.0, 0.01, 4.0
    x = np.arange(nx, dtype=np.float64)
    v = padded(np.broadcast_to((alpha * x * x)[:, None, None], (nx, ny, nz)))
    u = padded(np.full((nx, ny, nz), U0))
    z = padded(np.zeros((nx, ny, nz)))
    _, sv, _, _ = O.tvd_momentum(u, v, z, g, dt)
    c = U0 * dt / g.dx
    ref = -U0 * alpha * (2 * x - c) / g.dx
    np.testing.assert_allclose(interior(sv)[2:nx - 1, :, :],
                               np.broadcast_to(ref[2:nx - 1, None, None], (nx - 3, ny, nz)),
                               rtol=1e-12)


def test_quadratic_in_x_gives_quickest_for_w_lateral_courant():
    # The w lateral faces carry m = a_k u_k + b_k u_{k+1}; their Courant number
    # is |m|/rho_k dt/dx.  With u = U0 and w = alpha i^2 the x part is
    # -(m/rho_k) alpha (2 i - c)/dx; the z part is removed by subtracting the
    # same run with u = 0.
    nx, ny, nz = 16, 2, 6
    g = I.make_geometry(nx, ny, nz)
    U0, alpha, dt = 4.0, 0.02, 3.0
    x = np.arange(nx, dtype=np.float64)
    prof = np.broadcast_to((alpha * x * x)[:, None, None], (nx, ny, nz)).copy()
    prof[:, :, nz - 1] = 0.0
    w = padded(prof)
    z = padded(np.zeros((nx, ny, nz)))
    _, _, sw1, _ = O.tvd_momentum(padded(np.full((nx, ny, nz), U0)), z, w, g, dt)
    _, _, sw0, _ = O.tvd_momentum(z, z.copy(), w, g, dt)
    dz = 1.0 / g.rdz
    dzn = (dz[:-1] + dz[1:]) / 2
    a = dz[:-1] * g.rhon[:-1] / (2 * dzn)
    b = dz[1:] * g.rhon[1:] / (2 * dzn)
    m = (a + b) * U0
    c = m / g.rho[:-1] * dt / g.dx
    ref = -(m / g.rho[:-1])[None, :] * alpha * (2 * x[:, None] - c[None, :]) / g.dx
    got = interior(sw1 - sw0)[2:nx - 1, :, :nz - 1]
    for j in range(ny):
        np.testing.assert_allclose(got[:, j, :], ref[2:nx - 1], rtol=1e-11)


def test_quadratic_in_z_gives_quickest_for_w_vertical_courant():
    # w_k = alpha (k+1)^2 on faces 0..nz-2 (the ground face fits the parabola),
    # u = v = 0.  Faces at cell centres q: m_q = (rho_{q-1} w_{q-1} + rho_q w_q)/2,
    # c_q = m_q/rhon_q dt/dz_q, value QUICKEST(w_{q-2}, w_{q-1}, w_q) for q >= 1,
    # the ground value 0 for q = 0 (no far-upwind face); checked below the lid's
    # influence (k <= nz-3).
    nz = 12
    g = I.make_geometry(2, 2, nz)
    alpha, dt = 0.002, 2.0
    col = np.zeros(nz)
    col[:nz - 1] = alpha * (np.arange(nz - 1) + 1.0) ** 2
    w = padded(np.broadcast_to(col[None, None, :], (2, 2, nz)))
    z = padded(np.zeros((2, 2, nz)))
    _, _, sw, _ = O.tvd_momentum(z, z.copy(), w, g, dt)
    wf = np.concatenate([[0.0], col])  # wf[q+1] = w_q, wf[0] = ground
    F = np.zeros(nz)
    for q in range(nz - 1):
        rho_lo = g.rho[q - 1] if q >= 1 else 0.0
        m = (rho_lo * wf[q] + g.rho[q] * wf[q + 1]) / 2
        c = m / g.rhon[q] * dt * g.rdz[q]
        assert 0 < c < 0.5
        F[q] = 0.0 if q == 0 else m * quickest(wf[q - 1], wf[q], wf[q + 1], c)
    dz = 1.0 / g.rdz
    rdzn = 2.0 / (dz[:-1] + dz[1:])
    ref = -(1.0 / g.rho[:nz - 2]) * rdzn[:nz - 2] * (F[1:nz - 1] - F[:nz - 2])
    for i in range(2):
        for j in range(2):
            np.testing.assert_allclose(interior(sw)[i, j, :nz - 2], ref, rtol=1e-12)


def test_mirror_in_x():
    # x -> -x: u_i -> -u_{n-2-i}, v, w_i -> v, w_{n-1-i}; su -> -su, sv, sw mirrored
    g, (u, v, w) = flow(10, 8, 12, 7, amp=12.0)
    iu, iv, iw = (interior(a) for a in (u, v, w))
    mu = padded(-np.roll(iu[::-1], -1, 0))
    mv, mw = padded(iv[::-1].copy()), padded(iw[::-1].copy())
    su, sv, sw, c0 = O.tvd_momentum(u, v, w, g, 2.0)
    tu, tv, tw, c1 = O.tvd_momentum(mu, mv, mw, g, 2.0)
    np.testing.assert_allclose(interior(tu), -np.roll(interior(su)[::-1], -1, 0), rtol=0,
                               atol=1e-14 * np.abs(interior(su)).max())
    np.testing.assert_allclose(interior(tv), interior(sv)[::-1], rtol=0,
                               atol=1e-14 * np.abs(interior(sv)).max())
    np.testing.assert_allclose(interior(tw), interior(sw)[::-1], rtol=0,
                               atol=1e-14 * np.abs(interior(sw)).max())
    assert abs(c0 - c1) <= 1e-15 * c0


def test_mirror_in_z_on_a_uniform_column():
    # z -> -z with constant density and spacing: u_k -> u_{nz-1-k},
    # w_k -> -w_{nz-2-k}; the lid and the ground trade places
    nx, ny, nz = 6, 5, 10
    g = uniform_geometry(nx, ny, nz)
    f = I.make_fields(g, 0, 8, amp=8.0)
    u, v, w = f["u"], f["v"], f["w"]
    w[:, :, -1] = 0.0
    mu, mv = u[:, :, ::-1].copy(), v[:, :, ::-1].copy()
    mw = np.zeros_like(w)
    mw[:, :, :nz - 1] = -w[:, :, nz - 2::-1]
    su, sv, sw, _ = O.tvd_momentum(padded(u), padded(v), padded(w), g, 2.0)
    tu, tv, tw, _ = O.tvd_momentum(padded(mu), padded(mv), padded(mw), g, 2.0)
    sc = max(np.abs(interior(su)).max(), np.abs(interior(sw)).max())
    np.testing.assert_allclose(interior(tu), interior(su)[:, :, ::-1], rtol=0, atol=1e-13 * sc)
    np.testing.assert_allclose(interior(tv), interior(sv)[:, :, ::-1], rtol=0, atol=1e-13 * sc)
    ref_w = np.zeros_like(w)
    ref_w[:, :, :nz - 1] = -interior(sw)[:, :, nz - 2::-1]
    np.testing.assert_allclose(interior(tw), ref_w, rtol=0, atol=1e-13 * sc)


@pytest.mark.parametrize("seed", [9, 10])
def test_u_and_v_momentum_conserved(seed):
    g, (u, v, w) = flow(12, 10, 16, seed, amp=10.0)
    su, sv, _, _ = O.tvd_momentum(u, v, w, g, 2.0)
    mass = ((1.0 / g.rdz) * g.rhon)[None, None, :]
    for s in (su, sv):
        t = mass * interior(s)
        assert abs(t.sum()) <= 1e-13 * np.abs(t).sum()


def test_uniform_u_in_any_flow():
    # u = U0 everywhere: su = -U0 (D_i + D_{i+1}) / (2 rhon_k) with D the
    # p-cell mass divergence
    g, (u, v, w) = flow(10, 8, 12, 11)
    U0 = -2.5
    u = padded(np.full((g.nx, g.ny, g.nz), U0))
    su, _, _, _ = O.tvd_momentum(u, v, w, g, 1.0)
    D = interior(O.divergence(*(O.halo_fill(x) for x in (u, v, w)), g))
    ref = -U0 * (D + np.roll(D, -1, 0)) / (2 * g.rhon[None, None, :])
    np.testing.assert_allclose(interior(su), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_courant_number_above_one_is_reported():
    g, (u, v, w) = flow(6, 6, 8, 12)
    with pytest.raises(O.CourantError):
        O.tvd_momentum(u, v, w, g, 400.0)
    _, _, _, cm = O.tvd_momentum(u, v, w, g, 400.0, allow_cfl=True)
    assert cm > 1.0


def test_step_tvd_momentum_scalars_equal_plain_step():
    g = I.make_geometry(8, 8, 16)
    f = I.make_fields(g, 2, 13, padded=True)
    state = [f[n] for n in ("u", "v", "w", "th", "q1")]
    a = O.step_tvd_momentum([x.copy() for x in state], g, 0.5)
    b = O.step([O.halo_fill(x) for x in state], g, 0.5)
    for s in (3, 4):
        np.testing.assert_array_equal(interior(a[s]), interior(b[s]))
    su, sv, sw, _ = O.tvd_momentum(*state[:3], g, 0.5)
    for fi, s in enumerate((su, sv, sw)):
        ref = interior(state[fi]) + 0.5 * interior(s)
        if fi == 2:
            ref[:, :, -1] = 0.0
        np.testing.assert_array_equal(interior(a[fi]), ref)


def test_region_equals_whole_domain():
    g, (u, v, w) = flow(11, 9, 10, 14)
    full = O.tvd_momentum(u, v, w, g, 1.0)
    part = O.tvd_momentum(u, v, w, g, 1.0, region=(3, 8, 0, 5))
    for f in range(3):
        np.testing.assert_array_equal(interior(part[f])[3:8, 0:5], interior(full[f])[3:8, 0:5])
        assert np.abs(interior(part[f])[:3]).max() == 0.0


def test_worked_example_1d():
    """Hand-derived fixture (tests/golden/tvd_momentum_1d.txt): the face values
    of every limiter case (flat upwind, active QUICKEST, the ULTIMATE bound
    binding, extrema, zero mass flux) and the resulting su."""
    import os
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "tvd_momentum_1d.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                key, *vals = line.split()
                gold[key] = np.array([float(x) for x in vals])
    u = gold["u"]
    a = (u + np.roll(u, -1)) / 2
    faces = [O.ultimate_face(u[i - 1], u[i], u[(i + 1) % 6], a[i] * 0.25) for i in range(6)]
    np.testing.assert_allclose(faces, gold["face"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(a * gold["face"], gold["flux"], rtol=1e-15, atol=0)
    one = np.ones(2)
    zf = np.arange(1, 3, dtype=float)
    g = I.Geometry(6, 1, 2, 1.0, 1.0, one.copy(), one.copy(), one.copy(), zf, zf - 0.5)
    U = padded(np.repeat(u[:, None, None], 2, axis=2))
    Z = padded(np.zeros((6, 1, 2)))
    su, sv, sw, cm = O.tvd_momentum(U, Z, Z.copy(), g, 0.25)
    for k in range(2):
        np.testing.assert_allclose(interior(su)[:, 0, k], gold["su"], rtol=0, atol=1e-15)
    assert np.all(interior(sv) == 0) and np.all(interior(sw) == 0)
    assert gold["su"].sum() == 0.0
    assert cm == 0.75
