"""Pins of the oracle's budget entries and of the vertical Courant number of
its TVD scalar faces on a strongly stretched grid.

The budgets (largest Courant number, scalar mass, scalar minimum) are checked
against planted values and closed forms worked out here from their
definitions (the scalar mass is the density-weighted volume integral of a
scalar; the Courant number of a vertical face uses the distance between the
two cell centres beside it).  The vertical TVD faces are checked against the
exact swept average of a quadratic in index space (QUICKEST is exact for
quadratics where the limiter is idle, Leonard 1979), on a grid whose layer
thicknesses grow by half from one layer to the next, so that using the layer
thickness instead of the centre distance, or dropping the first-order rule
next to the ground and the lid, moves the face value far outside round-off.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_12850_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def steep_geometry(nx, ny, nz, ratio=1.5, dz0=10.0, dx=50.0, dy=35.0):
    """Layer thickness dz0 * ratio^k; densities decreasing with height."""
    dz = dz0 * ratio ** np.arange(nz, dtype=float)
    zf = np.cumsum(dz)
    zc = zf - 0.5 * dz
    rho = 1.2 * np.exp(-zf / 8000.0)
    rhon = 1.2 * np.exp(-zc / 8000.0)
    return I.Geometry(nx, ny, nz, dx, dy, 1.0 / dz, rho, rhon, zf, zc)


def filled(*arrs):
    return [O.halo_fill(I.pad(np.ascontiguousarray(a, dtype=np.float64))) for a in arrs]


def centre_distance(g, k):
    """Distance between the centres of cells k and k+1 (from the thicknesses)."""
    dz = 1.0 / g.rdz
    return 0.5 * (dz[k] + dz[k + 1])


# ---------------------------------------------------------------------------
# Largest Courant number
# ---------------------------------------------------------------------------
def test_max_courant_of_a_planted_vertical_face_uses_centre_distance():
    nx, ny, nz = 5, 4, 7
    g = steep_geometry(nx, ny, nz)
    dt = 0.5
    u = np.zeros((nx, ny, nz))
    v = np.zeros((nx, ny, nz))
    w = np.zeros((nx, ny, nz))
    k0 = 3
    dzn = centre_distance(g, k0)
    w[2, 1, k0] = -0.8 * dzn / dt          # Courant number 0.8 at face k0 + 1/2
    u[1, 3, 5] = 0.3 * g.dx / dt           # 0.3
    v[4, 0, 2] = 0.5 * g.dy / dt           # 0.5
    w[0, 0, nz - 1] = 1e6                  # the lid: not a face the flow crosses
    U, V, W = filled(u, v, w)
    c = O.max_courant(U, V, W, g, dt)
    np.testing.assert_allclose(c, 0.8, rtol=1e-14)
    # the layer thickness would give a different number on this grid
    assert abs(0.8 * dzn * g.rdz[k0] - 0.8) > 0.1


def test_max_courant_lateral_faces_use_their_own_spacing():
    nx, ny, nz = 4, 6, 5
    g = steep_geometry(nx, ny, nz, dx=50.0, dy=20.0)
    dt = 0.5
    z = np.zeros((nx, ny, nz))
    u, v, w = z.copy(), z.copy(), z.copy()
    u[3, 2, 1] = 0.9 * g.dx / dt
    v[1, 5, 4] = 0.6 * g.dy / dt
    U, V, W = filled(u, v, w)
    np.testing.assert_allclose(O.max_courant(U, V, W, g, dt), 0.9, rtol=1e-14)
    u[3, 2, 1] = 0.0
    v[1, 5, 4] = -0.7 * g.dy / dt
    U, V, W = filled(u, v, w)
    np.testing.assert_allclose(O.max_courant(U, V, W, g, dt), 0.7, rtol=1e-14)


# ---------------------------------------------------------------------------
# Scalar mass and minimum
# ---------------------------------------------------------------------------
def budgets_of(g, phis):
    shape = (g.nx, g.ny, g.nz)
    z = np.zeros(shape)
    U, V, W = filled(z, z, z)
    S = filled(*phis)
    T = filled(*[z for _ in phis])
    b, _ = O.budgets(U, V, W, U, V, W, S, T, g)
    return b


def test_scalar_mass_of_a_uniform_scalar_is_density_times_volume():
    g = steep_geometry(6, 5, 8)
    c = 2.75
    b = budgets_of(g, [np.full((6, 5, 8), c)])
    column = np.sum(g.rhon * (1.0 / g.rdz))  # density-weighted column height
    np.testing.assert_allclose(b["M_s0"], c * 6 * 5 * column, rtol=1e-14)


def test_scalar_mass_of_a_single_cell_is_its_density_and_thickness():
    g = steep_geometry(4, 3, 6)
    for k0 in (0, 2, 5):
        phi = np.zeros((4, 3, 6))
        phi[1, 2, k0] = 1.0
        b = budgets_of(g, [phi])
        np.testing.assert_allclose(b["M_s0"], g.rhon[k0] / g.rdz[k0], rtol=1e-15)


def test_scalar_minimum_is_the_planted_minimum():
    g = steep_geometry(5, 4, 6)
    rng = np.random.default_rng(3)
    phi = rng.uniform(1.0, 2.0, (5, 4, 6))
    phi[0, 3, 5] = 1e6       # a planted maximum far above everything else
    phi[4, 1, 2] = -7.25     # the planted minimum
    psi = rng.uniform(10.0, 20.0, (5, 4, 6))
    b = budgets_of(g, [phi, psi])
    assert b["min_s0"] == -7.25
    assert b["min_s1"] == psi.min()


# ---------------------------------------------------------------------------
# Vertical TVD faces on a strongly stretched grid
# ---------------------------------------------------------------------------
def primitive(t):
    """Primitive of q(t) = 3 + t + 0.02 t^2 (a gentle monotone quadratic)."""
    return 3.0 * t + 0.5 * t ** 2 + 0.02 * t ** 3 / 3.0


def cell_average(lo, hi):
    return (primitive(hi) - primitive(lo)) / (hi - lo)


def single_face_flux(g, k0, wval, prof, dt):
    """Face value at the top face of cell k0 when only that face carries flow:
    the flux enters the tendencies of cells k0 and k0+1 alone, and both give it
    back (rhon_k s_k / rdz_k = -(F_top - F_bottom))."""
    nx, ny, nz = g.nx, g.ny, g.nz
    z = np.zeros((nx, ny, nz))
    w = z.copy()
    w[:, :, k0] = wval
    phi = np.broadcast_to(prof[None, None, :], (nx, ny, nz)).copy()
    U, V, W, P = filled(z, z, w, phi)
    s = I.interior(O.tvd(U, V, W, P, g, dt))
    col = s[1, 1]
    f_from_below = -col[k0] * g.rhon[k0] / g.rdz[k0]
    f_from_above = col[k0 + 1] * g.rhon[k0 + 1] / g.rdz[k0 + 1]
    np.testing.assert_allclose(f_from_above, f_from_below, rtol=1e-13)
    others = np.delete(col, [k0, k0 + 1])
    assert np.all(others == 0.0)
    return f_from_below / (g.rho[k0] * wval)


@pytest.mark.parametrize("k0", [1, 3, 5])
@pytest.mark.parametrize("c", [0.2, 0.65])
@pytest.mark.parametrize("up", [True, False])
def test_vertical_quickest_face_is_the_swept_average_in_index_space(k0, c, up):
    """Courant number c = |w| dt / (distance between the centres beside the
    face); with the limiter idle the face value is the exact average of the
    quadratic over the part of the upwind cell that crosses the face in one
    step, in index space (cell k spans [k, k+1])."""
    nz = 8
    g = steep_geometry(3, 3, nz)
    dt = 0.5
    kk = np.arange(nz + 1, dtype=float)
    prof = cell_average(kk[:-1], kk[1:])
    dzn = centre_distance(g, k0)
    speed = c * dzn / dt
    if up:
        wval = speed
        expect = cell_average(k0 + 1 - c, k0 + 1.0)      # swept from cell k0
    else:
        wval = -speed
        expect = cell_average(k0 + 1.0, k0 + 1 + c)      # swept from cell k0+1
    got = single_face_flux(g, k0, wval, prof, dt)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-12)
    # with the layer thickness in place of the centre distance the Courant
    # number, and so the face value, would differ by far more than round-off
    c_wrong = c * dzn * g.rdz[k0]
    wrong = (cell_average(k0 + 1 - c_wrong, k0 + 1.0) if up
             else cell_average(k0 + 1.0, k0 + 1 + c_wrong))
    assert abs(wrong - expect) > 1e-3


@pytest.mark.parametrize("c", [0.3, 0.9])
def test_vertical_faces_next_to_ground_and_lid_are_first_order_upwind(c):
    """Where the far-upwind cell lies outside the column (upward flow through
    the face above the ground cell, downward flow through the face below the
    lid cell) the face takes the upwind cell's value; the faces with the other
    flow direction there keep the third-order value."""
    nz = 7
    g = steep_geometry(3, 3, nz)
    dt = 0.5
    kk = np.arange(nz + 1, dtype=float)
    prof = cell_average(kk[:-1], kk[1:])
    # ground: face 1/2, upward flow, upwind cell 0, no cell below it
    w0 = c * centre_distance(g, 0) / dt
    got = single_face_flux(g, 0, w0, prof, dt)
    np.testing.assert_allclose(got, prof[0], rtol=1e-14)
    assert abs(cell_average(1 - c, 1.0) - prof[0]) > 1e-2  # QUICKEST would differ
    # the same face with downward flow: upwind cell 1, far-upwind cell 2 exist
    got = single_face_flux(g, 0, -w0, prof, dt)
    np.testing.assert_allclose(got, cell_average(1.0, 1.0 + c), rtol=0, atol=1e-12)
    # lid: face nz-3/2, downward flow, upwind cell nz-1, nothing above it
    kt = nz - 2
    wt = c * centre_distance(g, kt) / dt
    got = single_face_flux(g, kt, -wt, prof, dt)
    np.testing.assert_allclose(got, prof[nz - 1], rtol=1e-14)
    assert abs(cell_average(kt + 1.0, kt + 1.0 + c) - prof[nz - 1]) > 1e-2
    # the same face with upward flow keeps the third-order value
    got = single_face_flux(g, kt, wt, prof, dt)
    np.testing.assert_allclose(got, cell_average(kt + 1 - c, kt + 1.0), rtol=0, atol=1e-12)
