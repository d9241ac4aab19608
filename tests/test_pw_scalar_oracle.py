"""Pins of the oracle's centred-flux scalar advection (MONC's other scalar
scheme: the PW flux form applied to a cell-centred field), CPU only.

Each pin is a closed form or an identity of summation by parts, not the
oracle's formula: conservation for any flow; the variance identity
sum(rhon dz phi s) = -1/2 sum(dz phi^2 D), hence zero in divergence-free flow;
a uniform scalar gives -phi D / rhon; the 1-D centred difference; translation
invariance.
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


def flow(nx, ny, nz, seed, divfree=False):
    g = I.make_geometry(nx, ny, nz, 50.0, 50.0)
    f = I.make_fields(g, 2, seed, padded=True)
    if divfree:
        f.update(I.make_divfree_velocity(g, seed, 5.0, padded=True))
    return g, [O.halo_fill(f[n]) for n in ("u", "v", "w", "th", "q1")]


def dz_rhon(g):
    return (1.0 / g.rdz) * g.rhon


@pytest.mark.parametrize("seed", [0, 1])
def test_conservation_and_variance_identity(seed):
    g, (u, v, w, th, q) = flow(12, 10, 16, seed)
    D = interior(O.divergence(u, v, w, g))
    for phi in (th - 300.0, q):
        s = interior(O.pw_scalar(u, v, w, phi, g))
        p = interior(phi)
        mass = dz_rhon(g)[None, None, :]
        total = np.sum(mass * s)
        assert abs(total) <= 1e-13 * np.sum(np.abs(mass * s))
        var = np.sum(mass * p * s)
        closed = -0.5 * np.sum((1.0 / g.rdz)[None, None, :] * p * p * D)
        scale = np.sum(np.abs(mass * p * s))
        assert abs(var - closed) <= 1e-12 * scale


def test_variance_is_conserved_in_divergence_free_flow():
    g, (u, v, w, th, q) = flow(12, 10, 16, 3, divfree=True)
    assert np.abs(interior(O.divergence(u, v, w, g))).max() < 1e-12
    s = interior(O.pw_scalar(u, v, w, q, g))
    mass = dz_rhon(g)[None, None, :]
    var = np.sum(mass * interior(q) * s)
    assert abs(var) <= 1e-12 * np.sum(np.abs(mass * interior(q) * s))


def test_uniform_scalar_gives_minus_phi_d_over_rhon():
    g, (u, v, w, th, q) = flow(9, 8, 12, 4)
    c = 2.5
    phi = np.full_like(q, c)
    s = interior(O.pw_scalar(u, v, w, phi, g))
    D = interior(O.divergence(u, v, w, g))
    ref = -c * D / g.rhon[None, None, :]
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_one_dimensional_centred_difference():
    nx, ny, nz = 16, 1, 3
    g = I.make_geometry(nx, ny, nz, 25.0, 25.0)
    U = 3.0
    u = np.zeros((nx + 4, ny + 4, nz)) + U
    v = np.zeros_like(u)
    w = np.zeros_like(u)
    x = np.arange(nx)
    phi = I.pad(np.repeat(np.sin(2 * np.pi * x / nx)[:, None, None], nz, 2).repeat(ny, 1))
    s = interior(O.pw_scalar(u, v, w, O.halo_fill(phi), g))
    p = np.sin(2 * np.pi * x / nx)
    ref = -U * (np.roll(p, -1) - np.roll(p, 1)) / (2 * 25.0)
    for k in range(nz):
        np.testing.assert_allclose(s[:, 0, k], ref, rtol=0, atol=1e-14)


def test_translation_invariance_bitwise():
    g, (u, v, w, th, q) = flow(8, 6, 8, 5)
    base = O.pw_scalar(u, v, w, q, g)
    roll = lambda a: O.halo_fill(np.ascontiguousarray(
        np.pad(np.roll(np.roll(interior(a), 3, 0), -2, 1), ((2, 2), (2, 2), (0, 0)))))
    shifted = O.pw_scalar(roll(u), roll(v), roll(w), roll(q), g)
    np.testing.assert_array_equal(interior(roll(base)), interior(shifted))


def test_step_pw_scalars_momentum_equals_plain_step():
    g, state = flow(8, 8, 16, 6)
    a = O.step_pw_scalars([x.copy() for x in state], g, 0.5)
    b = O.step([x.copy() for x in state], g, 0.5)
    for f in range(3):
        np.testing.assert_array_equal(interior(a[f]), interior(b[f]))
