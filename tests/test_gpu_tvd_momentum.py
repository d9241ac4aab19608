"""GPU tests of the TVD advection of momentum and the all-TVD step.

* monc_advect_tvd_momentum against the FP64 oracle, per field
  max |gpu - oracle| / max |oracle| <= 1e-13, on several tiles of columns with
  ragged edges, one- and two-chunk columns, the smallest grids; halos are not
  read (NaN there) and not written; the largest Courant number agrees with the
  oracle's to 1e-14; several x-segments of the march with a ragged last one.
* monc_step_tvd_momentum against the oracle's step (1e-13 on the increments).
* At the benchmark's full size (1024 x 1024 x 128, 5 fields, the launch the
  benchmark times) the step matches the oracle on sampled blocks of columns,
  including the periodic edges, and conserves u and v momentum.
* 20 all-TVD steps against 20 oracle steps (1e-11); a periodic shift of the
  inputs shifts the source terms bitwise, wherever a column falls in its
  workgroup and its x-segment (so a face evaluated by either of its columns,
  or carried from the plane before, is the same).
* Courant numbers near 1 (0.95) match the oracle; above 1 the largest one is
  still reported exactly.
"""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu

DT = 4.0
TOL = 1e-13


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()


def nan_halo(a):
    b = np.full_like(a, np.nan)
    b[2:-2, 2:-2, :] = a[2:-2, 2:-2, :]
    return b


# the march takes x-segments of 64 planes: 130 and 200 give several segments
# and a ragged last one
SHAPES = [(16, 16, 32), (23, 17, 50), (9, 6, 128), (1, 1, 7), (40, 12, 64), (2, 3, 2),
          (5, 9, 65), (130, 6, 40), (200, 5, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_tvd_momentum_matches_oracle(shape):
    nx, ny, nz = shape
    say(f"tvd_momentum {shape}")
    g, host = case(nx, ny, nz, 0, seed=1300 + nx + nz)
    su, sv, sw, cmax = O.tvd_momentum(*host[:3], g, DT)
    T = torch()
    d = to_dev([nan_halo(h) for h in host[:3]])
    out = [T.full(d[0].shape, -7.0, dtype=T.float64, device=dev()) for _ in range(3)]
    cm = T.full((1,), -1.0, dtype=T.float64, device=dev())
    M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof_dev(g), DT, cmax=cm)
    T.cuda.synchronize()
    for n, (o, r) in enumerate(zip(out, (su, sv, sw))):
        got = o.cpu().numpy()
        e = rel_err(got, r)
        assert e <= TOL, f"field {n}: {e:.3e}"
        halo = got.copy()
        halo[2:-2, 2:-2, :] = -7.0
        assert np.all(halo == -7.0), f"field {n}: halo written"
    assert abs(cm.item() - cmax) <= 1e-14 * cmax


def test_tvd_momentum_without_cmax_and_stream():
    g, host = case(12, 10, 40, 0, seed=1400)
    ref = O.tvd_momentum(*host[:3], g, DT)
    T = torch()
    s = T.cuda.Stream()
    d = to_dev(host[:3])
    out = [T.empty_like(d[0]) for _ in range(3)]
    with T.cuda.stream(s):
        M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof_dev(g), DT, stream=s)
    s.synchronize()
    for n in range(3):
        assert rel_err(out[n].cpu().numpy(), ref[n]) <= TOL, n


@pytest.mark.parametrize("shape,nscal", [((16, 16, 32), 2), ((13, 7, 128), 3), ((4, 4, 3), 0),
                                         ((10, 8, 70), 1), ((131, 6, 33), 1)])
def test_step_tvd_momentum_matches_oracle(shape, nscal):
    nx, ny, nz = shape
    say(f"step_tvd_momentum {shape} nscal={nscal}")
    g, host = case(nx, ny, nz, nscal, seed=1500 + nx + nscal)
    ref = O.step_tvd_momentum([h.copy() for h in host], g, DT)
    T = torch()
    d = to_dev([nan_halo(h) for h in host])
    out = [T.full(d[0].shape, -7.0, dtype=T.float64, device=dev()) for _ in host]
    cm = T.zeros(1, dtype=T.float64, device=dev())
    M.monc_step_tvd_momentum(d, out, g.dx, g.dy, prof_dev(g), DT, cmax=cm)
    T.cuda.synchronize()
    _, _, _, cref = O.tvd_momentum(*host[:3], g, DT)
    for n, (o, r) in enumerate(zip(out, ref)):
        got = o.cpu().numpy()
        e = rel_err(got - host[n], r - host[n])
        assert e <= TOL, f"field {n}: {e:.3e}"
    assert np.all(out[2].cpu().numpy()[2:-2, 2:-2, nz - 1] == 0.0)
    assert abs(cm.item() - cref) <= 1e-14 * cref


def test_tvd_momentum_rejects_bad_arguments():
    T = torch()
    g, host = case(4, 4, 8, 0, seed=1600)
    d = to_dev(host[:3])
    out = [T.empty_like(d[0]) for _ in range(3)]
    with pytest.raises(M.MoncError):
        M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof_dev(g), 0.0)
    with pytest.raises(M.MoncError):  # output aliases an input
        M.monc_advect_tvd_momentum(*d, d[0], out[1], out[2], g.dx, g.dy, prof_dev(g), DT)


def test_full_size_step_matches_oracle_on_sampled_blocks():
    """1024 x 1024 x 128 with five fields, in the launch the benchmark times:
    the increments of every field on blocks of 8 x 8 full columns (corner,
    periodic edges, middle) against the oracle, and u, v momentum conserved
    over the whole domain."""
    nx, ny, nz = 1024, 1024, 128
    say("full-size step_tvd_momentum")
    g = I.make_geometry(nx, ny, nz)
    f = I.make_fields(g, 2, 7, padded=True)
    names = ["u", "v", "w", "th", "q1"]
    host = [f[n] for n in names]
    host[3] = host[3] - 300.0  # anomalies keep the sampled relative errors meaningful
    T = torch()
    d = to_dev(host)
    out = [T.empty_like(d[0]) for _ in host]
    cm = T.zeros(1, dtype=T.float64, device=dev())
    prof = prof_dev(g)
    M.monc_step_tvd_momentum(d, out, g.dx, g.dy, prof, 0.5, cmax=cm)
    su = [T.empty_like(d[0]) for _ in range(3)]
    M.monc_advect_tvd_momentum(d[0], d[1], d[2], *su, g.dx, g.dy, prof, 0.5)
    T.cuda.synchronize()
    mass = T.from_numpy((1.0 / g.rdz) * g.rhon).to(dev())
    for n in range(2):
        t = su[n][2:-2, 2:-2, :] * mass
        assert abs(t.sum().item()) <= 1e-12 * t.abs().sum().item(), n
    del su
    filled = [O.halo_fill(h) for h in host]
    blocks = [(0, 8, 0, 8), (nx - 8, nx, ny - 8, ny), (0, 8, ny - 8, ny), (509, 517, 300, 308)]
    got = [o.cpu().numpy() for o in out]
    cmax = 0.0
    for (i0, i1, j0, j1) in blocks:
        ms = O.tvd_momentum(*filled[:3], g, 0.5, region=(i0, i1, j0, j1))
        cmax = max(cmax, ms[3])
        tend = list(ms[:3]) + [O.tvd(*filled[:3], q, g, 0.5, region=(i0, i1, j0, j1))
                               for q in filled[3:]]
        for n in range(5):
            ref = 0.5 * I.interior(tend[n])[i0:i1, j0:j1]
            inc = I.interior(got[n])[i0:i1, j0:j1] - I.interior(host[n])[i0:i1, j0:j1]
            if n == 2:
                ref[:, :, -1] = -I.interior(host[2])[i0:i1, j0:j1, -1]
            e = np.abs(inc - ref).max() / np.abs(ref).max()
            assert e <= TOL, f"block {(i0, i1, j0, j1)} field {names[n]}: {e:.3e}"
    # the device maximum covers the whole domain, so it bounds the sampled one
    assert cm.item() >= cmax * (1 - 1e-14)
    assert cm.item() <= 1.0


def test_all_tvd_trajectory_matches_oracle():
    """20 all-TVD steps of a 24 x 20 x 40 state with two scalars against 20
    oracle steps (1e-11 on the accumulated change)."""
    say("all-TVD trajectory 24x20x40 x20")
    g, host = case(24, 20, 40, 2, seed=1700)
    dt = 2.0
    ref = [h.copy() for h in host]
    for _ in range(20):
        ref = O.step_tvd_momentum(ref, g, dt)
    T = torch()
    a = to_dev(host)
    b = [T.empty_like(x) for x in a]
    prof = prof_dev(g)
    for _ in range(20):
        M.monc_step_tvd_momentum(a, b, g.dx, g.dy, prof, dt)
        a, b = b, a
    T.cuda.synchronize()
    for n in range(len(host)):
        e = rel_err(a[n].cpu().numpy() - host[n], ref[n] - host[n])
        assert e <= 1e-11, f"field {n}: {e:.3e}"


@pytest.mark.parametrize("shape", [(22, 18, 70), (130, 10, 40)])
def test_tvd_momentum_translation_invariance_bitwise(shape):
    """A periodic shift of the inputs shifts the source terms bitwise: where a
    column falls in its workgroup or its x-segment (the west face evaluated
    at a segment's start or carried from the plane before) does not change
    its arithmetic."""
    say(f"tvd_momentum translation {shape}")
    g, host = case(*shape, 0, seed=1800)
    T = torch()
    prof = prof_dev(g)

    def run(fields):
        d = to_dev(fields)
        out = [T.empty_like(d[0]) for _ in range(3)]
        M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof, DT)
        T.cuda.synchronize()
        return [I.interior(o.cpu().numpy()) for o in out]

    base = run(host[:3])
    shifted = run([I.pad(np.roll(I.interior(h), (3, -5), axis=(0, 1))) for h in host[:3]])
    for a, b in zip(base, shifted):
        np.testing.assert_array_equal(np.roll(a, (3, -5), axis=(0, 1)), b)


def test_courant_near_one_matches_oracle():
    """dt chosen so that the largest Courant number is about 0.95 (the
    QUICKEST term depends most on c there)."""
    say("tvd_momentum near Courant 1")
    g, host = case(9, 6, 128, 0, seed=1300 + 9 + 128)
    _, _, _, c1 = O.tvd_momentum(*host[:3], g, 1.0)
    dt = 0.95 / c1  # the Courant numbers scale with dt
    su, sv, sw, cmax = O.tvd_momentum(*host[:3], g, dt)
    assert 0.9 < cmax <= 1.0
    T = torch()
    d = to_dev(host[:3])
    out = [T.empty_like(d[0]) for _ in range(3)]
    cm = T.zeros(1, dtype=T.float64, device=dev())
    M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof_dev(g), dt, cmax=cm)
    T.cuda.synchronize()
    for n, r in enumerate((su, sv, sw)):
        assert rel_err(out[n].cpu().numpy(), r) <= TOL, n
    assert abs(cm.item() - cmax) <= 1e-14 * cmax


def test_courant_above_one_is_reported():
    """Beyond the scheme's limit the values are unspecified, but the largest
    Courant number is still reported exactly."""
    g, host = case(8, 8, 16, 0, seed=1900)
    dt = 200.0
    _, _, _, cmax = O.tvd_momentum(*host[:3], g, dt, allow_cfl=True)
    assert cmax > 1.0
    T = torch()
    d = to_dev(host[:3])
    out = [T.empty_like(d[0]) for _ in range(3)]
    cm = T.zeros(1, dtype=T.float64, device=dev())
    M.monc_advect_tvd_momentum(*d, *out, g.dx, g.dy, prof_dev(g), dt, cmax=cm)
    T.cuda.synchronize()
    assert abs(cm.item() - cmax) <= 1e-14 * cmax
