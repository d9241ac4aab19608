"""GPU tests of the other dynamics source terms and the combined step.

* monc_dyn_tend (Coriolis + buoyancy) against the FP64 oracle, per field
  max |gpu - oracle| / max |oracle| <= 1e-13, on several tiles with ragged
  edges; halos are not read (NaN there) and not written.
* monc_combine_step against its definition (the FMA of the kernel differs from
  NumPy's separate rounding by at most one rounding of the increment).
* monc_hybrid_step (two streams, and one) and the fused monc_step_dyn against
  the oracle's combined step (1e-13 on the increments), and bitwise against
  each other; at the benchmark's full size (1024 x 1024 x 128, 5 fields) the
  fused and hybrid steps agree bitwise and the dynamics terms match the oracle.
"""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu

PARAMS = (1.0e-4, 5.0, -2.0, 9.81, 300.0)  # fcor, ug, vg, grav, th0
DT = 0.5
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


SHAPES = [(16, 16, 32), (23, 17, 50), (9, 6, 128), (1, 1, 7), (40, 12, 64)]


@pytest.mark.parametrize("shape", SHAPES)
def test_dyn_tend_matches_oracle(shape):
    nx, ny, nz = shape
    say(f"dyn_tend {shape}")
    g, host = case(nx, ny, nz, 1, seed=900 + nx + nz)
    ref = O.dyn(host[0], host[1], host[3], *PARAMS)
    T = torch()
    d = to_dev([nan_halo(host[0]), nan_halo(host[1]), nan_halo(host[3])])
    out = [T.full(d[0].shape, -7.0, dtype=T.float64, device=dev()) for _ in range(3)]
    M.monc_dyn_tend(d[0], d[1], d[2], *out, PARAMS)
    T.cuda.synchronize()
    for q in range(3):
        o = out[q].cpu().numpy()
        assert np.all(np.isfinite(I.interior(o))), q
        assert rel_err(o, ref[q]) <= TOL, q
        halo = o.copy()
        halo[2:-2, 2:-2, :] = -7.0
        assert np.all(halo == -7.0), q  # nothing written outside the interior


def test_combine_step_definition():
    say("combine_step")
    nx, ny, nz = 13, 10, 70
    rng = np.random.default_rng(5)
    T = torch()
    sh = (nx + 4, ny + 4, nz)
    ins = [rng.normal(size=sh) for _ in range(5)]
    ta = [rng.normal(size=sh) for _ in range(5)]
    tb = [rng.normal(size=sh), rng.normal(size=sh), rng.normal(size=sh), None, None]
    di, da = to_dev(ins), to_dev(ta)
    db = [None if t is None else to_dev([t])[0] for t in tb]
    out = [T.full(sh, -7.0, dtype=T.float64, device=dev()) for _ in range(5)]
    M.monc_combine_step(di, da, db, out, DT)
    out_a = [T.full(sh, -7.0, dtype=T.float64, device=dev()) for _ in range(5)]
    M.monc_combine_step(di, da, None, out_a, DT)
    T.cuda.synchronize()
    for f in range(5):
        ref = ins[f] + DT * (ta[f] + (tb[f] if tb[f] is not None else 0.0))
        ref_a = ins[f] + DT * ta[f]
        if f == 2:
            ref[:, :, -1] = 0.0
            ref_a[:, :, -1] = 0.0
        for o, r in ((out[f], ref), (out_a[f], ref_a)):
            o = o.cpu().numpy()
            inc = DT * np.abs(ta[f]).max() * 4
            np.testing.assert_allclose(I.interior(o), I.interior(r), rtol=0,
                                       atol=2 * np.finfo(float).eps * (np.abs(r).max() + inc))
            h = o.copy()
            h[2:-2, 2:-2, :] = -7.0
            assert np.all(h == -7.0)
    # no second term for a field: bitwise the same as passing none at all
    for f in (3, 4):
        assert T.equal(out[f], out_a[f])


def run_three(host, g, params):
    """hybrid on two streams, hybrid on one stream, fused; returns device states."""
    T = torch()
    nf = len(host)
    d = to_dev(host)
    prof = prof_dev(g)
    sh = d[0].shape
    res = []
    side = T.cuda.Stream()
    for mode in ("two", "one", "fused"):
        out = [T.full(sh, float("nan"), dtype=T.float64, device=dev()) for _ in range(nf)]
        if mode == "fused":
            M.monc_step_dyn(d, out, g.dx, g.dy, prof, DT, params)
        else:
            tend = [T.empty_like(x) for x in d]
            dyn = [T.empty_like(x) for x in d[:3]]
            M.monc_hybrid_step(d, out, tend, dyn, g.dx, g.dy, prof, DT, params,
                               side_stream=side if mode == "two" else None)
        T.cuda.synchronize()
        res.append(out)
    return d, res


@pytest.mark.parametrize("shape,nscal", [((16, 16, 32), 1), ((23, 17, 50), 2),
                                         ((9, 6, 128), 3), ((20, 12, 64), 4)])
def test_hybrid_and_fused_steps_match_oracle_and_each_other(shape, nscal):
    nx, ny, nz = shape
    say(f"hybrid/fused {shape} nscal={nscal}")
    g, host = case(nx, ny, nz, nscal, seed=950 + nx + nscal)
    ref = O.step_dyn([h.copy() for h in host], g, DT, *PARAMS)
    d, (two, one, fused) = run_three(host, g, PARAMS)
    T = torch()
    for f in range(len(host)):
        assert T.equal(two[f][2:-2, 2:-2], one[f][2:-2, 2:-2]), f
        assert T.equal(fused[f][2:-2, 2:-2], two[f][2:-2, 2:-2]), f
        o = two[f].cpu().numpy()
        inc_gpu = I.interior(o) - I.interior(host[f])
        inc_ref = I.interior(ref[f]) - I.interior(host[f])
        den = np.abs(inc_ref).max()
        assert np.abs(inc_gpu - inc_ref).max() <= TOL * den + 1e-300, f


def test_dynamics_off_gives_the_plain_step_bitwise():
    say("dyn params zero == monc_step")
    g, host = case(24, 16, 64, 2, seed=977)
    T = torch()
    d = to_dev(host)
    prof = prof_dev(g)
    plain = [T.full_like(x, float("nan")) for x in d]
    M.monc_step(d, plain, g.dx, g.dy, prof, DT)
    zero = (0.0, 0.0, 0.0, 0.0, 300.0)
    _, (two, _, fused) = run_three(host, g, zero)
    for f in range(len(host)):
        assert T.equal(fused[f][2:-2, 2:-2], plain[f][2:-2, 2:-2]), f
        assert T.equal(two[f][2:-2, 2:-2], plain[f][2:-2, 2:-2]), f


def test_full_size_fused_equals_hybrid_and_dyn_matches_oracle():
    """At the benchmark's size and launch configuration."""
    w = I.WORKLOADS["big1024"]
    say(f"full size {w.nx}x{w.ny}x{w.nz}")
    T = torch()
    g = I.make_geometry(w.nx, w.ny, w.nz, w.dx, w.dx)
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    f = I.make_fields(g, w.nscal, w.seed, padded=True)
    d = [T.from_numpy(f[n]).to(dev()) for n in names]
    prof = prof_dev(g)
    fused = [T.empty_like(x) for x in d]
    M.monc_step_dyn(d, fused, g.dx, g.dy, prof, w.dt, PARAMS)
    hyb = [T.empty_like(x) for x in d]
    tend = [T.empty_like(x) for x in d]
    dyn = [T.empty_like(x) for x in d[:3]]
    side = T.cuda.Stream()
    M.monc_hybrid_step(d, hyb, tend, dyn, g.dx, g.dy, prof, w.dt, PARAMS, side_stream=side)
    T.cuda.synchronize()
    for q in range(len(d)):
        assert T.equal(fused[q][2:-2, 2:-2], hyb[q][2:-2, 2:-2]), q
    del fused, hyb, tend
    ref = O.dyn(f["u"], f["v"], f[names[3]], *PARAMS)
    for q in range(3):
        assert rel_err(dyn[q].cpu().numpy(), ref[q]) <= TOL, q


@pytest.mark.parametrize("shape,nscal", [((16, 16, 32), 2), ((23, 17, 50), 1),
                                         ((9, 6, 128), 4), ((5, 3, 7), 3)])
def test_step_pw_scalars_matches_oracle(shape, nscal):
    """MONC's other scalar scheme (centred flux form) in the fused step:
    scalar increments within 1e-13 of the oracle, momentum bitwise that of
    monc_step (the same PW pass)."""
    nx, ny, nz = shape
    say(f"step_pw_scalars {shape} nscal={nscal}")
    g, host = case(nx, ny, nz, nscal, seed=990 + nx + nscal)
    ref = O.step_pw_scalars([h.copy() for h in host], g, DT)
    T = torch()
    d = to_dev(host)
    prof = prof_dev(g)
    out = [T.full_like(x, float("nan")) for x in d]
    M.monc_step_pw_scalars(d, out, g.dx, g.dy, prof, DT)
    plain = [T.full_like(x, float("nan")) for x in d]
    M.monc_step(d, plain, g.dx, g.dy, prof, DT)
    T.cuda.synchronize()
    for f in range(3):
        assert T.equal(out[f][2:-2, 2:-2], plain[f][2:-2, 2:-2]), f
    for f in range(len(host)):
        o = out[f].cpu().numpy()
        inc = I.interior(o) - I.interior(host[f])
        inc_ref = I.interior(ref[f]) - I.interior(host[f])
        assert np.abs(inc - inc_ref).max() <= TOL * np.abs(inc_ref).max() + 1e-300, f


def test_full_size_pw_scalars_step_properties():
    """At the benchmark's size: momentum bitwise that of monc_step, and the
    centred scalar fluxes conserve each scalar's mass (sum of rhon dz times
    the increment vanishes to rounding)."""
    w = I.WORKLOADS["big1024"]
    say(f"full size pw scalars {w.nx}x{w.ny}x{w.nz}")
    T = torch()
    g = I.make_geometry(w.nx, w.ny, w.nz, w.dx, w.dx)
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    f = I.make_fields(g, w.nscal, w.seed, padded=True)
    d = [T.from_numpy(f[n]).to(dev()) for n in names]
    del f
    prof = prof_dev(g)
    a = [T.empty_like(x) for x in d]
    M.monc_step_pw_scalars(d, a, g.dx, g.dy, prof, w.dt)
    b = [T.empty_like(x) for x in d]
    M.monc_step(d, b, g.dx, g.dy, prof, w.dt)
    T.cuda.synchronize()
    for q in range(3):
        assert T.equal(a[q][2:-2, 2:-2], b[q][2:-2, 2:-2]), q
    del b
    mass = T.from_numpy(np.ascontiguousarray((1.0 / g.rdz) * g.rhon)).to(dev())
    for q in range(3, len(d)):
        inc = a[q][2:-2, 2:-2] - d[q][2:-2, 2:-2]
        total = float((inc * mass).sum())
        scale = float((inc.abs() * mass).sum())
        assert abs(total) <= 1e-12 * scale, (q, total, scale)
