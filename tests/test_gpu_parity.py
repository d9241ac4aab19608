"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar (FP64): per field max |gpu - oracle| / max |oracle| <= 1e-13 for the
tendencies; the step compares increments (new - old) at the same bar; halo
fill and repeat runs are bitwise.
"""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, oracle_tendencies, prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-13

SHAPES = [
    (32, 32, 32),   # the tiny workload's grid
    (37, 29, 45),   # ragged in every direction
    (5, 3, 2),      # two levels only: ground and lid faces meet
    (1, 1, 7),      # one column: periodic with itself
    (2, 7, 64),
    (16, 9, 128),
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()
    T = torch()
    assert T.cuda.is_available()


@pytest.mark.parametrize("shape", SHAPES + [(3, 2, 5)])
def test_halo_fill_bitwise(shape):
    nx, ny, nz = shape
    say(f"halo {shape}")
    rng = np.random.default_rng(7)
    arrs = [I.pad(rng.standard_normal((nx, ny, nz))) for _ in range(3)]
    d = to_dev(arrs)
    M.monc_halo_fill(d)
    T = torch()
    T.cuda.synchronize()
    for a, h in zip(d, arrs):
        np.testing.assert_array_equal(a.cpu().numpy(), O.halo_fill(h))
    # float32 and bfloat16-bit storage use the same copy
    d32 = [T.from_numpy(I.pad(rng.standard_normal((nx, ny, nz))).astype(np.float32)).to(dev())
           for _ in range(2)]
    ref32 = [O.halo_fill(a.cpu().numpy().astype(np.float64)) for a in d32]
    M.monc_halo_fill(d32)
    for a, r in zip(d32, ref32):
        np.testing.assert_array_equal(a.cpu().numpy().astype(np.float64), r)
    d16 = [a.to(T.bfloat16).view(T.int16).contiguous() for a in d32]
    ref16 = [O.halo_fill(a.view(T.bfloat16).float().cpu().numpy().astype(np.float64))
             for a in d16]
    M.monc_halo_fill(d16)
    for a, r in zip(d16, ref16):
        np.testing.assert_array_equal(
            a.view(T.bfloat16).float().cpu().numpy().astype(np.float64), r)


@pytest.mark.parametrize("shape", SHAPES)
def test_pw_and_tvd_match_oracle(shape):
    nx, ny, nz = shape
    say(f"pw/tvd {shape}")
    g, host = case(nx, ny, nz, 2, seed=100 + nx)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    d = to_dev(host)
    prof = prof_dev(g)
    T = torch()
    su, sv, sw = (T.zeros_like(d[0]) for _ in range(3))
    M.monc_advect_pw(d[0], d[1], d[2], su, sv, sw, g.dx, g.dy, prof)
    sq = [T.zeros_like(d[0]) for _ in range(2)]
    M.monc_advect_tvd(d[0], d[1], d[2], d[3:], sq, g.dx, g.dy, prof, dt)
    T.cuda.synchronize()
    got = [su, sv, sw] + sq
    for n, (a, b) in enumerate(zip(got, ref)):
        e = rel_err(a.cpu().numpy(), b)
        assert e <= TOL64, f"field {n}: {e:.3e}"
    # the lid row of sw is exactly zero
    assert np.all(I.interior(sw.cpu().numpy())[:, :, -1] == 0)


@pytest.mark.parametrize("shape", [(32, 32, 32), (37, 29, 45), (1, 1, 7)])
def test_fused_advect_f64_matches_oracle(shape):
    nx, ny, nz = shape
    say(f"fused {shape}")
    g, host = case(nx, ny, nz, 3, seed=200 + nx)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    d = to_dev(host)
    T = torch()
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), dt)
    T.cuda.synchronize()
    for n, (a, b) in enumerate(zip(out, ref)):
        e = rel_err(a.cpu().numpy(), b)
        assert e <= TOL64, f"field {n}: {e:.3e}"


def run_step(d, g, dt, with_budgets=True):
    T = torch()
    out = [T.full_like(x, float("nan")) for x in d]
    nx, ny, nz = d[0].shape[0] - 4, d[0].shape[1] - 4, d[0].shape[2]
    b = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev()) if with_budgets else None
    ws = (T.empty(M.monc_step_workspace_bytes(nx, ny, nz, len(d) - 3), dtype=T.uint8,
                  device=dev()) if with_budgets else None)
    M.monc_step(d, out, g.dx, g.dy, prof_dev(g), dt, b, ws)
    T.cuda.synchronize()
    return out, (b.cpu().numpy() if with_budgets else None)


@pytest.mark.parametrize("shape", [(32, 32, 32), (37, 29, 45), (5, 3, 2)])
def test_step_and_budgets_match_oracle(shape):
    nx, ny, nz = shape
    say(f"step {shape}")
    g, host = case(nx, ny, nz, 2, seed=300 + nx)
    dt = 0.5
    ref = O.step([h.copy() for h in host], g, dt)
    d = to_dev(host)
    out, b = run_step(d, g, dt)
    for n in range(len(host)):
        inc_g = out[n].cpu().numpy() - host[n]
        inc_o = ref[n] - host[n]
        e = rel_err(inc_g, inc_o)
        assert e <= TOL64, f"field {n}: {e:.3e}"
    assert np.all(I.interior(out[2].cpu().numpy())[:, :, -1] == 0)
    check_budgets(b, host, g, dt, 2)


def check_budgets(b, host, g, dt, nscal):
    """The step's budgets against the oracle's budgets of the same evaluation
    (small grids: sums within 1e-13 of their sums of absolute terms)."""
    tend = oracle_tendencies(host, g, dt)
    ob, sc = O.budgets(*host[:3], *tend[:3], host[3:], tend[3:], g)
    gb = M.budgets_dict(b, nscal)
    for name in ["C_u", "C_v", "C_w", "P_u", "Q_u", "P_v", "Q_v", "P_w", "Q_w"]:
        assert abs(gb[name] - ob[name]) <= 1e-13 * sc[name] + 1e-300, name
    for s in range(nscal):
        scale = np.sum(np.abs(I.interior(tend[3 + s])) * (g.rhon / g.rdz)[None, None, :])
        assert abs(gb[f"C_s{s}"] - ob[f"C_s{s}"]) <= 1e-13 * scale
        assert abs(gb[f"M_s{s}"] - ob[f"M_s{s}"]) <= 1e-13 * abs(ob[f"M_s{s}"])
        assert gb[f"min_s{s}"] == ob[f"min_s{s}"]
    cmax = O.max_courant(*host[:3], g, dt)
    assert abs(gb["courant"] - cmax) <= 1e-15 * cmax
    assert gb["nonfinite"] == 0
    assert M.monc_budgets_check(b) == M.MONC_OK


def test_multistep_trajectory_matches_oracle():
    """30 steps of a 48x40x32 state with four scalars against 30 oracle steps."""
    say("trajectory 48x40x32 x30")
    g, host = case(48, 40, 32, 4, seed=400)
    dt = 0.5
    ref = [h.copy() for h in host]
    for _ in range(30):
        ref = O.step(ref, g, dt)
    d = to_dev(host)
    for _ in range(30):
        d, _b = run_step(d, g, dt, with_budgets=False)
    for n in range(len(host)):
        e = rel_err(d[n].cpu().numpy() - host[n], ref[n] - host[n])
        assert e <= 1e-11, f"field {n}: {e:.3e}"


def test_repeat_runs_are_bitwise_equal():
    say("determinism")
    g, host = case(37, 29, 45, 2, seed=500)
    d = to_dev(host)
    o1, b1 = run_step(d, g, 0.5)
    o2, b2 = run_step(d, g, 0.5)
    for a, b in zip(o1, o2):
        assert torch().equal(a[2:-2, 2:-2], b[2:-2, 2:-2])
    np.testing.assert_array_equal(b1, b2)


def test_translation_invariance_on_gpu():
    say("translation")
    g, host = case(24, 20, 16, 2, seed=510)
    rolled = [O.halo_fill(I.pad(np.roll(I.interior(h), (5, -3), axis=(0, 1))))
              for h in host]
    T = torch()
    outs = []
    for src in (host, rolled):
        d = to_dev(src)
        out = [T.zeros_like(x) for x in d]
        M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), 0.5)
        T.cuda.synchronize()
        outs.append([I.interior(o.cpu().numpy()) for o in out])
    for a, b in zip(*outs):
        np.testing.assert_array_equal(np.roll(a, (5, -3), axis=(0, 1)), b)


def test_courant_and_nonfinite_flags():
    say("flags")
    g, host = case(16, 16, 16, 2, seed=520)
    T = torch()
    fast = [h.copy() for h in host]
    fast[0] = O.halo_fill(I.pad(I.interior(host[0]) * 40.0))  # |u| dt/dx ~ 2
    _, b = run_step(to_dev(fast), g, 0.5)
    assert b[M.B_COURANT] > 1.0
    assert M.monc_budgets_check(b) == M.MONC_ECFL
    bad = [h.copy() for h in host]
    bad[4][5, 6, 3] = np.nan
    out, b = run_step(to_dev(bad), g, 0.5)
    # the count is that of the non-finite values the step wrote
    written = sum(int(np.sum(~np.isfinite(I.interior(o.cpu().numpy())))) for o in out)
    assert written >= 1
    assert b[M.B_NONFINITE] == written
    assert M.monc_budgets_check(b) == M.MONC_ENONFINITE
    del T


def test_big1024_subdomains_match_oracle():
    """The headline grid (1024 x 1024 x 128, u v w th q1) evaluated whole on the
    GPU; the oracle computes a 128 x 128 column block and the blocks that touch
    the periodic seams."""
    say("big1024 tendencies")
    w, g, f = I.make_workload("big1024")
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    T = torch()
    hosts = [O.halo_fill(I.pad(f.pop(n))) for n in names]
    d = [T.from_numpy(h).to(dev()) for h in hosts]
    out = [T.empty_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), w.dt)
    T.cuda.synchronize()
    regions = [(0, 128, 0, 128), (1020, 1024, 0, 8), (0, 8, 1018, 1024),
               (1021, 1024, 1021, 1024), (500, 516, 700, 716)]
    for (i0, i1, j0, j1) in regions:
        ref = oracle_tendencies(hosts, g, w.dt, region=(i0, i1, j0, j1))
        for n, o in enumerate(out):
            got = o[i0 + 2:i1 + 2, j0 + 2:j1 + 2].cpu().numpy()
            exp = ref[n][i0 + 2:i1 + 2, j0 + 2:j1 + 2]
            e = np.abs(got - exp).max() / np.abs(exp).max()
            assert e <= TOL64, f"region {(i0, i1, j0, j1)} field {n}: {e:.3e}"


def test_big1024_budgeted_step_matches_oracle():
    """The launch the benchmark times: monc_step with budgets on 1024 x 1024 x
    128 (u v w th q1), inputs straight from the generator (halos never
    filled), in the benchmark's configuration.  Increments on five column
    blocks (the periodic seams among them) against the oracle; every budget
    entry against the oracle's budgets of the whole domain.

    Bars (derived from the arithmetic): the GPU forms f + dt s with one
    rounding (a fused multiply-add) and the oracle rounds dt s first, so the
    new values may differ by one unit in the last place of the new value on
    top of the source terms' 1e-13; sums of N terms taken in two orders differ
    by at most (chain lengths) x 2^-53 x sum |terms| (the oracle's chain is
    one x-slab, ny nz terms, then nx slabs; the GPU's is one lane's planes,
    then a wave, a workgroup and the partial rows)."""
    say("big1024 budgeted step")
    w, g, f = I.make_workload("big1024")
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    T = torch()
    raw = [I.pad(f.pop(n)) for n in names]  # NaN halos, as the benchmark hands them over
    d = [T.from_numpy(h).to(dev()) for h in raw]
    hosts = [O.halo_fill(h) for h in raw]
    del raw
    out = [T.empty_like(x) for x in d]
    b = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev())
    ws = T.empty(M.monc_step_workspace_bytes(w.nx, w.ny, w.nz, w.nscal), dtype=T.uint8,
                 device=dev())
    M.monc_step(d, out, g.dx, g.dy, prof_dev(g), w.dt, b, ws)
    T.cuda.synchronize()
    del d
    regions = [(0, 128, 0, 128), (1020, 1024, 0, 8), (0, 8, 1018, 1024),
               (1021, 1024, 1021, 1024), (500, 516, 700, 716)]
    for (i0, i1, j0, j1) in regions:
        ref = oracle_tendencies(hosts, g, w.dt, region=(i0, i1, j0, j1))
        for n, o in enumerate(out):
            sl = (slice(i0 + 2, i1 + 2), slice(j0 + 2, j1 + 2))
            old = hosts[n][sl]
            new_o = old + w.dt * ref[n][sl]
            if n == 2:
                new_o[:, :, -1] = 0.0
            got = o[sl].cpu().numpy()
            inc_o = new_o - old
            bar = TOL64 * np.abs(inc_o).max() + np.spacing(np.abs(new_o).max())
            err = np.abs((got - old) - inc_o).max()
            assert err <= bar, f"region {(i0, i1, j0, j1)} field {n}: {err:.3e} > {bar:.3e}"
    del out
    say("  oracle budgets of the whole domain")
    tend = oracle_tendencies(hosts, g, w.dt)
    ob, sc = O.budgets(*hosts[:3], *tend[:3], hosts[3:], tend[3:], g)
    gb = M.budgets_dict(b.cpu().numpy(), w.nscal)
    chains = (w.ny * w.nz + w.nx + 4096) * 2.0 ** -53
    for name in ["C_u", "C_v", "C_w", "P_u", "Q_u", "P_v", "Q_v", "P_w", "Q_w"]:
        scale = sc[name]
        bar = (chains + TOL64) * scale
        assert abs(gb[name] - ob[name]) <= bar, (name, gb[name], ob[name], bar)
    mass = (g.rhon / g.rdz)[None, None, :]
    for s in range(w.nscal):
        t = I.interior(tend[3 + s])
        scale = np.sum(np.abs(t) * mass)
        assert abs(gb[f"C_s{s}"] - ob[f"C_s{s}"]) <= (chains + TOL64) * scale, s
        assert abs(gb[f"M_s{s}"] - ob[f"M_s{s}"]) <= chains * abs(ob[f"M_s{s}"]), s
        assert gb[f"min_s{s}"] == ob[f"min_s{s}"], s
    cmax = O.max_courant(*hosts[:3], g, w.dt)
    assert abs(gb["courant"] - cmax) <= 1e-15 * cmax
    assert gb["nonfinite"] == 0
    say("  budgets " + " ".join(f"{k}={v:.3e}" for k, v in gb.items()))


@pytest.mark.parametrize("nscal,nz,budgets", [(1, 128, False), (1, 128, True), (2, 128, False),
                                             (3, 96, False), (4, 128, False), (1, 64, False),
                                             (4, 64, True), (5, 128, True)])
def test_step_with_unfilled_halos_every_grouping(nscal, nz, budgets):
    """NaN halos, every scalar grouping (passes of 2 or 3 scalars; with budgets
    3 on one-chunk columns, 2 on two-chunk ones), one and two z-chunks, with
    and without budgets: the step and its budgets match the oracle.  ny = 14
    leaves the last tile columns past ny that read NaN and store nothing; their
    sums must not reach the budgets."""
    say(f"unfilled halos step nscal={nscal} nz={nz} budgets={budgets}")
    g, host = case(20, 14, nz, nscal, seed=540 + nscal + nz)
    dt = 0.5
    ref = O.step([h.copy() for h in host], g, dt)
    poisoned = [I.pad(I.interior(h)) for h in host]
    o, b = run_step(to_dev(poisoned), g, dt, with_budgets=budgets)
    for n in range(3 + nscal):
        got = o[n].cpu().numpy()
        assert np.all(np.isfinite(I.interior(got))), n
        assert rel_err(got - host[n], ref[n] - host[n]) <= TOL64, n
    if budgets:
        check_budgets(b, host, g, dt, nscal)


def test_halos_are_never_read():
    """Inputs with NaN halos (never filled) give the oracle's result: periodic
    neighbours are read at wrapped interior indices."""
    say("unfilled halos")
    g, host = case(20, 14, 40, 2, seed=530)
    dt = 0.5
    ref = oracle_tendencies(host, g, dt)
    poisoned = [I.pad(I.interior(h)) for h in host]  # NaN halos
    T = torch()
    d = to_dev(poisoned)
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof_dev(g), dt)
    T.cuda.synchronize()
    for n, (a, b) in enumerate(zip(out, ref)):
        assert rel_err(a.cpu().numpy(), b) <= TOL64, n
    step_ref = O.step([h.copy() for h in host], g, dt)
    o, b = run_step(to_dev(poisoned), g, dt)
    for n in range(5):
        assert rel_err(o[n].cpu().numpy() - host[n], step_ref[n] - host[n]) <= TOL64, n
    assert b[M.B_NONFINITE] == 0
