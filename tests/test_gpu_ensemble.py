"""GPU tests of the batched ensemble: members of uneven size advanced by the
persistent work-list kernel give bitwise the result of advancing each member
alone with monc_step_mixed; the captured graph replays bitwise what eager
launches compute; the autotuner writes and then reuses its cache; every
member against the FP64 oracle with its budgets."""
import json
import os
import sys
import tempfile

import numpy as np
import pytest

from gpu_util import dev, oracle_tendencies, prof_dev, rel_err, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu

SHAPES = [(40, 33, 64), (24, 56, 96), (64, 16, 32), (17, 23, 100), (32, 32, 64), (9, 70, 128)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_members(nscal=2, seed0=1000):
    T = torch()
    members = []
    for n, (nx, ny, nz) in enumerate(SHAPES):
        dx = 30.0 + 10 * n
        g = I.make_geometry(nx, ny, nz, dx=dx, dy=dx)
        f = I.make_fields(g, nscal, seed0 + n, amp=2.0 + n, padded=True)
        names = ["u", "v", "w"] + I.scalar_names(nscal)
        s0 = [T.from_numpy(f[k]).to(dev()) for k in names]
        s1 = [T.full_like(x, float("nan")) for x in s0]
        members.append(dict(state0=s0, state1=s1, prof=prof_dev(g), dx=dx, dy=dx, dt=0.5,
                            phi0=[300.0] + [0.0] * (nscal - 1), g=g))
    return members


def alone(mem, nsteps):
    T = torch()
    A = [x.clone() for x in mem["state0"]]
    B = [T.full_like(x, float("nan")) for x in A]
    for _ in range(nsteps):
        M.monc_step_mixed(A, B, mem["phi0"], mem["dx"], mem["dy"], mem["prof"], mem["dt"])
        A, B = B, A
    T.cuda.synchronize()
    return A


def current(mem, parity):
    return mem["state0"] if parity == 0 else mem["state1"]


def test_ensemble_equals_members_alone_bitwise():
    say("ensemble vs alone")
    T = torch()
    members = make_members()
    refs = [alone(m, 3) for m in members]
    ens = M.Ensemble(members, 2, tune_cache=None, tune=False)
    ens.run(3)
    T.cuda.synchronize()
    for mem, ref in zip(members, refs):
        got = current(mem, ens.parity)
        for a, b in zip(got, ref):
            assert T.equal(a[2:-2, 2:-2], b[2:-2, 2:-2])
    ens.close()


def test_graph_replay_equals_eager_steps():
    say("graph vs eager")
    T = torch()
    m1 = make_members(seed0=1100)
    m2 = make_members(seed0=1100)
    e1 = M.Ensemble(m1, 2, tune=False)
    e2 = M.Ensemble(m2, 2, tune=False)
    e1.run(4)
    e1.run(4)  # replay of the same graph
    for _ in range(8):
        e2.step()
    T.cuda.synchronize()
    assert e1.parity == e2.parity == 0
    for a, b in zip(m1, m2):
        for x, y in zip(current(a, 0), current(b, 0)):
            assert T.equal(x[2:-2, 2:-2], y[2:-2, 2:-2])
    e1.close()
    e2.close()


def test_odd_step_counts_track_parity():
    T = torch()
    members = make_members(seed0=1200)
    refs = [alone(m, 5) for m in members]
    ens = M.Ensemble(members, 2, tune=False)
    ens.run(3)
    ens.run(2)
    T.cuda.synchronize()
    assert ens.parity == 1
    for mem, ref in zip(members, refs):
        for a, b in zip(current(mem, 1), ref):
            assert T.equal(a[2:-2, 2:-2], b[2:-2, 2:-2])
    ens.close()


def test_autotuner_writes_and_reuses_cache():
    say("autotune")
    members = make_members(seed0=1300)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        ens = M.Ensemble(members, 2, tune_cache=path, tune=True)
        info = ens.info()
        ens.close()
        data = json.load(open(path))
        # one entry: the single work list of both column-height classes
        assert len(data) == 1
        for key, (ti, grid) in data.items():
            assert "gfx" in key and "nscal2" in key and ti in (16, 32, 64, 128) and grid > 0
        assert info["nitems"][0] > 0 and info["nitems"][1] > 0  # both classes in the list
        ens2 = M.Ensemble(members, 2, tune_cache=path, tune=True)
        assert ens2.info()["ti"] == info["ti"] and ens2.info()["grid"] == info["grid"]
        ens2.close()


def test_more_than_three_scalars_is_unsupported():
    members = make_members(nscal=4, seed0=1400)[:2]
    with pytest.raises(M.MoncError) as e:
        M.Ensemble(members, 4, tune=False)
    assert e.value.code == M.MONC_EUNSUPPORTED


ORACLE_SHAPES = [(40, 33, 64), (24, 56, 96), (17, 23, 100), (9, 70, 128), (33, 9, 32)]


def test_ensemble_members_match_oracle_with_budgets():
    """Every member of an uneven ensemble (three scalars; 32, 64, 96, 100 and
    128 levels, so both column-height classes) against the FP64 oracle after
    one and after three steps, at the mixed step's bar (FP32 source terms:
    increments within 1e-5 of the oracle's, relative to their largest value),
    and every member's FP64 budgets of each step against the oracle's budgets
    of the state that step read (the Q sides of the energy identity are
    left out: they take the cell divergence from FP32 arithmetic)."""
    say("ensemble vs oracle")
    T = torch()
    nscal = 3
    members, hosts = [], []
    for n, (nx, ny, nz) in enumerate(ORACLE_SHAPES):
        dx = 25.0 + 15.0 * n
        g = I.make_geometry(nx, ny, nz, dx=dx, dy=dx)
        f = I.make_fields(g, nscal, 1500 + n, amp=2.0 + 2.0 * n, padded=True)
        names = ["u", "v", "w"] + I.scalar_names(nscal)
        h = [O.halo_fill(f[k]) for k in names]
        hosts.append(h)
        s0 = [T.from_numpy(x.copy()).to(dev()) for x in h]
        s1 = [T.full_like(x, float("nan")) for x in s0]
        members.append(dict(state0=s0, state1=s1, prof=prof_dev(g), dx=dx, dy=dx, dt=0.5,
                            phi0=[300.0, 1e-3, 1e-3], g=g))
    ens = M.Ensemble(members, nscal, tune=False)
    bud = T.zeros((2, len(members), M.MONC_NBUDGET), dtype=T.float64, device=dev())
    ens.set_budgets(bud)

    def check_budgets(b, state, mem):
        g = mem["g"]
        tend = oracle_tendencies(state, g, mem["dt"])
        ob, _ = O.budgets(*state[:3], *tend[:3], state[3:], tend[3:], g)
        gb = M.budgets_dict(b, nscal)
        # FP32 source terms within 1e-5 max|s| of the oracle's at every point
        # bound each weighted sum's error by 1e-5 max|s| sum(weight); the
        # weights are rhon dz (u, v, scalars), rho dzn (w, levels below the
        # lid), times |u|, |v|, |w| for the energy production P
        cell = np.broadcast_to((g.rhon / g.rdz)[None, None, :], (g.nx, g.ny, g.nz))
        dzn = 0.5 * (1.0 / g.rdz[:-1] + 1.0 / g.rdz[1:])
        wcell = np.zeros(g.nz)
        wcell[:-1] = g.rho[:-1] * dzn
        wcell = np.broadcast_to(wcell[None, None, :], (g.nx, g.ny, g.nz))
        for c, q, wt in (("u", 0, cell), ("v", 1, cell), ("w", 2, wcell)):
            smax = np.abs(I.interior(tend[q])).max()
            vel = np.abs(I.interior(state[q]))
            assert abs(gb[f"C_{c}"] - ob[f"C_{c}"]) <= 1e-5 * smax * wt.sum(), c
            assert abs(gb[f"P_{c}"] - ob[f"P_{c}"]) <= 1e-5 * smax * (wt * vel).sum(), c
        for s in range(nscal):
            smax = np.abs(I.interior(tend[3 + s])).max()
            assert abs(gb[f"C_s{s}"] - ob[f"C_s{s}"]) <= 1e-5 * smax * cell.sum(), s
            # M_s and min_s come from the FP64 state itself
            assert abs(gb[f"M_s{s}"] - ob[f"M_s{s}"]) <= 1e-13 * abs(ob[f"M_s{s}"]), s
            assert gb[f"min_s{s}"] == ob[f"min_s{s}"], s
        cmax = O.max_courant(*state[:3], g, mem["dt"])
        assert abs(gb["courant"] - cmax) <= 1e-15 * cmax
        assert gb["nonfinite"] == 0

    ens.run(1)
    T.cuda.synchronize()
    assert ens.parity == 1
    bh = bud.cpu().numpy()
    ref1 = []
    for m, (mem, h) in enumerate(zip(members, hosts)):
        ref = O.step([x.copy() for x in h], mem["g"], mem["dt"])
        ref1.append(ref)
        for n in range(3 + nscal):
            e = rel_err(mem["state1"][n].cpu().numpy() - h[n], ref[n] - h[n])
            assert e <= 1e-5, (m, n, e)
        check_budgets(bh[0, m], h, mem)
    ens.run(2)
    T.cuda.synchronize()
    assert ens.parity == 1
    bh = bud.cpu().numpy()
    for m, (mem, h) in enumerate(zip(members, hosts)):
        g = mem["g"]
        ref = ref1[m]
        for _ in range(2):
            ref = O.step(ref, g, mem["dt"])
        for n in range(3 + nscal):
            e = rel_err(mem["state1"][n].cpu().numpy() - h[n], ref[n] - h[n])
            assert e <= 1e-5, (m, n, e)
        # slot 1 holds the budgets of the state after two steps (buffer 0 now)
        mid = [O.halo_fill(x.cpu().numpy()) for x in mem["state0"]]
        check_budgets(bh[1, m], mid, mem)
    ens.close()
