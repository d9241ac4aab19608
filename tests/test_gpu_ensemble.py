"""GPU tests of the batched ensemble: members of uneven size advanced by the
persistent work-list kernel give bitwise the result of advancing each member
alone with monc_step_mixed; the captured graph replays bitwise what eager
launches compute; the autotuner writes and then reuses its cache."""
import json
import os
import sys
import tempfile

import numpy as np
import pytest

from gpu_util import dev, prof_dev, torch
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
        assert len(data) == 2
        for key, (ti, grid) in data.items():
            assert "gfx" in key and ti in (16, 32, 64, 128) and grid > 0
        ens2 = M.Ensemble(members, 2, tune_cache=path, tune=True)
        assert ens2.info()["ti"] == info["ti"]
        ens2.close()


def test_more_than_three_scalars_is_unsupported():
    members = make_members(nscal=4, seed0=1400)[:2]
    with pytest.raises(M.MoncError) as e:
        M.Ensemble(members, 4, tune=False)
    assert e.value.code == M.MONC_EUNSUPPORTED
