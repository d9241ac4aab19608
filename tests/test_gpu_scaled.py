"""GPU tests of the work-scaled PW kernel: one evaluation matches the FP64
oracle (FP32: within 1e-5), and any work factor gives bitwise the result of
one evaluation."""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()


def run(dtype, d, g, work):
    T = torch()
    out = [T.full_like(x, float("nan")) for x in d[:3]]
    M.monc_advect_pw_scaled(dtype, *d[:3], *out, g.dx, g.dy, prof_dev(g), work)
    T.cuda.synchronize()
    return out


@pytest.mark.parametrize("shape", [(32, 32, 32), (17, 23, 96), (5, 3, 2), (1, 1, 7), (9, 6, 128)])
def test_scaled_pw_matches_oracle_and_is_work_independent(shape):
    nx, ny, nz = shape
    say(f"pw_scaled {shape}")
    g, host = case(nx, ny, nz, 0, seed=700 + nx + nz)
    ref = O.pw(*host[:3], g)
    d = to_dev(host[:3])
    one = run(M.MONC_F64, d, g, 1)
    for n in range(3):
        assert rel_err(one[n].cpu().numpy(), ref[n]) <= 1e-13, n
    for work in (2, 7, 16):
        many = run(M.MONC_F64, d, g, work)
        for n in range(3):
            assert torch().equal(many[n][2:-2, 2:-2], one[n][2:-2, 2:-2]), (work, n)
    d32 = [x.float() for x in d]
    one32 = run(M.MONC_F32, d32, g, 1)
    for n in range(3):
        assert rel_err(one32[n].double().cpu().numpy(), ref[n]) <= 1e-5, n
    five32 = run(M.MONC_F32, d32, g, 5)
    for n in range(3):
        assert torch().equal(five32[n][2:-2, 2:-2], one32[n][2:-2, 2:-2]), n
