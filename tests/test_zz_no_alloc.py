"""The allocation-free step (monc_step_static: budget partials in the
library's static device scratch) against monc_step with a caller workspace,
through the C ABI: two calls in a row, the second on a smaller grid, each
bitwise equal to the workspace step (same kernels, same partial rows, same
summation order)."""
import sys

import numpy as np
import pytest

from gpu_util import case, dev, prof_dev, to_dev, torch
from paper_2009_12850_amd import _lib as M

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(nx, ny, nz, nscal, seed):
    T = torch()
    g, host = case(nx, ny, nz, nscal, seed=seed)
    d = to_dev(host)
    prof = prof_dev(g)
    ref = [T.full_like(x, float("nan")) for x in d]
    got = [T.full_like(x, float("nan")) for x in d]
    b_ref = T.zeros(M.MONC_NBUDGET, dtype=T.float64, device=dev())
    b_got = T.full((M.MONC_NBUDGET,), float("nan"), dtype=T.float64, device=dev())
    ws = T.empty(M.monc_step_workspace_bytes(nx, ny, nz, nscal), dtype=T.uint8, device=dev())
    M.monc_step(d, ref, g.dx, g.dy, prof, 0.5, b_ref, ws)
    M.monc_step_static(d, got, g.dx, g.dy, prof, 0.5, b_got)
    T.cuda.synchronize()
    for n, (a, b) in enumerate(zip(got, ref)):
        ai, bi = a[2:-2, 2:-2].cpu().numpy(), b[2:-2, 2:-2].cpu().numpy()
        assert np.array_equal(ai, bi), (nx, ny, nz, n)
    assert np.array_equal(b_got.cpu().numpy(), b_ref.cpu().numpy())
    assert M.monc_budgets_check(b_got.cpu().numpy()) == M.MONC_OK


def test_static_step_equals_workspace_step_twice():
    say("static step 72x60x100, 3 scalars")
    run_both(72, 60, 100, 3, seed=901)
    say("static step 20x14x32, 2 scalars")
    run_both(20, 14, 32, 2, seed=902)
