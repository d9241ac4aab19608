"""GPU parity of the TVD face flux at the limiter's edge cases.

The kernels evaluate the ULTIMATE-limited QUICKEST face value in an offset
arrangement (C plus a clamped offset, in the frame where the near difference
is non-negative) that equals the oracle's textbook form for Courant numbers
up to 1.  These inputs aim at the places where the two arrangements could
part: Courant numbers of exactly 0 and exactly 1 along x, y and z (spacings,
time step and velocities are powers of two, so c is exact), piecewise-constant
scalars (ties: zero differences on either side), monotone ramps where the
limiter clamps, and isolated extrema.  FP64 against the oracle at 1e-13 per
field (max |gpu - oracle| / max |oracle|), FP32 at 1e-5.
"""
import sys

import numpy as np
import pytest

from gpu_util import prof_dev, rel_err, to_dev, torch
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu

DT = 0.5
DX = 64.0   # dx / dt = 128 exactly
DZ = 32.0   # uniform layers: 1/(dt rdzn) = 64 exactly


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()


def geometry(nx, ny, nz):
    rdz = np.full(nz, 1.0 / DZ)
    zf = DZ * np.arange(1, nz + 1)
    zc = zf - DZ / 2
    rho = 1.2 * np.exp(-zf / 8000.0)
    rhon = 1.2 * np.exp(-zc / 8000.0)
    return I.Geometry(nx, ny, nz, DX, DX, rdz, rho, rhon, zf, zc)


def fields(nx, ny, nz, seed, kind):
    rng = np.random.default_rng(seed)
    sh = (nx, ny, nz)
    # Courant numbers drawn from {-1, -1/2, 0, 1/2, 1} on every face
    cx, cy, cz = (rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], size=sh) for _ in range(3))
    u = cx * DX / DT
    v = cy * DX / DT
    w = cz * DZ / DT
    w[:, :, -1] = 0.0
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    if kind == "ties":
        phi = np.round(rng.uniform(0, 3, sh)) * 0.5 + 1.0
    elif kind == "ramps":
        phi = 1.0 + 0.1 * (np.minimum(i, nx - 1 - i) + 2 * np.minimum(j, ny - 1 - j)
                           + 3 * np.minimum(k, nz - 1 - k))
    else:  # isolated extrema on a smooth background
        phi = 2.0 + 0.01 * np.sin(i) * np.cos(j) + 0.001 * k
        mask = rng.uniform(size=sh) < 0.05
        phi = np.where(mask, phi + rng.choice([-1.0, 1.0], size=sh), phi)
    th = 300.0 + phi
    return [O.halo_fill(I.pad(a)) for a in (u, v, w, th, phi)]


@pytest.mark.parametrize("kind", ["ties", "ramps", "extrema"])
@pytest.mark.parametrize("shape", [(16, 12, 24), (9, 7, 70)])
def test_limiter_edge_cases_match_oracle(kind, shape):
    nx, ny, nz = shape
    say(f"limiter {kind} {shape}")
    g = geometry(nx, ny, nz)
    host = fields(nx, ny, nz, seed={"ties": 11, "ramps": 12, "extrema": 13}[kind] + nx, kind=kind)
    assert O.max_courant(*host[:3], g, DT) == 1.0
    ref = [O.tvd(*host[:3], q, g, DT) for q in host[3:]]
    T = torch()
    d = to_dev(host)
    prof = prof_dev(g)
    out = [T.zeros_like(x) for x in d]
    M.monc_advect(M.MONC_F64, d, out, g.dx, g.dy, prof, DT)
    T.cuda.synchronize()
    for s in range(2):
        e = rel_err(out[3 + s].cpu().numpy(), ref[s])
        assert e <= 1e-13, f"scalar {s}: {e:.3e}"
    # the step's scalar increments too (state in FP64, same face fluxes)
    st = [T.full_like(x, float("nan")) for x in d]
    M.monc_step(d, st, g.dx, g.dy, prof, DT)
    T.cuda.synchronize()
    for s in range(2):
        inc = I.interior(st[3 + s].cpu().numpy()) - I.interior(host[3 + s])
        refinc = DT * I.interior(ref[s])
        assert np.abs(inc - refinc).max() <= 1e-13 * np.abs(refinc).max() + 1e-12 * np.abs(
            I.interior(host[3 + s])).max() * np.finfo(float).eps
    # FP32 working copies (scalars as anomalies from phi0)
    phi0 = [300.0, 0.0]
    work = [T.empty(x.shape, dtype=T.float32, device=x.device) for x in d]
    M.monc_cast_working(M.MONC_F32, d, work, [0.0, 0.0, 0.0] + phi0)
    out32 = [T.zeros(x.shape, dtype=T.float32, device=x.device) for x in d]
    M.monc_advect(M.MONC_F32, work, out32, g.dx, g.dy, prof, DT, phi0=phi0)
    T.cuda.synchronize()
    for s in range(2):
        e = rel_err(out32[3 + s].double().cpu().numpy(), ref[s])
        assert e <= 1e-5, f"fp32 scalar {s}: {e:.3e}"
