"""Shared helpers of the GPU tests: move seeded inputs to the device, run the
oracle on the same inputs, and measure errors the way the parity bar states
them (per field, max |gpu - oracle| / max |oracle|)."""
import numpy as np

from oracle import pyoracle as O
from paper_2009_12850_amd import inputs as I


def torch():
    import torch as T
    return T


def dev():
    return torch().device("cuda:0")


def case(nx, ny, nz, nscal, seed, dx=50.0, dy=50.0, amp=5.0):
    g = I.make_geometry(nx, ny, nz, dx=dx, dy=dy)
    f = I.make_fields(g, nscal, seed, amp=amp)
    names = ["u", "v", "w"] + I.scalar_names(nscal)
    host = [O.halo_fill(I.pad(f[n])) for n in names]
    return g, host


def to_dev(arrs):
    T = torch()
    return [T.from_numpy(np.ascontiguousarray(a)).to(dev()) for a in arrs]


def prof_dev(g):
    return to_dev([g.rdz, g.rho, g.rhon])


def rel_err(gpu, ref, region=None):
    """max |g - o| / max |o| over the interior (or a region of it)."""
    a = I.interior(gpu)
    b = I.interior(ref)
    if region is not None:
        i0, i1, j0, j1 = region
        a = a[i0:i1, j0:j1]
        b = b[i0:i1, j0:j1]
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    if den == 0:
        return float(num)
    return float(num / den)


def oracle_tendencies(host, g, dt, region=None):
    u, v, w = host[:3]
    su, sv, sw = O.pw(u, v, w, g, region=region)
    ss = [O.tvd(u, v, w, q, g, dt, region=region) for q in host[3:]]
    return [su, sv, sw] + ss
