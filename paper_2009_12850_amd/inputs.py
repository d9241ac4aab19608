"""Seeded synthetic inputs for the MONC advection path.

This module only draws and lays out inputs; it holds none of the advection
arithmetic.  Both the CPU oracle (tests) and the HIP path (tests, bench) are fed
from it, so they always see the same arrays.

The paper's test case (the "tank experiment" of warm and cold bubbles,
Sec. 4) is not available, so fields are smooth random flows of the same kind:
each field is a normalised sum of 8 low-wavenumber modes plus small noise, on a
vertically stretched grid with an exponential reference density.

Recipe (all FP64, NumPy PCG64, fixed draw order):
  geometry  H = 3000 m, dz_k = dz0 * 1.02**k with dz0 = H*0.02/(1.02**nz - 1);
            z_{k+1/2} = cumulative sum of dz (top faces), zn_k = z_{k+1/2} - dz_k/2,
            rho_k = 1.2 exp(-z_{k+1/2}/8000), rhon_k = 1.2 exp(-zn_k/8000), rdz = 1/dz.
  modes     per field, 8 modes; each draws integer kx, ky in [-3, 3] (not both 0),
            vertical index m in {0,1,2}, phase ~ U[0, 2pi), weight r ~ U[0.5, 1];
            mode = r cos(2pi(kx x/Lx + ky y/Ly) + phase) Z_m(z), with
            Z_m = cos(pi m z/H) for u, v and scalars and sin(pi (m+1) z/H) for w;
            the sum is divided by sum(r).  Each field is evaluated at its own
            C-grid position (u on +x faces, v on +y faces, w on top faces,
            scalars at centres; cell centre x_i = (i+1/2) dx).
  values    u, v, w = amp*sum + N(0, 0.01^2), then w = 0 on the lid level;
            theta = 300 + 2*sum + N(0, 0.01^2);
            q_n = 1e-3 exp(0.5*sum + N(0, 0.01^2))  (positive, log-normal).
Field order is u, v, w, theta, q1, q2, ...; field number n draws its modes and
then its noise from its own generator, seeded with [seed, n], so that fields can
be generated in parallel threads.
"""
from __future__ import annotations

import dataclasses
import math
import threading

import numpy as np

H_TOP = 3000.0
STRETCH = 1.02


@dataclasses.dataclass
class Geometry:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    rdz: np.ndarray   # [nz] 1/dz_k
    rho: np.ndarray   # [nz] density at the top face of cell k
    rhon: np.ndarray  # [nz] density at the centre of cell k
    z_face: np.ndarray  # [nz] height of the top face of cell k
    z_centre: np.ndarray  # [nz] height of the centre of cell k


def make_geometry(nx: int, ny: int, nz: int, dx: float = 50.0, dy: float = 50.0,
                  height: float = H_TOP, ratio: float = STRETCH) -> Geometry:
    """Stretched vertical grid and exponential reference density profiles."""
    k = np.arange(nz, dtype=np.float64)
    dz0 = height * (ratio - 1.0) / (ratio ** nz - 1.0)
    dz = dz0 * ratio ** k
    z_face = np.cumsum(dz)
    z_centre = z_face - 0.5 * dz
    rho = 1.2 * np.exp(-z_face / 8000.0)
    rhon = 1.2 * np.exp(-z_centre / 8000.0)
    return Geometry(nx, ny, nz, float(dx), float(dy), 1.0 / dz, rho, rhon,
                    z_face, z_centre)


def _draw_modes(rng: np.random.Generator, nmodes: int = 8):
    modes = []
    for _ in range(nmodes):
        while True:
            kx, ky = (int(a) for a in rng.integers(-3, 4, size=2))
            if kx != 0 or ky != 0:
                break
        m = int(rng.integers(0, 3))
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        r = float(rng.uniform(0.5, 1.0))
        modes.append((kx, ky, m, phase, r))
    return modes


# The field generators run in threads; their one BLAS call (the matrix product
# below) is made one at a time, since concurrent calls into a multithreaded
# BLAS from several Python threads have returned corrupted products on hosts
# with many cores, which made the generated fields depend on thread timing.
_BLAS_LOCK = threading.Lock()


def _mode_sum(g: Geometry, modes, xs: np.ndarray, ys: np.ndarray,
              zs: np.ndarray, vertical_sine: bool) -> np.ndarray:
    """Normalised sum of the modes at positions xs (nx), ys (ny), zs (nz)."""
    lx, ly = g.nx * g.dx, g.ny * g.dy
    horiz = np.empty((g.nx * g.ny, len(modes)))
    vert = np.empty((len(modes), g.nz))
    for n, (kx, ky, m, phase, r) in enumerate(modes):
        ax = 2.0 * math.pi * kx * xs / lx
        by = 2.0 * math.pi * ky * ys / ly + phase
        # cos(a + b) = cos a cos b - sin a sin b, as an outer product
        h = np.outer(np.cos(ax), np.cos(by)) - np.outer(np.sin(ax), np.sin(by))
        horiz[:, n] = r * h.reshape(-1)
        if vertical_sine:
            vert[n] = np.sin(math.pi * (m + 1) * zs / H_TOP)
        else:
            vert[n] = np.cos(math.pi * m * zs / H_TOP)
    total_r = sum(md[4] for md in modes)
    with _BLAS_LOCK:
        prod = horiz @ vert
    return prod.reshape(g.nx, g.ny, g.nz) / total_r


def scalar_names(nscal: int):
    return ["th"] + [f"q{n}" for n in range(1, nscal)]


def _one_field(g: Geometry, name: str, n: int, seed: int, amp: float, noise: float,
               out: np.ndarray) -> None:
    rng = np.random.default_rng([seed, n])
    xc = (np.arange(g.nx) + 0.5) * g.dx
    xf = (np.arange(g.nx) + 1.0) * g.dx
    yc = (np.arange(g.ny) + 0.5) * g.dy
    yf = (np.arange(g.ny) + 1.0) * g.dy
    modes = _draw_modes(rng)
    if name == "u":
        s = _mode_sum(g, modes, xf, yc, g.z_centre, False)
    elif name == "v":
        s = _mode_sum(g, modes, xc, yf, g.z_centre, False)
    elif name == "w":
        s = _mode_sum(g, modes, xc, yc, g.z_face, True)
    else:
        s = _mode_sum(g, modes, xc, yc, g.z_centre, False)
    eps = rng.standard_normal(size=s.shape)
    eps *= noise
    if name in ("u", "v", "w"):
        s *= amp
        s += eps
        if name == "w":
            s[:, :, g.nz - 1] = 0.0
    elif name == "th":
        s *= 2.0
        s += eps
        s += 300.0
    else:
        s *= 0.5
        s += eps
        np.exp(s, out=s)
        s *= 1e-3
    out[...] = s


def make_fields(g: Geometry, nscal: int, seed: int, amp: float = 5.0,
                noise: float = 0.01, padded: bool = False, threads: int = 8,
                only=None) -> dict:
    """Fields u, v, w and nscal scalars (th, q1, ...), interior (nx, ny, nz)
    arrays, or [(nx+4)][(ny+4)][nz] arrays with a NaN halo if padded.  `only`
    restricts the output to the named fields (each field's draws depend only
    on the seed and its position in the full list, so a subset is the same)."""
    import concurrent.futures as cf
    names = ["u", "v", "w"] + scalar_names(nscal)
    index = {name: n for n, name in enumerate(names)}
    if only is not None:
        names = [n for n in names if n in only]
    out = {}
    views = {}
    for name in names:
        if padded:
            a = np.full((g.nx + 4, g.ny + 4, g.nz), np.nan)
            out[name] = a
            views[name] = a[2:g.nx + 2, 2:g.ny + 2, :]
        else:
            out[name] = np.empty((g.nx, g.ny, g.nz))
            views[name] = out[name]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(threads, len(names)))) as ex:
        futs = [ex.submit(_one_field, g, name, index[name], seed, amp, noise, views[name])
                for name in names]
        for f in futs:
            f.result()
    return out


def make_divfree_velocity(g: Geometry, seed: int, amp: float = 5.0,
                          padded: bool = False) -> dict:
    """u, v, w whose anelastic mass divergence vanishes to round-off.

    Built from three periodic potentials on the C-grid: A (x-z, at
    (x_{i+1/2}, y_j, z_{k+1/2})), B (y-z) and C (x-y corners), with A = B = 0
    on the lid level so that w vanishes there and on the ground:
        rhon_k u = -rdz_k (A_k - A_{k-1}) + rhon_k (C_j - C_{j-1})/dy
        rhon_k v = -rdz_k (B_k - B_{k-1}) - rhon_k (C_i - C_{i-1})/dx
        rho_k  w =  (A_i - A_{i-1})/dx + (B_j - B_{j-1})/dy,   A_{-1} = B_{-1} = 0.
    The result is scaled so that the largest speed component equals amp (the
    divergence is linear in the potentials, so scaling keeps it zero).
    Padded output: [(nx+4)][(ny+4)][nz] with a NaN halo.
    """
    import concurrent.futures as cf
    rng = np.random.default_rng(seed)
    xf = (np.arange(g.nx) + 1.0) * g.dx
    yc = (np.arange(g.ny) + 0.5) * g.dy
    xc = (np.arange(g.nx) + 0.5) * g.dx
    yf = (np.arange(g.ny) + 1.0) * g.dy
    modes = [_draw_modes(rng) for _ in range(3)]
    with cf.ThreadPoolExecutor(3) as ex:
        fa = ex.submit(_mode_sum, g, modes[0], xf, yc, g.z_face, True)
        fb = ex.submit(_mode_sum, g, modes[1], xc, yf, g.z_face, True)
        fc = ex.submit(_mode_sum, g, modes[2], xf, yf, g.z_centre, False)
        pa, pb, pc = fa.result(), fb.result(), fc.result()
    pa[:, :, g.nz - 1] = 0.0
    pb[:, :, g.nz - 1] = 0.0
    pa *= g.dx * g.rhon.max()
    pb *= g.dy * g.rhon.max()
    pc *= g.dx
    rdz = g.rdz[None, None, :]
    rhon = g.rhon[None, None, :]
    rho = g.rho[None, None, :]

    def alloc():
        if padded:
            a = np.full((g.nx + 4, g.ny + 4, g.nz), np.nan)
            return a, a[2:g.nx + 2, 2:g.ny + 2, :]
        a = np.empty((g.nx, g.ny, g.nz))
        return a, a

    def vertical(a, out):
        # -rdz_k (a_k - a_{k-1}) / rhon_k with a_{-1} = 0
        out[:, :, 0] = a[:, :, 0]
        np.subtract(a[:, :, 1:], a[:, :, :-1], out=out[:, :, 1:])
        out *= -rdz / rhon

    def u_part(out):
        vertical(pa, out)
        out += (pc - np.roll(pc, 1, axis=1)) / g.dy

    def v_part(out):
        vertical(pb, out)
        out -= (pc - np.roll(pc, 1, axis=0)) / g.dx

    def w_part(out):
        np.subtract(pa, np.roll(pa, 1, axis=0), out=out)
        out /= g.dx
        out += (pb - np.roll(pb, 1, axis=1)) / g.dy
        out /= rho
        out[:, :, g.nz - 1] = 0.0

    (U, u), (V, v), (W, w) = alloc(), alloc(), alloc()
    with cf.ThreadPoolExecutor(3) as ex:
        for f in [ex.submit(u_part, u), ex.submit(v_part, v), ex.submit(w_part, w)]:
            f.result()
    scale = amp / max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    for x in (u, v, w):
        x *= scale
    return {"u": U, "v": V, "w": W}


def pad(f: np.ndarray, fill: float = np.nan) -> np.ndarray:
    """Embed an interior (nx, ny, nz) array in the [(nx+4)][(ny+4)][nz] layout.

    The 2-deep lateral halo is left as `fill` (NaN by default, so that a kernel
    that reads an unfilled halo is caught)."""
    nx, ny, nz = f.shape
    out = np.full((nx + 4, ny + 4, nz), fill, dtype=np.float64)
    out[2:nx + 2, 2:ny + 2, :] = f
    return out


def interior(a: np.ndarray) -> np.ndarray:
    return a[2:-2, 2:-2, :]


# ---------------------------------------------------------------------------
# The five workloads (sizes, fields and seeds)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    nscal: int
    seed: int
    dt: float = 0.5
    steps: int = 1
    dx: float = 50.0
    divfree: bool = False   # divergence-free velocity (for runs of many steps)


WORKLOADS = {
    # one PW + TVD evaluation, 32^3, u v w th q1
    "tiny32": Workload("tiny32", 32, 32, 32, 2, seed=1),
    # 100 forward steps, 512x512x128, u v w th q1 q2 q3
    "steps512": Workload("steps512", 512, 512, 128, 4, seed=2, steps=100, divfree=True),
    # headline throughput, 1024x1024x128, u v w th q1
    "big1024": Workload("big1024", 1024, 1024, 128, 2, seed=3),
}


def make_workload(name: str, padded: bool = False):
    w = WORKLOADS[name]
    g = make_geometry(w.nx, w.ny, w.nz, w.dx, w.dx)
    if not w.divfree:
        return w, g, make_fields(g, w.nscal, w.seed, padded=padded)
    f = make_divfree_velocity(g, w.seed, padded=padded)
    f.update(make_fields(g, w.nscal, w.seed, padded=padded, only=scalar_names(w.nscal)))
    return w, g, f


def ensemble_members(n: int = 64, seed: int = 4):
    """Geometry draws for the uneven ensemble: nx, ny in {64, 96, ..., 256},
    nz in {64, 96}, wind amplitude ~ U[2, 10] m/s, dx = dy ~ U[25, 100] m,
    member m seeded 1000 + m."""
    rng = np.random.default_rng(seed)
    sizes = np.arange(64, 257, 32)
    members = []
    for m in range(n):
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        nz = int(rng.choice([64, 96]))
        amp = float(rng.uniform(2.0, 10.0))
        dx = float(rng.uniform(25.0, 100.0))
        members.append(dict(nx=nx, ny=ny, nz=nz, amp=amp, dx=dx, seed=1000 + m))
    return members
