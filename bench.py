"""Benchmark of the MONC advection step on one MI355X.

One step = one call of monc_step on the 1024 x 1024 x 128 grid with u, v, w,
theta, q1 in FP64: Piacsek-Williams momentum + ULTIMATE/TVD scalar source
terms (periodic neighbours read at wrapped indices), forward update into the
second buffer, and the FP64 budgets.  Inputs are seeded synthetic fields,
resident in HBM before timing starts.

Prints one JSON line: grid-point updates per second (nx*ny*nz per step),
the roofline of the dominant kernel (HBM-bound stencil, algorithmic bytes =
one read and one write of every field), the oracle timed on the host cores on
a bounded sample, and the other forms: FP32 / BF16 tendencies, the mixed
step, the batched ensemble, and the learned coarse-grid correction.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E

# Sources of the dominant kernel (the timed launch: the FP64 step with budgets):
# a measured HBM traffic figure is reported
# only while these files are unchanged since the counters were taken.
KERNEL_SOURCES = ["paper_2009_12850_amd/build.py",  # compile flags
                  "paper_2009_12850_amd/csrc/march.hpp",
                  "paper_2009_12850_amd/csrc/march_launch.hpp",
                  "paper_2009_12850_amd/csrc/march_step64.hip",
                  "paper_2009_12850_amd/csrc/monc_scheme.hpp",
                  "paper_2009_12850_amd/csrc/advect.hip"]
TRAFFIC_FILE = "profiles/advect_march_step_f64_big1024_traffic.txt"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain device copy of known size), or None if there is none for this
    workload or the kernel sources have changed since."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("workload") != workload or kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="big1024")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-forms", action="store_true")
    p.add_argument("--only-form", choices=["tvd_momentum", "dynamics"], default=None,
                   help="after the headline, run only this form (for profiling it)")
    p.add_argument("--no-learned", action="store_true",
                   help="skip the learned-correction form (fine runs, training, coarse runs)")
    p.add_argument("--learned-seeds", type=int, default=16,
                   help="fine runs for the learned form; the last quarter is held out")
    p.add_argument("--learned-train-steps", type=int, default=3000)
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 1 GiB device-to-device copy (reference for "
                        "the HBM byte counters)")
    return p.parse_args()


def event_time_ms(torch, stream, fn, reps):
    """Average duration of fn() on `stream`, bracketed by HIP events."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(reps):
            fn()
        end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def launch_times_ms(torch, stream, fn, reps):
    """Durations of `reps` single launches of fn() on `stream`, each bracketed
    by its own pair of HIP events."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    with torch.cuda.stream(stream):
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
    ev[-1][1].synchronize()
    return [a.elapsed_time(b) for a, b in ev]


PW_FLOP = 92  # floating-point operations of one PW evaluation per grid point


def bench_scaled(torch, M, vel64, g, prof, stream, npts, reps):
    """Work-scaled PW (the PW arithmetic repeated 1..16 times on the same data)
    in FP64 and FP32: time, effective FLOP rate and HBM fraction per factor."""
    vel32 = [v.float() for v in vel64]
    out = {}
    for name, code, vel, eb in (("f64", M.MONC_F64, vel64, 8), ("f32", M.MONC_F32, vel32, 4)):
        outs = [torch.empty_like(v) for v in vel]
        M.monc_advect_pw_scaled(code, *vel, *outs, g.dx, g.dy, prof, 1, stream)  # warm-up
        rows = {}
        for work in (1, 2, 4, 8, 16):
            ms = event_time_ms(torch, stream, lambda: M.monc_advect_pw_scaled(
                code, *vel, *outs, g.dx, g.dy, prof, work, stream), reps)
            rows[str(work)] = {"ms": ms,
                               "tflops": PW_FLOP * work * npts / (ms * 1e-3) / 1e12,
                               "hbm_frac": 6.0 * eb * npts / (ms * 1e-3) / HBM_PEAK}
        out[name] = rows
        del outs
    del vel32
    return out


REGION = (0, 128, 0, 128)  # the subdomain of the precision forms' errors (all levels)


def precision_outputs(torch, M, host, g, prof, w, dev, stream):
    """The precision forms on the benchmark's input: FP32 and BF16 working
    copies (scalars stored as anomalies from their nominal values) advected in
    FP32, and the mixed step with budgets.  Returns host arrays of the
    region's results and the domain sums of the source terms (float64 sums of
    the GPU's values, measurement only)."""
    i0, i1, j0, j1 = REGION
    sl = (slice(i0 + 2, i1 + 2), slice(j0 + 2, j1 + 2))
    X = [torch.from_numpy(h).to(dev) for h in host]
    nscal = len(host) - 3
    phi0 = [300.0] + [1e-3] * (nscal - 1)
    offs = [0.0, 0.0, 0.0] + phi0
    mass = torch.from_numpy(g.rhon / g.rdz).to(dev)
    dzn = 0.5 * (1.0 / g.rdz[:-1] + 1.0 / g.rdz[1:])
    wm = np.zeros(g.nz)
    wm[:-1] = g.rho[:-1] * dzn
    wmass = torch.from_numpy(wm).to(dev)
    res = {}
    for name, code, tdt in (("f32", M.MONC_F32, torch.float32), ("bf16", M.MONC_BF16, torch.int16)):
        work = [torch.empty(x.shape, dtype=tdt, device=dev) for x in X]
        M.monc_cast_working(code, X, work, offs, stream)
        outs = [torch.empty(x.shape, dtype=torch.float32, device=dev) for x in X]
        M.monc_advect(code, work, outs, g.dx, g.dy, prof, w.dt, phi0=phi0, stream=stream)
        sums = {}
        for n, o in enumerate(outs):
            wt = wmass if n == 2 else mass
            sums[n] = float((o[2:-2, 2:-2, :].double() * wt).sum())
        res[name] = {"region": [o[sl].double().cpu().numpy() for o in outs], "sums": sums}
        del work, outs
    out = [torch.empty_like(x) for x in X]
    bud = torch.zeros(M.MONC_NBUDGET, dtype=torch.float64, device=dev)
    ws = torch.empty(M.monc_step_workspace_bytes(g.nx, g.ny, g.nz, nscal), dtype=torch.uint8,
                     device=dev)
    M.monc_step_mixed(X, out, phi0, g.dx, g.dy, prof, w.dt, bud, ws, stream)
    res["mixed"] = {"region_inc": [(o[sl] - x[sl]).cpu().numpy() for o, x in zip(out, X)],
                    "budgets": M.budgets_dict(bud.cpu().numpy(), nscal)}
    del X, out
    torch.cuda.empty_cache()
    return res


def precision_errors(res, host, g, dt):
    """Errors of the precision forms against the FP64 oracle: per field
    max |gpu - oracle| / max |oracle| of the source terms on the region (the
    mixed step: of the increments, against dt times the oracle's source terms),
    and the domain budgets' differences relative to the oracle's sum of
    |terms| (conservation sums C, energy production P, scalar mass M)."""
    from oracle import pyoracle as O
    O.build(force=False)
    hosts = [O.halo_fill(h.copy()) for h in host]
    i0, i1, j0, j1 = REGION
    sl = (slice(i0 + 2, i1 + 2), slice(j0 + 2, j1 + 2))
    u, v, w = hosts[:3]
    full = list(O.pw(u, v, w, g)) + [O.tvd(u, v, w, q, g, dt) for q in hosts[3:]]
    ob, sc = O.budgets(*hosts[:3], *full[:3], hosts[3:], full[3:], g)
    mass = (g.rhon / g.rdz)[None, None, :]
    sscale = [float(np.sum(np.abs(full[3 + s][2:-2, 2:-2]) * mass)) for s in range(len(host) - 3)]
    names = ["u", "v", "w"] + [f"s{s}" for s in range(len(host) - 3)]
    out = {"region": f"i, j in [{i0}, {i1}) x [{j0}, {j1}), all levels"}
    for form in ("f32", "bf16"):
        errs, berr = {}, {}
        for n, nm in enumerate(names):
            exp = full[n][sl]
            errs[nm] = float(np.abs(res[form]["region"][n] - exp).max() / np.abs(exp).max())
            key = f"C_{nm}" if n < 3 else f"C_s{n - 3}"
            scale = sc[key] if n < 3 else sscale[n - 3]
            berr[key] = abs(res[form]["sums"][n] - ob[key]) / scale
        out[form] = {"field_rel_err": errs, "budget_rel_err": berr}
    errs, berr = {}, {}
    for n, nm in enumerate(names):
        exp = dt * full[n][sl]
        if n == 2:
            exp[:, :, -1] = 0.0
        errs[nm] = float(np.abs(res["mixed"]["region_inc"][n] - exp).max() / np.abs(exp).max())
    gb = res["mixed"]["budgets"]
    for key in ["C_u", "C_v", "C_w", "P_u", "P_v", "P_w"]:
        berr[key] = abs(gb[key] - ob[key]) / sc[key]
    for s in range(len(host) - 3):
        berr[f"C_s{s}"] = abs(gb[f"C_s{s}"] - ob[f"C_s{s}"]) / sscale[s]
        berr[f"M_s{s}"] = abs(gb[f"M_s{s}"] - ob[f"M_s{s}"]) / abs(ob[f"M_s{s}"])
        berr[f"min_s{s}"] = abs(gb[f"min_s{s}"] - ob[f"min_s{s}"]) / abs(ob[f"min_s{s}"])
    out["mixed"] = {"field_rel_err": errs, "budget_rel_err": berr}
    return out


def learned_gradient_check(torch, M, dev, m=32768, seed=5):
    """The learned form's gradients at the training batch's row count (4 face
    rows for each of 8192 cells): the GPU forward (saving its activations)
    and backward on seeded features, against the FP64 oracle's backward from
    the GPU's own activations with BF16 rounding emulated where the kernels
    round; per parameter block, max |gpu - oracle| / max |oracle|."""
    from oracle import mlp_ref as R
    rng = np.random.default_rng(seed)
    p = R.init_params(seed).astype(np.float32).astype(np.float64)
    X = rng.standard_normal((m, R.K))
    X[:, R.PAD] = 0.0
    Xb = R.bf16(X)
    Xd = torch.from_numpy(Xb.astype(np.float32)).to(dev).to(torch.bfloat16).view(torch.int16)
    pd = torch.from_numpy(p.astype(np.float32)).to(dev)
    wp = torch.zeros(M.MONC_MLP_WPACK, dtype=torch.int16, device=dev)
    M.monc_mlp_pack(pd, wp)
    Y = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    H1 = torch.zeros((m, 64), dtype=torch.int16, device=dev)
    H2 = torch.zeros_like(H1)
    Z1 = torch.zeros((m, 64), dtype=torch.float32, device=dev)
    Z2 = torch.zeros_like(Z1)
    M.monc_mlp_forward(Xd, m, pd, wp, Y, H1, H2, Z1, Z2)
    dY = (rng.standard_normal((m, 4)) / m).astype(np.float32)
    grad = torch.zeros(R.NPARAM, dtype=torch.float32, device=dev)
    ws = torch.zeros(M.monc_mlp_backward_workspace_bytes(m), dtype=torch.uint8, device=dev)
    M.monc_mlp_backward(Xd, H1, H2, Z1, Z2, torch.from_numpy(dY).to(dev), m, wp, grad, ws)
    torch.cuda.synchronize()
    bf = lambda t: t.view(torch.bfloat16).double().cpu().numpy()
    _, b1, W2, b2, W3, b3 = R.unpack(p)
    cache = dict(Xb=Xb, Z1=Z1.double().cpu().numpy(), H1=bf(H1), Z2=Z2.double().cpu().numpy(),
                 H2=bf(H2), W2b=R.bf16(W2), W3b=R.bf16(W3))
    ref = R.unpack(R.backward(dY.astype(np.float64), cache, emulate=True))
    got = R.unpack(grad.double().cpu().numpy())
    out = {}
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], got, ref):
        out[name] = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    return {"rows": m, "block_rel_err": out}


def learned_fused_gradient_check(torch, M, dev, B=8192, seed=6):
    """The fused training step's gradient (monc_mlp_train_step, B cells on a
    128 x 128 x 32 coarse grid of seeded fields: 4 B rows) against the FP64
    oracle's backward from the separate kernels' activations and dY for the
    same rows (the fused step computes each row with the same operations);
    per parameter block, max |gpu - oracle| / max |oracle|."""
    from oracle import mlp_ref as R
    NX, NY, NZ = 128, 128, 32
    rng = np.random.default_rng(seed)
    mk = lambda a, b: rng.standard_normal((NX + 4, NY + 4, NZ)) * a + b
    c0 = [mk(3.0, 1.0), mk(2.0, -0.5), mk(0.7, 0.0), mk(0.5, 300.0)]
    c0[2][:, :, -1] = 0.0
    c1 = [a + 0.5 * rng.standard_normal(a.shape) for a in c0]
    c1[2][:, :, -1] = 0.0
    tend = [0.1 * rng.standard_normal(a.shape) for a in c0]
    dv = lambda arrs: [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs]
    d0, d1, dte = dv(c0), dv(c1), dv(tend)
    prof = dv([np.zeros(NZ), 1.2 * np.exp(-np.arange(NZ) / 5.0),
               1.2 * np.exp(-(np.arange(NZ) + 0.5) / 5.0)])
    n = NX * NY * NZ
    cells = np.sort(rng.integers(0, n, B)).astype(np.int32)
    k = cells % NZ
    i, j = cells // (NY * NZ), (cells // NZ) % NY
    xm = ((((i - 1) % NX) * NY + j) * NZ + k).astype(np.int32)
    ym = ((i * NY + (j - 1) % NY) * NZ + k).astype(np.int32)
    cx, cy, cd = dv([np.concatenate([cells, xm]), np.concatenate([cells, ym]), cells])
    nterm = 4 * B - int(np.sum(k == NZ - 1))
    norm = [1.0, 3.0, -0.5, 2.0, 0.0, 0.7, 300.0, 0.5]
    scale, dt, m = [0.3, 0.2, 0.05, 0.01], 2.0, 4 * B
    p = R.init_params(seed).astype(np.float32)
    pd = torch.from_numpy(p.copy()).to(dev)
    wp = torch.zeros(M.MONC_MLP_WPACK, dtype=torch.int16, device=dev)
    M.monc_mlp_pack(pd, wp)
    X = torch.zeros((m, R.K), dtype=torch.int16, device=dev)
    M.monc_mlp_features(d0, norm, 0, cx, X.narrow(0, 0, 2 * B))
    M.monc_mlp_features(d0, norm, 1, cy, X.narrow(0, 2 * B, 2 * B))
    Y = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    H1 = torch.zeros((m, 64), dtype=torch.int16, device=dev)
    H2 = torch.zeros_like(H1)
    Z1 = torch.zeros((m, 64), dtype=torch.float32, device=dev)
    Z2 = torch.zeros_like(Z1)
    M.monc_mlp_forward(X, m, pd, wp, Y, H1, H2, Z1, Z2)
    dY = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    wsl = torch.zeros(M.monc_mlp_loss_workspace_bytes(B), dtype=torch.uint8, device=dev)
    M.monc_mlp_loss(Y, B, cd, d0, d1, dte, dt, scale, prof, 1.0 / nterm, dY, loss, wsl)
    m1, m2 = torch.zeros_like(pd), torch.zeros_like(pd)
    grad = torch.zeros_like(pd)
    lf = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.zeros(M.monc_mlp_train_workspace_bytes(B), dtype=torch.uint8, device=dev)
    M.monc_mlp_train_step(d0, d1, dte, norm, cd, dt, scale, prof, 1.0 / nterm, pd, m1, m2, 1,
                          1e-3, 0.9, 0.999, 1e-8, wp, grad, lf, ws)
    torch.cuda.synchronize()
    bf = lambda t: t.view(torch.bfloat16).double().cpu().numpy()
    _, b1, W2, b2, W3, b3 = R.unpack(p.astype(np.float64))
    cache = dict(Xb=bf(X), Z1=Z1.double().cpu().numpy(), H1=bf(H1), Z2=Z2.double().cpu().numpy(),
                 H2=bf(H2), W2b=R.bf16(W2), W3b=R.bf16(W3))
    ref = R.unpack(R.backward(dY.double().cpu().numpy(), cache, emulate=True))
    got = R.unpack(grad.double().cpu().numpy())
    out = {}
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3"], got, ref):
        out[name] = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    # b3's exact gradient is 0 (a constant flux has no divergence): report
    # its largest entry against the sum of |dY|
    out["b3_abs_over_sum_abs_dY"] = float(np.abs(got[5]).max() /
                                          np.abs(dY.double().cpu().numpy()).sum(axis=0).max())
    return {"rows": m, "cells": B, "block_rel_err": out,
            "loss_rel_diff_vs_separate": abs(float(lf.item()) - float(loss.item())) /
            float(loss.item())}


def cpu_baseline():
    """The FP64 oracle, unchanged, timed on the host cores with one thread and
    with all of them: one forward step (every source term and the update) of
    an x-slab of each of the two FP64 workloads (64 x 1024 x 128 with u v w th
    q1, of the 1024 x 1024 x 128 grid; 32 x 512 x 128 with u v w th q1 q2 q3,
    of the 512 x 512 x 128 grid), same generator and profiles, periodic on the
    slab; median of 5 timed steps after one warm-up.  A slab's cost per point
    is that of the whole grid (the oracle's loops are per point), and it keeps
    the run bounded."""
    from oracle import pyoracle as O
    from paper_2009_12850_amd import inputs as I
    O.build(force=False)
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        ncores = min(ncores, int(omp))
    rows = []
    for name, (nx, ny, nz, nscal, seed) in (("big1024", (64, 1024, 128, 2, 3)),
                                            ("steps512", (32, 512, 128, 4, 2))):
        g = I.make_geometry(nx, ny, nz)
        f = I.make_fields(g, nscal, seed=seed, padded=True)
        st = [f[n] for n in ["u", "v", "w"] + I.scalar_names(nscal)]
        out = [np.empty_like(x) for x in st]
        nf = 3 + nscal
        for threads in (1, ncores):
            used = O.set_threads(threads)
            O.step(st, g, 0.5, out=out)  # warm-up
            times = []
            for _ in range(5):
                t0 = time.perf_counter()
                O.step(st, g, 0.5, out=out)
                times.append(time.perf_counter() - t0)
            med = float(np.median(times))
            pts = nx * ny * nz
            rows.append({"workload": name, "sample": f"{nx}x{ny}x{nz} slab, {nf} fields",
                         "threads": used, "median_s": med, "gpups": pts / med,
                         "gbps": 16.0 * nf * pts / med / 1e9})
            log(f"  oracle {name} slab, {used} threads: {med:.3f} s per step")
    O.set_threads(ncores)
    head = [r for r in rows if r["workload"] == "big1024" and r["threads"] == ncores][0]
    return {"value": head["gpups"], "unit": "grid-point updates/s", "cores": head["threads"],
            "kind": "oracle",
            "sample": "one oracle step of a 64x1024x128 slab of the headline grid "
                      "(u v w th q1), median of 5 after 1 warm-up, all cores",
            "rows": rows}


DYN_PARAMS = (1.0e-4, 5.0, 0.0, 9.81, 300.0)  # fcor, ug, vg, grav, th0


def bench_dynamics(torch, M, state, g, prof, w, stream, npts, nf, reps):
    """The step with the other dynamics source terms (Coriolis, buoyancy):
    the paper's hybrid structure (other components beside the advection,
    source terms combined before the step) on one stream and on two, against
    the same terms fused into the advection pass."""
    tend = [torch.empty_like(a) for a in state[0]]
    dyn = [torch.empty_like(a) for a in state[0][:3]]
    side = torch.cuda.Stream()
    out = {}
    runs = {
        "plain_step": lambda: M.monc_step(state[0], state[1], g.dx, g.dy, prof, w.dt,
                                          None, None, stream),
        "sequential": lambda: M.monc_hybrid_step(state[0], state[1], tend, dyn, g.dx, g.dy,
                                                 prof, w.dt, DYN_PARAMS, stream),
        "two_streams": lambda: M.monc_hybrid_step(state[0], state[1], tend, dyn, g.dx,
                                                  g.dy, prof, w.dt, DYN_PARAMS, stream,
                                                  side_stream=side),
        "fused": lambda: M.monc_step_dyn(state[0], state[1], g.dx, g.dy, prof, w.dt,
                                         DYN_PARAMS, stream),
        # MONC's other scalar scheme (centred flux form) in the same pass
        "pw_scalars_step": lambda: M.monc_step_pw_scalars(state[0], state[1], g.dx, g.dy,
                                                          prof, w.dt, stream),
    }
    for name, fn in runs.items():
        fn()
        torch.cuda.synchronize()
        ms = event_time_ms(torch, stream, fn, reps)
        torch.cuda.synchronize()
        out[name] = {"ms": ms, "gpups": npts / (ms * 1e-3)}
    # bytes: the hybrid path writes and re-reads every source term
    out["fused"]["bytes_per_point"] = 16.0 * nf
    # advection source terms 16 nf, Coriolis + buoyancy 48, combine 8 (3 nf + 3)
    out["two_streams"]["bytes_per_point"] = 16.0 * nf + 48.0 + 8.0 * (3 * nf + 3)
    out["fused_speedup_vs_two_streams"] = out["two_streams"]["ms"] / out["fused"]["ms"]
    out["fused_cost_vs_plain_step"] = out["fused"]["ms"] / out["plain_step"]["ms"]
    del tend, dyn
    return out


def bench_tvd_momentum(torch, M, state, g, prof, w, stream, npts, plain_ms, reps):
    """TVD advection of momentum: the source-term pass alone (one read of u, v,
    w and one write of su, sv, sw: 48 bytes per point) and the all-TVD step
    (that pass stepping u, v, w, then the scalar march)."""
    src = [torch.empty_like(a) for a in state[0][:3]]
    run = lambda: M.monc_advect_tvd_momentum(*state[0][:3], *src, g.dx, g.dy, prof, w.dt,
                                             stream=stream)
    step = lambda: M.monc_step_tvd_momentum(state[0], state[1], g.dx, g.dy, prof, w.dt,
                                            stream=stream)
    out = {}
    for name, fn in (("source_terms", run), ("step", step)):
        fn()
        torch.cuda.synchronize()
        ms = event_time_ms(torch, stream, fn, reps)
        out[name] = {"ms": ms, "gpups": npts / (ms * 1e-3)}
    gbps = 48.0 * npts / (out["source_terms"]["ms"] * 1e-3) / 1e9
    out["source_terms"].update({"bytes_per_point": 48.0, "achieved_gbps": gbps,
                                "hbm_frac": gbps * 1e9 / HBM_PEAK})
    out["step_cost_vs_pw_step"] = out["step"]["ms"] / plain_ms
    del src
    return out


CEIL_BLOCKS = 32768  # workgroups of the streaming kernels (the best of 8192 .. 65536)


def stream_ceiling(torch, M, dev, stream, reps=10):
    """HBM rates of the library's streaming kernels (16-byte accesses,
    non-temporal stores) over 2 GiB buffers: read only, write only and a 1:1
    copy (the read/write mix of the advection step), median of `reps`."""
    nbytes = 1 << 31
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    sink = torch.empty(M.monc_ceiling_sink_bytes(CEIL_BLOCKS), dtype=torch.uint8, device=dev)
    out = {}
    for name, mode, a, b, moved in (("read", M.MONC_CEIL_READ, src, sink, nbytes),
                                    ("write", M.MONC_CEIL_WRITE, None, dst, nbytes),
                                    ("copy", M.MONC_CEIL_COPY, src, dst, 2 * nbytes)):
        fn = lambda: M.monc_stream_ceiling(mode, a, b, nbytes, CEIL_BLOCKS, stream)
        fn()
        med = float(np.median(launch_times_ms(torch, stream, fn, reps)))
        out[f"{name}_gbps"] = moved / (med * 1e-3) / 1e9
    del src, dst, sink
    torch.cuda.empty_cache()
    out["kernel"] = "monc_stream_ceiling (16-byte accesses, non-temporal stores)"
    return out


def synthetic_state(torch, dev, shape, nscal, seed):
    """Seeded device-side fields of the usual kinds for throughput-only runs
    (the kernels have no data-dependent branches): velocities of a few m/s, w
    zero on the lid, theta near 300 K, positive tracers."""
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    r = lambda s: torch.randn(shape, dtype=torch.float64, device=dev, generator=gen) * s
    u, v, w = r(2.0), r(2.0), r(0.2)
    w[:, :, -1] = 0.0
    out = [u, v, w, 300.0 + r(1.0)]
    out += [1e-3 * torch.exp(r(0.5)) for _ in range(nscal - 1)]
    return out


def bench_step_shape(torch, M, I, dev, stream, nx, ny, nz, nscal, reps, seed):
    """GPUPS of monc_step (with budgets) on another grid shape."""
    g = I.make_geometry(nx, ny, nz, 50.0, 50.0)
    prof = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (g.rdz, g.rho, g.rhon)]
    A = synthetic_state(torch, dev, (nx + 4, ny + 4, nz), nscal, seed)
    B = [torch.empty_like(a) for a in A]
    bud = torch.zeros(M.MONC_NBUDGET, dtype=torch.float64, device=dev)
    ws = torch.empty(M.monc_step_workspace_bytes(nx, ny, nz, nscal), dtype=torch.uint8,
                     device=dev)
    # Every repetition steps the same input state: the work and the HBM
    # traffic are those of any step (the state is far larger than every cache),
    # and white-noise fields are not stepped on until forward Euler makes them
    # grow without bound.

    def step():
        M.monc_step(A, B, g.dx, g.dy, prof, 0.5, bud, ws, stream)

    step()
    torch.cuda.synchronize()
    ms = event_time_ms(torch, stream, step, reps)
    torch.cuda.synchronize()
    status = M.monc_budgets_check(bud.cpu().numpy())
    npts = nx * ny * nz
    nf = 3 + nscal
    out = {"grid": [nx, ny, nz], "fields": nf, "ms": ms, "gpups": npts / (ms * 1e-3),
           "hbm_frac": 16.0 * nf * npts / (ms * 1e-3) / HBM_PEAK,
           "status": "ok" if status == M.MONC_OK else M.lib().monc_strerror(status).decode(),
           "data": "seeded device-side random fields (throughput only)"}
    del A, B
    torch.cuda.empty_cache()
    return out


def bench_ensemble(torch, M, I, dev, steps, log):
    """64 uneven members (nx, ny in {64..256}, nz in {64, 96}), FP32 source
    terms from the FP64 state, `steps` steps in one captured graph launch,
    against the same steps launched member by member."""
    import tempfile
    nscal = 2
    geo = I.ensemble_members(64, seed=4)
    members = []
    for md in geo:
        g = I.make_geometry(md["nx"], md["ny"], md["nz"], dx=md["dx"], dy=md["dx"])
        f = I.make_fields(g, nscal, md["seed"], amp=md["amp"], padded=True)
        names = ["u", "v", "w"] + I.scalar_names(nscal)
        s0 = [torch.from_numpy(f.pop(k)).to(dev) for k in names]
        s1 = [torch.empty_like(x) for x in s0]
        prof = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (g.rdz, g.rho, g.rhon)]
        members.append(dict(state0=s0, state1=s1, prof=prof, dx=md["dx"], dy=md["dx"], dt=0.5,
                            phi0=[300.0, 1e-3]))
    pts = sum(md["nx"] * md["ny"] * md["nz"] for md in geo)
    cache = os.path.join(tempfile.gettempdir(), "monc_ensemble_tune.json")
    log("ensemble: plan + autotune")
    t0 = time.perf_counter()
    ens = M.Ensemble(members, nscal, tune_cache=cache, tune=True)
    t_plan = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    ens.run(steps, stream)  # builds the graph
    torch.cuda.synchronize()
    t_graph = event_time_ms(torch, stream, lambda: ens.run(steps, stream), 1)

    def eager():
        for mem in members:
            cur = mem["state0"] if ens.parity == 0 else mem["state1"]
            nxt = mem["state1"] if ens.parity == 0 else mem["state0"]
            a, b = cur, nxt
            for _ in range(steps):
                M.monc_step_mixed(a, b, mem["phi0"], mem["dx"], mem["dy"], mem["prof"],
                                  mem["dt"], stream=stream)
                a, b = b, a
    t_eager = event_time_ms(torch, stream, eager, 1)
    info = ens.info()
    ens.close()
    gpups = pts * steps / (t_graph * 1e-3)
    return {"members": len(geo), "points": pts, "steps": steps, "ms": t_graph,
            "gpups": gpups, "hbm_frac": 16.0 * (3 + nscal) * gpups / HBM_PEAK,
            "eager_ms": t_eager, "speedup_vs_eager": t_eager / t_graph,
            "plan_s": t_plan, "tuned": info}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the advection "
              "path runs on a single device", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2009_12850_amd import _lib as M
    from paper_2009_12850_amd import inputs as I

    M.lib()
    dev = torch.device("cuda:0")
    w = I.WORKLOADS[args.workload]
    log(f"generating {args.workload} inputs")
    g = I.make_geometry(w.nx, w.ny, w.nz, w.dx, w.dx)
    names = ["u", "v", "w"] + I.scalar_names(w.nscal)
    f = I.make_fields(g, w.nscal, w.seed, padded=True)
    host = [f.pop(n) for n in names]  # kept for the oracle's error check
    del f
    A = [torch.from_numpy(h).to(dev) for h in host]
    B = [torch.empty_like(a) for a in A]
    prof = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (g.rdz, g.rho, g.rhon)]
    budgets = torch.zeros(M.MONC_NBUDGET, dtype=torch.float64, device=dev)
    ws = torch.empty(M.monc_step_workspace_bytes(w.nx, w.ny, w.nz, w.nscal),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    npts = w.nx * w.ny * w.nz
    nf = len(names)
    state = [A, B]

    def step(budget=True):
        M.monc_step(state[0], state[1], g.dx, g.dy, prof, w.dt,
                    budgets if budget else None, ws if budget else None, stream)
        state.reverse()

    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    bh = budgets.cpu().numpy()
    status = M.monc_budgets_check(bh)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = event_time_ms(torch, stream, step, args.steps)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    value = npts / (ms * 1e-3)

    # The dominant kernel is the timed launch itself (the advection march
    # with budget partials; the final budget pass adds about 5 us): its
    # average duration over the timed region gives the roofline; the median
    # of per-launch timings and the same launch without budgets are reported
    # beside it.
    bytes_alg = 16.0 * nf * npts  # one read and one write of every FP64 field
    lt = launch_times_ms(torch, stream, step, max(20, args.steps))
    lt0 = launch_times_ms(torch, stream, lambda: step(False), max(20, args.steps))
    achieved = bytes_alg / (ms * 1e-3)
    traffic = measured_traffic(args.workload)
    ceil = stream_ceiling(torch, M, dev, stream)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": traffic / 1e9 if traffic else None, "traffic_unit": "GB per launch",
                # measured bytes of the launch (counters) over its duration, vs the peak
                "traffic_frac": (traffic / (ms * 1e-3) / HBM_PEAK) if traffic else None,
                "traffic_over_algorithmic": traffic / bytes_alg if traffic else None,
                "kernel": "monc_step with budgets (fused PW + TVD + update + budget "
                          "partials, FP64): the timed launch",
                "bytes_per_launch": bytes_alg, "launch_ms_mean": ms,
                "launch_ms_median": float(np.median(lt)),
                "ceiling": ceil,
                "frac_of_copy_ceiling": achieved / 1e9 / ceil["copy_gbps"],
                "no_budgets": {"launch_ms_median": float(np.median(lt0)),
                               "frac": bytes_alg / (np.median(lt0) * 1e-3) / HBM_PEAK}}

    forms = None
    prec_res = None
    if not args.no_forms and args.only_form:
        log(f"form {args.only_form}")
        if args.only_form == "dynamics":
            forms = {"dynamics": bench_dynamics(torch, M, state, g, prof, w, stream, npts, nf,
                                                args.steps)}
        else:
            plain = event_time_ms(torch, stream, lambda: M.monc_step(
                state[0], state[1], g.dx, g.dy, prof, w.dt, None, None, stream), args.steps)
            forms = {"tvd_momentum": bench_tvd_momentum(torch, M, state, g, prof, w, stream,
                                                        npts, plain, args.steps)}
    elif not args.no_forms:
        log("precision forms")
        forms = {}
        tend64 = [torch.empty_like(a) for a in A]
        M.monc_halo_fill(state[0], stream)
        t64 = event_time_ms(torch, stream, lambda: M.monc_advect(
            M.MONC_F64, state[0], tend64, g.dx, g.dy, prof, w.dt, stream=stream), args.steps)
        forms["f64_tendencies"] = {"ms": t64, "gpups": npts / (t64 * 1e-3),
                                   "hbm_frac": 16.0 * nf * npts / (t64 * 1e-3) / HBM_PEAK}
        del tend64
        phi0 = [300.0] + [1e-3] * (w.nscal - 1)  # nominal theta and tracer values
        offs = [0.0, 0.0, 0.0] + phi0
        for dt_name, code, tdt in (("f32", M.MONC_F32, torch.float32),
                                   ("bf16", M.MONC_BF16, torch.int16)):
            work = [torch.empty(a.shape, dtype=tdt, device=dev) for a in A]
            M.monc_cast_working(code, state[0], work, offs, stream)
            outs = [torch.empty(a.shape, dtype=torch.float32, device=dev) for a in A]
            t = event_time_ms(torch, stream, lambda: M.monc_advect(
                code, work, outs, g.dx, g.dy, prof, w.dt, phi0=phi0, stream=stream),
                args.steps)
            eb = 4 if code == M.MONC_F32 else 2
            forms[f"{dt_name}_tendencies"] = {
                "ms": t, "gpups": npts / (t * 1e-3),
                "hbm_frac": (eb + 4.0) * nf * npts / (t * 1e-3) / HBM_PEAK,
                "speedup_vs_f64": t64 / t}
            # the marshalling cast of all fields (whole padded arrays: 8 bytes
            # read and 4 or 2 written per value)
            tc = event_time_ms(torch, stream, lambda: M.monc_cast_working(
                code, state[0], work, offs, stream), args.steps)
            cbytes = (8.0 + eb) * nf * A[0].numel()
            forms[f"{dt_name}_tendencies"]["cast"] = {
                "ms": tc, "gbps": cbytes / (tc * 1e-3) / 1e9,
                "hbm_frac": cbytes / (tc * 1e-3) / HBM_PEAK,
                # one cast then the FP32 source terms, against the FP64 source terms
                "cast_plus_tendencies_speedup_vs_f64": t64 / (t + tc)}
            del work, outs
        log("precision forms on the benchmark input (for the oracle's error check)")
        prec_res = precision_outputs(torch, M, host, g, prof, w, dev, stream)
        forms["work_scaled_pw"] = bench_scaled(torch, M, state[0][:3], g, prof, stream, npts,
                                               max(3, args.steps // 4))
        mixed = lambda: M.monc_step_mixed(state[0], state[1], phi0, g.dx, g.dy, prof, w.dt,
                                          None, None, stream)
        tm = event_time_ms(torch, stream, mixed, args.steps)
        forms["mixed_step"] = {"ms": tm, "gpups": npts / (tm * 1e-3)}
        forms["dynamics"] = bench_dynamics(torch, M, state, g, prof, w, stream, npts, nf,
                                           args.steps)
        forms["tvd_momentum"] = bench_tvd_momentum(torch, M, state, g, prof, w, stream, npts,
                                                   forms["dynamics"]["plain_step"]["ms"],
                                                   args.steps)
        # the step on the other grids the method is quoted on: 512 x 512 x 128
        # with 7 fields, and the paper's tank-case shape 2048 x 2048 x 64 with
        # 9 fields (its strong-scaling problem, on one device)
        forms["steps512_step"] = bench_step_shape(torch, M, I, dev, stream, 512, 512, 128, 4,
                                                  args.steps, 21)
        forms["tank_shape_step"] = bench_step_shape(torch, M, I, dev, stream, 2048, 2048, 64,
                                                    6, max(5, args.steps // 4), 22)

    if not args.no_forms and not args.only_form:
        del B
        state.clear()
        torch.cuda.empty_cache()
        forms["ensemble"] = bench_ensemble(torch, M, I, dev, 50, log)
    if not args.no_forms and not args.only_form and not args.no_learned:
        from paper_2009_12850_amd import learned as L
        log("learned correction: fine runs, training, coarse runs")
        ns = args.learned_seeds
        forms["learned"] = L.run_experiment(
            seeds=range(2000, 2000 + ns), n_train=ns - max(1, ns // 4),
            train_steps=args.learned_train_steps, device=dev, log=log)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
        if prec_res is not None:
            # the precision forms' errors against the FP64 oracle (this leg is
            # the only part of the benchmark that runs the oracle)
            log("precision forms: errors against the oracle")
            forms["precision_errors"] = precision_errors(prec_res, host, g, w.dt)
        if forms is not None and "learned" in forms:
            log("learned form: gradient check against the oracle")
            forms["learned"]["gradient_check"] = learned_gradient_check(torch, M, dev)
            forms["learned"]["gradient_check"]["fused_step"] = learned_fused_gradient_check(
                torch, M, dev)
    del host

    rec = {
        "metric": "advection grid-point updates/s + % HBM peak; FP64 plain vs FP32/batched/learned",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_ms_per_step": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded smooth random flow + noise, stretched grid)",
        "config": {"workload": f"{args.workload}: {w.nx}x{w.ny}x{w.nz}, fields "
                               f"{' '.join(names)}, FP64 step (PW + TVD + update + budgets)",
                   "nx": w.nx, "ny": w.ny, "nz": w.nz, "fields": nf, "dt": w.dt},
        "status": M.lib().monc_strerror(status).decode(),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
