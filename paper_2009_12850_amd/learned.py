"""Learned coarse-grid flux correction: data, training and coarse runs.

Fine runs of the plain scheme (monc_step, FP64) are restricted every
`every` steps to a grid 4x coarser (monc_restrict4).  A coarse step of
dt_c = every * dt is then corrected by the flux divergence of a small MLP,
trained so that the corrected coarse source terms reproduce the restricted
fine evolution.  All arithmetic on the fields and the network runs in the
library's kernels; this module only orchestrates the calls, samples training
cells (seeded, on the host) and computes normalisation statistics from a few
host copies.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import _lib as M
from . import inputs as I

FIELDS = ["u", "v", "w", "th"]


def _torch():
    import torch
    return torch


@dataclasses.dataclass
class CoarseSeries:
    snaps: list          # coarse states (4 padded FP64 device tensors each)
    tend: list           # plain coarse source terms of snaps[:-1]
    prof_c: list         # rdz_c, rho_c, rhon_c device tensors
    dxc: float
    dtc: float


THETA_REF = 300.0  # K; theta is carried as its anomaly from this reference
# Largest wind component of the fine runs.  Advection alone (no pressure solve)
# lets the flow steepen; at 5 m/s two of the sixteen seeds overflow before step
# 200, at 2 m/s every run keeps its Courant number and theta range.
FINE_AMP = 2.0


def fine_fields(seed, nx, ny, nz, dx, amp=FINE_AMP):
    """Seeded fine initial state (host, padded) of u, v, w, theta.  The flow
    starts divergence-free, as an anelastic flow after its pressure solve, and
    theta is carried as its anomaly from THETA_REF.  Advection alone has no
    pressure solve, so the flow develops divergence D over the run; in flux
    form a scalar near 300 K would turn that into spurious sources 300 D
    (tens of kelvin within 15 steps next to the thin ground layers), while the
    anomaly of a few kelvin stays bounded over the 200 steps used here."""
    g = I.make_geometry(nx, ny, nz, dx, dx)
    f = I.make_divfree_velocity(g, seed, amp=amp, padded=True)
    f.update(I.make_fields(g, 1, seed, amp=amp, padded=True, only=["th"]))
    f["th"] -= THETA_REF
    return f


def fine_series(seed, nx, ny, nz, steps, every, dt, dx, device, amp=FINE_AMP, timing=None,
                fields=None):
    """Run the plain fine scheme and keep the restricted state every `every`
    steps (including the initial state).  `fields`: a prefetched
    fine_fields(seed, ...) result, else it is generated here."""
    torch = _torch()
    g = I.make_geometry(nx, ny, nz, dx, dx)
    f = dict(fields) if fields is not None else fine_fields(seed, nx, ny, nz, dx, amp)
    A = [torch.from_numpy(f.pop(n)).to(device) for n in FIELDS]
    B = [torch.empty_like(x) for x in A]
    prof = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in (g.rdz, g.rho, g.rhon)]
    nzc = nz // 4
    prof_c = [torch.empty(nzc, dtype=torch.float64, device=device) for _ in range(3)]
    shape_c = (nx // 4 + 4, ny // 4 + 4, nzc)
    snaps = []

    def snap(state):
        c = [torch.zeros(shape_c, dtype=torch.float64, device=device) for _ in range(4)]
        M.monc_restrict4(state, c, prof, prof_c)
        snaps.append(c)

    snap(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        M.monc_step(A, B, dx, dx, prof, dt)
        A, B = B, A
        if s % every == 0:
            snap(A)
    torch.cuda.synchronize()
    if timing is not None:
        timing.append(time.perf_counter() - t0)
    dtc = every * dt
    tend = []
    for c in snaps[:-1]:
        t = [torch.zeros_like(x) for x in c]
        M.monc_advect(M.MONC_F64, c, t, 4 * dx, 4 * dx, prof_c, dtc)
        tend.append(t)
    return CoarseSeries(snaps, tend, prof_c, 4 * dx, dtc)


def _coarse_dims(ser):
    sh = ser.snaps[0][0].shape
    return sh[0] - 4, sh[1] - 4, sh[2]


def _interior(t):
    return t[2:-2, 2:-2, :]


def residual_extremes(series_list, scale):
    """Largest |r_q| / scale_q over every snapshot pair of every run (a check
    that the data hold no outliers)."""
    out = [0.0] * 4
    for ser in series_list:
        for n in range(len(ser.tend)):
            for q in range(4):
                r = (_interior(ser.snaps[n + 1][q]) - _interior(ser.snaps[n][q])) / ser.dtc \
                    - _interior(ser.tend[n][q])
                if q == 2:
                    r = r[:, :, :-1]
                out[q] = max(out[q], float(r.abs().max()) / scale[q])
    return out


def statistics(series_list, nsample=4):
    """Input means/stds per field and residual scales per field, from a few
    host copies of the coarse data."""
    vals = [[] for _ in range(4)]
    res = [[] for _ in range(4)]
    for ser in series_list:
        idx = np.linspace(0, len(ser.tend) - 1, min(nsample, len(ser.tend))).astype(int)
        for n in idx:
            c0 = [_interior(x).cpu().numpy() for x in ser.snaps[n]]
            c1 = [_interior(x).cpu().numpy() for x in ser.snaps[n + 1]]
            td = [_interior(x).cpu().numpy() for x in ser.tend[n]]
            for q in range(4):
                vals[q].append(c0[q].ravel())
                r = (c1[q] - c0[q]) / ser.dtc - td[q]
                if q == 2:
                    r = r[:, :, :-1]
                res[q].append(r.ravel())
    norm = []
    for q in range(4):
        v = np.concatenate(vals[q])
        norm += [float(v.mean()), float(max(v.std(), 1e-12))]
    scale = [float(max(np.concatenate(res[q]).std(), 1e-30)) for q in range(4)]
    return norm, scale


class Correction:
    """The MLP, its FP32 master weights, Adam moments and training buffers."""

    def __init__(self, device, seed, norm, scale, batch=8192):
        torch = _torch()
        from_np = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        self.device = device
        self.norm, self.scale = list(norm), list(scale)
        self.params = from_np(init_params(seed), torch.float32)
        self.m1 = torch.zeros_like(self.params)
        self.m2 = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.wpack = torch.zeros(M.MONC_MLP_WPACK, dtype=torch.int16, device=device)
        M.monc_mlp_pack(self.params, self.wpack)
        self.t = 0
        self.B = batch
        R = 4 * batch
        self.X = torch.zeros((R, M.MONC_MLP_K), dtype=torch.int16, device=device)
        self.Y = torch.zeros((R, 4), dtype=torch.float32, device=device)
        self.H1 = torch.zeros((R, 64), dtype=torch.int16, device=device)
        self.H2 = torch.zeros_like(self.H1)
        self.Z1 = torch.zeros((R, 64), dtype=torch.float32, device=device)
        self.Z2 = torch.zeros_like(self.Z1)
        self.dY = torch.zeros_like(self.Y)
        self.ws_b = torch.zeros(M.monc_mlp_backward_workspace_bytes(R), dtype=torch.uint8,
                                device=device)
        self.ws_l = torch.zeros(M.monc_mlp_loss_workspace_bytes(batch), dtype=torch.uint8,
                                device=device)
        self.ws_t = torch.zeros(M.monc_mlp_train_workspace_bytes(batch), dtype=torch.uint8,
                                device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.cells = torch.zeros(batch, dtype=torch.int32, device=device)
        self.cx = torch.zeros(2 * batch, dtype=torch.int32, device=device)
        self.cy = torch.zeros(2 * batch, dtype=torch.int32, device=device)

    def sample(self, rng, NX, NY, NZ):
        B = self.B
        i = rng.integers(0, NX, B)
        j = rng.integers(0, NY, B)
        k = rng.integers(0, NZ, B)
        c = (i * NY + j) * NZ + k
        # in memory order, so that neighbouring rows' feature gathers share
        # cache lines (the loss is a mean over the cells: order is free)
        order = np.argsort(c, kind="stable")
        i, j, k, c = i[order], j[order], k[order], c[order]
        xm = (((i - 1) % NX) * NY + j) * NZ + k
        ym = (i * NY + (j - 1) % NY) * NZ + k
        n_terms = 4 * B - int(np.sum(k == NZ - 1))  # w on the lid is masked
        return c, xm, ym, n_terms

    def _forward_loss(self, ser, n, rng, save):
        """Features, forward pass and loss on B seeded random cells of snapshot
        pair n of a series."""
        torch = _torch()
        NX, NY, NZ = _coarse_dims(ser)
        c, xm, ym, nterm = self.sample(rng, NX, NY, NZ)
        B = self.B
        host = np.concatenate([c, xm, c, ym, c]).astype(np.int32)
        dev = torch.from_numpy(host).to(self.device)
        self.cx.copy_(dev[:2 * B])
        self.cy.copy_(dev[2 * B:4 * B])
        self.cells.copy_(dev[4 * B:])
        c0, c1, td = ser.snaps[n], ser.snaps[n + 1], ser.tend[n]
        M.monc_mlp_features(c0, self.norm, 0, self.cx, self.X.narrow(0, 0, 2 * B))
        M.monc_mlp_features(c0, self.norm, 1, self.cy, self.X.narrow(0, 2 * B, 2 * B))
        saved = (self.H1, self.H2, self.Z1, self.Z2) if save else (None,) * 4
        M.monc_mlp_forward(self.X, 4 * B, self.params, self.wpack, self.Y, *saved)
        M.monc_mlp_loss(self.Y, B, self.cells, c0, c1, td, ser.dtc, self.scale, ser.prof_c,
                        1.0 / nterm, self.dY, self.loss, self.ws_l)

    def train_step(self, ser, n, rng, lr=1e-3):
        """One Adam step on B seeded random cells of snapshot pair n of a
        series (the fused step: two launches); returns the (device) loss
        before the update."""
        torch = _torch()
        NX, NY, NZ = _coarse_dims(ser)
        c, _, _, nterm = self.sample(rng, NX, NY, NZ)
        self.cells.copy_(torch.from_numpy(c.astype(np.int32)).to(self.device))
        self.device_step(ser, n, nterm, lr)
        return self.loss

    def device_step(self, ser, n, nterm, lr=1e-3):
        """The device work of one training step on the cells already in
        `cells`: no host sampling or copies, so it can be captured in a
        graph."""
        self.t += 1
        M.monc_mlp_train_step(ser.snaps[n], ser.snaps[n + 1], ser.tend[n], self.norm, self.cells,
                              ser.dtc, self.scale, ser.prof_c, 1.0 / nterm, self.params, self.m1,
                              self.m2, self.t, lr, 0.9, 0.999, 1e-8, self.wpack, self.grad,
                              self.loss, self.ws_t)

    def train_step_separate(self, ser, n, rng, lr=1e-3):
        """The same step through the separate entry points (features, forward
        with saved activations, loss, backward with its gradient reduction,
        Adam and pack)."""
        self._forward_loss(ser, n, rng, save=True)
        self._backward_adam(lr)
        return self.loss

    def _backward_adam(self, lr):
        M.monc_mlp_backward(self.X, self.H1, self.H2, self.Z1, self.Z2, self.dY, 4 * self.B,
                            self.wpack, self.grad, self.ws_b)
        self.t += 1
        M.monc_mlp_adam(self.params, self.m1, self.m2, self.grad, self.t, lr, 0.9, 0.999, 1e-8,
                        self.wpack)

    def device_step_separate(self, ser, n, nterm, lr=1e-3):
        """The device work of train_step_separate on the cells already in cx,
        cy, cells."""
        B = self.B
        c0, c1, td = ser.snaps[n], ser.snaps[n + 1], ser.tend[n]
        M.monc_mlp_features(c0, self.norm, 0, self.cx, self.X.narrow(0, 0, 2 * B))
        M.monc_mlp_features(c0, self.norm, 1, self.cy, self.X.narrow(0, 2 * B, 2 * B))
        M.monc_mlp_forward(self.X, 4 * B, self.params, self.wpack, self.Y, self.H1, self.H2,
                           self.Z1, self.Z2)
        M.monc_mlp_loss(self.Y, B, self.cells, c0, c1, td, ser.dtc, self.scale, ser.prof_c,
                        1.0 / nterm, self.dY, self.loss, self.ws_l)
        self._backward_adam(lr)

    def evaluate_loss(self, ser, n, rng):
        """Loss on B cells without updating the weights."""
        self._forward_loss(ser, n, rng, save=False)
        return float(self.loss.item())


def init_params(seed):
    """FP32 master weights ~ N(0, 1/fan_in), biases 0, padded inputs 0 (drawn
    on the host from a seeded generator)."""
    rng = np.random.default_rng(seed)
    H, K, NIN = M.MONC_MLP_H, M.MONC_MLP_K, M.MONC_MLP_NIN
    W1 = rng.standard_normal((H, K)) / np.sqrt(NIN)
    W1.reshape(H, 4, K // 4)[:, :, 75:] = 0.0  # each field's 5 padding slots
    W2 = rng.standard_normal((H, H)) / np.sqrt(H)
    W3 = rng.standard_normal((4, H)) / np.sqrt(H) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(),
                           np.zeros(4)]).astype(np.float32)


def train(model, series_list, steps, seed=0, lr=1e-3, log=None, every=100):
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(steps):
        ser = series_list[rng.integers(0, len(series_list))]
        n = int(rng.integers(0, len(ser.tend)))
        loss = model.train_step(ser, n, rng, lr=lr)
        if (it + 1) % every == 0 or it == 0:
            hist.append((it + 1, float(loss.item())))
            if log:
                log(f"  train step {it + 1}: loss {hist[-1][1]:.4f}")
    return hist


class CoarseRunner:
    """Coarse steps, plain or corrected, on one coarse grid.  `growth` is the
    factor by which a corrected step may raise the kinetic energy or the theta
    variance over the plain step before the plain step is taken instead."""

    def __init__(self, ser, model=None, growth=1.01):
        torch = _torch()
        self.ser = ser
        self.model = model
        self.growth = growth
        shape = ser.snaps[0][0].shape
        dev = ser.snaps[0][0].device
        self.tend = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(4)]
        NX, NY, NZ = shape[0] - 4, shape[1] - 4, shape[2]
        self.N = NX * NY * NZ
        if model is not None:
            self.G = torch.zeros((2 * self.N, 4), dtype=torch.float32, device=dev)
            self.flags = torch.zeros(4, dtype=torch.int32, device=dev)
            self.ws = torch.zeros(M.monc_correct_step_workspace_bytes(NX, NY, NZ),
                                  dtype=torch.uint8, device=dev)

    def step(self, A, B):
        s = self.ser
        if self.model is None:
            M.monc_step(A, B, s.dxc, s.dxc, s.prof_c, s.dtc)
            return
        mdl, N = self.model, self.N
        M.monc_advect(M.MONC_F64, A, self.tend, s.dxc, s.dxc, s.prof_c, s.dtc)
        M.monc_mlp_infer(A, mdl.norm, 2, mdl.params, mdl.wpack, self.G)  # both orientations
        M.monc_correct_step(A, self.tend, self.G.narrow(0, 0, N), self.G.narrow(0, N, N), B,
                            s.dxc, s.dxc, mdl.scale, s.prof_c, s.dtc, self.growth, self.flags,
                            self.ws)

    def fallbacks(self):
        """(non-finite fallbacks, growth fallbacks, clamped theta faces) so far."""
        f = self.flags.cpu().numpy()
        return int(f[1]), int(f[2]), int(f[3])

    def run(self, state0, nsteps):
        torch = _torch()
        A = [x.clone() for x in state0]
        B = [torch.zeros_like(x) for x in A]
        for _ in range(nsteps):
            self.step(A, B)
            A, B = B, A
        return A


def errors(state, ref, ref0):
    """Per field: RMS(state - ref) / RMS(ref - ref0) over the interior (the
    error relative to the change of the restricted fine solution)."""
    out = []
    for q in range(4):
        a, r, r0 = _interior(state[q]), _interior(ref[q]), _interior(ref0[q])
        num = float(((a - r) ** 2).mean().sqrt())
        den = float(((r - r0) ** 2).mean().sqrt())
        out.append(num / max(den, 1e-300))
    return out


def _event_ms(fn, stream=None):
    torch = _torch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1)


def time_fine_steps(fields, nx, ny, nz, dx, dt, steps, device):
    """Milliseconds for `steps` plain fine steps (FP64, u v w theta)."""
    torch = _torch()
    g = I.make_geometry(nx, ny, nz, dx, dx)
    A = [torch.from_numpy(fields[n]).to(device) for n in FIELDS]
    B = [torch.empty_like(x) for x in A]
    prof = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in (g.rdz, g.rho, g.rhon)]
    M.monc_step(A, B, dx, dx, prof, dt)         # warm-up
    state = [A, B]

    def run():
        a, b = state
        for _ in range(steps):
            M.monc_step(a, b, dx, dx, prof, dt)
            a, b = b, a

    return _event_ms(run)


def run_experiment(nx=512, ny=512, nz=128, seeds=range(2000, 2016), n_train=12, steps=200,
                   every=4, dt=0.5, dx=50.0, train_steps=3000, batch=8192, lr=1e-3,
                   coarse_steps=50, growth=1.01, device=None, log=None):
    """Fine runs -> restricted data -> training -> coarse runs on held-out seeds.

    Returns a dict with the one-step held-out loss (trained vs no correction),
    the coarse-run errors after `coarse_steps` steps against the restricted
    fine solution (plain and learned, per field), fallback counts, and the
    timings behind the speedup T_fine(steps) / T_coarse+MLP(coarse_steps)."""
    import concurrent.futures as cf
    torch = _torch()
    device = device or torch.device("cuda:0")
    say = log or (lambda m: None)
    seeds = list(seeds)
    series = []
    t_fine_runs = []
    with cf.ThreadPoolExecutor(2) as ex:
        nxt = ex.submit(fine_fields, seeds[0], nx, ny, nz, dx)
        first = None
        for n, sd in enumerate(seeds):
            f = nxt.result()
            if n + 1 < len(seeds):
                nxt = ex.submit(fine_fields, seeds[n + 1], nx, ny, nz, dx)
            if first is None:
                first = f
            series.append(fine_series(sd, nx, ny, nz, steps, every, dt, dx, device,
                                      timing=t_fine_runs, fields=f))
            say(f"  fine run seed {sd}: {t_fine_runs[-1]:.2f} s")
    t_fine = time_fine_steps(first, nx, ny, nz, dx, dt, steps, device)
    del first
    train_set, held = series[:n_train], series[n_train:]
    norm, scale = statistics(train_set)
    say(f"  input mean/std {['%.4g' % x for x in norm]}, residual scales {['%.4g' % x for x in scale]}")
    rmax = residual_extremes(series, scale)
    say(f"  largest |residual|/scale per field over all snapshots: {['%.3g' % x for x in rmax]}")
    model = Correction(device, seed=0, norm=norm, scale=scale, batch=batch)
    zero = Correction(device, seed=0, norm=norm, scale=scale, batch=batch)
    zero.params.zero_()
    M.monc_mlp_pack(zero.params, zero.wpack)
    t0 = time.perf_counter()
    hist = train(model, train_set, int(train_steps * 2 / 3), seed=1, lr=lr, log=say, every=500)
    hist += train(model, train_set, train_steps - int(train_steps * 2 / 3), seed=2, lr=lr * 0.3,
                  log=say, every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    def held_loss(mdl):
        rng = np.random.default_rng(99)
        return float(np.mean([mdl.evaluate_loss(ser, n, rng) for ser in held
                              for n in range(0, len(ser.tend), max(1, len(ser.tend) // 8))]))

    loss_zero, loss_trained = held_loss(zero), held_loss(model)
    # one training step on its own, timed on a separate copy of the network:
    # the fused step (two launches) as issued from Python (host sampling and a
    # copy of the cell list included), and its device work captured once in a
    # graph and replayed; the same step through the separate entry points (ten
    # launches), replayed likewise
    probe = Correction(device, seed=0, norm=norm, scale=scale, batch=batch)
    prng = np.random.default_rng(7)
    probe.train_step(train_set[0], 0, prng)
    treps = 50
    t_step = _event_ms(lambda: [probe.train_step(train_set[0], n % len(train_set[0].tend), prng)
                                for n in range(treps)]) / treps
    t_graph = t_graph_sep = None
    ser0 = train_set[0]
    nterm = 4 * batch
    probe.train_step_separate(ser0, 0, prng)  # leaves cx, cy, cells of one sample
    for fn, key in ((probe.device_step, "fused"), (probe.device_step_separate, "separate")):
        try:
            fn(ser0, 0, nterm)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                fn(ser0, 0, nterm)
            graph.replay()
            torch.cuda.synchronize()
            ms = _event_ms(lambda: [graph.replay() for _ in range(treps)]) / treps
            del graph
        except Exception as exc:  # graph capture unavailable: report the eager time only
            say(f"  training-step graph ({key}) not captured: {exc}")
            ms = None
        if key == "fused":
            t_graph = ms
        else:
            t_graph_sep = ms
    del probe
    nsteps = min(coarse_steps, len(held[0].tend))
    err_plain, err_learned, fb = [], [], [0, 0, 0]
    t_plain = t_learned = 0.0
    for ser in held:
        ref, ref0 = ser.snaps[nsteps], ser.snaps[0]
        for mdl, errs in ((None, err_plain), (model, err_learned)):
            runner = CoarseRunner(ser, mdl, growth=growth)
            runner.run(ser.snaps[0], 1)            # warm-up
            if mdl is not None:
                runner.flags.zero_()
            box = {}
            ms = _event_ms(lambda: box.setdefault("out", runner.run(ser.snaps[0], nsteps)))
            errs.append(errors(box["out"], ref, ref0))
            if mdl is None:
                t_plain += ms / len(held)
            else:
                t_learned += ms / len(held)
                fb = [a + b for a, b in zip(fb, runner.fallbacks())]
    # the fused gather + MLP over one coarse step's rows (both face orientations)
    runner = CoarseRunner(held[0], model, growth=growth)
    N = runner.N
    A0 = held[0].snaps[0]

    def infer():
        M.monc_mlp_infer(A0, model.norm, 2, model.params, model.wpack, runner.G)

    infer()
    reps = 20
    fwd_ms = _event_ms(lambda: [infer() for _ in range(reps)]) / reps
    flop = 2.0 * (M.MONC_MLP_NIN * M.MONC_MLP_H + M.MONC_MLP_H * M.MONC_MLP_H +
                  M.MONC_MLP_H * M.MONC_MLP_NOUT)
    mean = lambda errs: [float(np.mean([e[q] for e in errs])) for q in range(4)]
    return {
        "fine": [nx, ny, nz], "coarse": [nx // 4, ny // 4, nz // 4],
        "seeds_train": seeds[:n_train], "seeds_held_out": seeds[n_train:],
        "train_steps": train_steps, "batch_cells": batch, "train_s": t_train,
        "loss_first": hist[0][1], "loss_last": hist[-1][1],
        "held_out_loss_no_correction": loss_zero, "held_out_loss_trained": loss_trained,
        "coarse_steps": nsteps, "fields": FIELDS, "norm": norm, "scale": scale,
        "residual_max_over_scale": rmax,
        "err_plain": mean(err_plain), "err_learned": mean(err_learned),
        # per field: the plain coarse error over the learned one (> 1: the
        # correction helps)
        "gain": [p / l for p, l in zip(mean(err_plain), mean(err_learned))],
        # one training step as issued from Python (host sampling, a copy of
        # the cell list, two launches) and its device work replayed as a
        # graph; the separate entry points' ten launches replayed likewise
        "train_step_ms": t_step, "train_step_graph_ms": t_graph,
        "train_step_separate_graph_ms": t_graph_sep,
        "fallback_nonfinite": fb[0], "fallback_growth": fb[1], "theta_faces_clamped": fb[2],
        "t_fine_ms": t_fine, "t_coarse_plain_ms": t_plain, "t_coarse_learned_ms": t_learned,
        "speedup_vs_fine": t_fine / t_learned,
        "mlp_infer_ms": fwd_ms, "mlp_rows": 2 * N,
        "mlp_tflops": 2 * N * flop / (fwd_ms * 1e-3) / 1e12,
        # against the dense BF16 MFMA peak of the device (2.5 PFLOP/s)
        "mlp_frac_of_bf16_peak": 2 * N * flop / (fwd_ms * 1e-3) / 2.5e15,
    }
