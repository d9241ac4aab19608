"""GPU parity of the learned coarse-grid flux correction against the FP64 oracle.

Every kernel of the learned form is checked through the C ABI: the 4x
restriction against the C oracle, the BF16 features, each MLP layer (given the
GPU's own inputs to that layer, so the bound is FP32 accumulation, not
accumulated BF16 rounding), the parameter gradient, the loss and its gradient,
Adam, and the corrected step with its plain-step fallback.  A short training
run must lower the loss on held-out data.
"""
import sys

import numpy as np
import pytest

from gpu_util import dev, to_dev, torch
from oracle import mlp_ref as R
from oracle import pyoracle as O
from paper_2009_12850_amd import _lib as M
from paper_2009_12850_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    O.build(force=False)
    M.lib()


def bf16_bits_to_f64(t):
    T = torch()
    return t.view(T.bfloat16).double().cpu().numpy()


def fine_case(nx, ny, nz, seed, nscal=1):
    g = I.make_geometry(nx, ny, nz, dx=50.0, dy=50.0)
    f = I.make_fields(g, nscal, seed, amp=5.0)
    names = ["u", "v", "w"] + I.scalar_names(nscal)
    return g, [O.halo_fill(I.pad(f[n])) for n in names]


def coarse_state(NX, NY, NZ, seed):
    """A random coarse state (padded, halos unused) with realistic magnitudes."""
    rng = np.random.default_rng(seed)
    s = [rng.standard_normal((NX + 4, NY + 4, NZ)) * a + b
         for a, b in ((3.0, 1.0), (2.0, -0.5), (0.7, 0.0), (0.5, 300.0))]
    s[2][:, :, -1] = 0.0
    return s


@pytest.mark.parametrize("shape,nscal", [((32, 32, 32), 1), ((16, 24, 8), 2), ((8, 4, 128), 1),
                                         ((512, 512, 128), 1)])
def test_restriction_matches_oracle(shape, nscal):
    nx, ny, nz = shape
    say(f"restrict4 {shape} nscal={nscal}")
    g, host = fine_case(nx, ny, nz, 900 + nx + nscal, nscal)
    ref, gc = O.restrict4(host, g)
    T = torch()
    fine = to_dev(host)
    shc = (nx // 4 + 4, ny // 4 + 4, nz // 4)
    coarse = [T.zeros(shc, dtype=T.float64, device=dev()) for _ in host]
    prof_c = [T.zeros(nz // 4, dtype=T.float64, device=dev()) for _ in range(3)]
    M.monc_restrict4(fine, coarse, to_dev([g.rdz, g.rho, g.rhon]), prof_c)
    T.cuda.synchronize()
    for n, (a, b) in enumerate(zip(coarse, ref)):
        a, b = I.interior(a.cpu().numpy()), I.interior(b)
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        assert err <= 1e-14, (n, err)
    for a, b in zip(prof_c, (gc.rdz, gc.rho, gc.rhon)):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=1e-15, atol=0)


@pytest.mark.parametrize("orient", [0, 1])
def test_features_match_oracle(orient):
    NX, NY, NZ = 12, 10, 7
    say(f"features orient={orient}")
    s = coarse_state(NX, NY, NZ, 31 + orient)
    norm = [1.0, 3.0, -0.5, 2.0, 0.0, 0.7, 300.0, 0.5]
    T = torch()
    ds = to_dev(s)
    inner = [I.interior(a) for a in s]
    n = NX * NY * NZ
    X = T.zeros((n, R.K), dtype=T.int16, device=dev())
    M.monc_mlp_features(ds, norm, orient, None, X)
    rng = np.random.default_rng(5)
    cells = rng.integers(0, n, 300).astype(np.int32)
    Xs = T.zeros((300, R.K), dtype=T.int16, device=dev())
    M.monc_mlp_features(ds, norm, orient, to_dev([cells])[0], Xs)
    T.cuda.synchronize()
    for got, idx in ((X, np.arange(n)), (Xs, cells)):
        ref = R.bf16(R.features(inner, norm, orient, idx))
        g = bf16_bits_to_f64(got)
        bad = g != ref
        # (x - mean) * (1/std) on the GPU vs (x - mean) / std: equal after
        # rounding to BF16 unless a value sits on a rounding boundary.
        assert bad.sum() <= 2, bad.sum()
        if bad.any():
            assert np.all(np.abs(g[bad] - ref[bad]) <= 2.0 ** -7 * np.abs(ref[bad]))


def run_forward(X_host_bf16, params, m):
    T = torch()
    Xd = T.from_numpy(X_host_bf16.astype(np.float32)).to(dev()).to(T.bfloat16).view(T.int16)
    pd = T.from_numpy(params.astype(np.float32)).to(dev())
    wp = T.zeros(M.MONC_MLP_WPACK, dtype=T.int16, device=dev())
    M.monc_mlp_pack(pd, wp)
    Y = T.zeros((m, 4), dtype=T.float32, device=dev())
    H1 = T.zeros((m, 64), dtype=T.int16, device=dev())
    H2 = T.zeros_like(H1)
    Z1 = T.zeros((m, 64), dtype=T.float32, device=dev())
    Z2 = T.zeros_like(Z1)
    M.monc_mlp_forward(Xd, m, pd, wp, Y, H1, H2, Z1, Z2)
    T.cuda.synchronize()
    return Xd, pd, wp, Y, H1, H2, Z1, Z2


def layer_tol(A, W):
    """FP32-accumulation bound for rows of A @ W.T: a few ulps of sum |a w|."""
    return 64 * np.finfo(np.float32).eps * (np.abs(A) @ np.abs(W).T) + 1e-30


@pytest.mark.parametrize("m", [1, 127, 128, 1000])
def test_forward_layers_match_oracle(m):
    say(f"forward m={m}")
    rng = np.random.default_rng(100 + m)
    p = R.init_params(7).astype(np.float32).astype(np.float64)
    p[R.H * R.K:R.H * R.K + R.H] = rng.standard_normal(R.H) * 0.1        # nonzero b1
    X = rng.standard_normal((m, R.K))
    X[:, R.PAD] = 0.0
    Xb = R.bf16(X)
    _, _, _, Y, H1, H2, Z1, Z2 = run_forward(Xb, p, m)
    W1, b1, W2, b2, W3, b3 = R.unpack(p)
    W1b, W2b, W3b = R.bf16(W1), R.bf16(W2), R.bf16(W3)
    z1, h1 = Z1.double().cpu().numpy(), bf16_bits_to_f64(H1)
    z2, h2 = Z2.double().cpu().numpy(), bf16_bits_to_f64(H2)
    y = Y.double().cpu().numpy()
    # each layer from the GPU's own input to that layer
    assert np.all(np.abs(z1 - (Xb @ W1b.T + b1)) <= layer_tol(Xb, W1b))
    assert np.all(np.abs(z2 - (h1 @ W2b.T + b2)) <= layer_tol(h1, W2b))
    assert np.all(np.abs(y - (h2 @ W3b.T + b3)) <= layer_tol(h2, W3b))
    # activations: BF16(GELU(z)) of the GPU's z, to one BF16 ulp (at most 2^-7
    # relative); the FP32 GELU rarely moves a value across a rounding boundary
    for z, h in ((z1, h1), (z2, h2)):
        ref = R.bf16(R.gelu(z))
        assert np.all(np.abs(h - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
        assert (h != ref).mean() <= 0.01
    # end to end against the emulated oracle
    Yr, _ = R.forward(Xb, p, emulate=True)
    assert np.abs(y - Yr).max() <= 0.02 * np.abs(Yr).max()


@pytest.mark.parametrize("m", [64, 200, 4096, 32768])
def test_backward_matches_oracle(m):
    """The parameter gradient against the BF16-emulating FP64 oracle from the
    GPU's own activations, entry by entry within the bounds of
    backward_bounds (up to 32768 rows: the training batch)."""
    say(f"backward m={m}")
    T = torch()
    rng = np.random.default_rng(200 + m)
    p = R.init_params(11).astype(np.float32).astype(np.float64)
    X = rng.standard_normal((m, R.K))
    X[:, R.PAD] = 0.0
    Xd, pd, wp, Y, H1, H2, Z1, Z2 = run_forward(R.bf16(X), p, m)
    dY = (rng.standard_normal((m, 4)) / m).astype(np.float32)
    ws = T.zeros(M.monc_mlp_backward_workspace_bytes(m), dtype=T.uint8, device=dev())
    grad = T.zeros(R.NPARAM, dtype=T.float32, device=dev())
    dYd = T.from_numpy(dY).to(dev())
    M.monc_mlp_backward(Xd, H1, H2, Z1, Z2, dYd, m, wp, grad, ws)
    g1 = grad.double().cpu().numpy()
    grad2 = T.full_like(grad, np.nan)
    M.monc_mlp_backward(Xd, H1, H2, Z1, Z2, dYd, m, wp, grad2, ws)
    T.cuda.synchronize()
    assert T.equal(grad, grad2), "backward is not deterministic"
    _, b1, W2, b2, W3, b3 = R.unpack(p)
    cache = dict(Xb=bf16_bits_to_f64(Xd), Z1=Z1.double().cpu().numpy(), H1=bf16_bits_to_f64(H1),
                 Z2=Z2.double().cpu().numpy(), H2=bf16_bits_to_f64(H2), W2b=R.bf16(W2),
                 W3b=R.bf16(W3))
    ref = R.backward(dY.astype(np.float64), cache, emulate=True)
    gb, rb = R.unpack(g1), R.unpack(ref)
    bounds = backward_bounds(dY.astype(np.float64), cache, rb)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for name, a, b, bd in zip(names, gb, rb, bounds):
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
        worst = float(np.max(np.abs(a - b) / bd))
        say(f"  {name}: rel err {err:.2e}, largest |error| / entry bound {worst:.3f}")
        assert np.all(np.abs(a - b) <= bd), (name, worst)
    assert np.all(gb[0][:, R.PAD] == 0.0)


# FP32 unit roundoff, a bound on the relative error of the kernels' FP32
# GELU derivative (erfc fit 1.2e-7, exponential and products), and the
# allowance for FP32 accumulation of the sums over rows relative to the
# block's largest entry (the blocks that no BF16 rounding touches, W3, b3 and
# b2, come out near 3e-7)
U32 = 2.0 ** -24
DGELU = 1.0e-6
ACC = 1.0e-5


def bf16_spread(v, e):
    """Where rounding v to BF16 is ambiguous within +-e (the FP32 value the
    kernel rounds may lie anywhere in [v - e, v + e]), the largest change a
    different rounding can make; 0 where both ends round alike."""
    lo, hi, mid = R.bf16(v - e), R.bf16(v + e), R.bf16(v)
    return np.where(lo == hi, 0.0, np.maximum(np.abs(hi - mid), np.abs(mid - lo)))


def backward_bounds(dY, cache, ref):
    """Per entry bounds on |gpu - oracle| of the parameter gradient.  Both
    sides round dZ2 and dZ1 to BF16 before the products; they may round an
    entry differently only where its FP32 value lies within the kernel's
    arithmetic error of a rounding midpoint.  Such entries (and, through dH1,
    their effect on dZ1) are found from the oracle's own values; the bound of
    each gradient entry adds their largest possible effect to the FP32
    accumulation allowance."""
    Xb, Z1, H1, Z2 = cache["Xb"], cache["Z1"], cache["H1"], cache["Z2"]
    W2b, W3b = cache["W2b"], cache["W3b"]
    g2, g1 = R.gelu_grad(Z2), R.gelu_grad(Z1)
    v2 = (dY @ W3b) * g2                                   # dZ2 before rounding
    e2 = (np.abs(dY) @ np.abs(W3b)) * np.abs(g2) * (8 * U32 + DGELU)
    d2 = bf16_spread(v2, e2)
    dZ2b = R.bf16(v2)
    v1 = (dZ2b @ W2b) * g1                                 # dZ1 before rounding
    prop = (d2 @ np.abs(W2b)) * np.abs(g1)                 # through a flipped dZ2
    e1 = prop + (np.abs(dZ2b) @ np.abs(W2b)) * np.abs(g1) * (70 * U32 + DGELU)
    d1 = bf16_spread(v1, e1)
    acc = [ACC * np.abs(r).max() for r in ref]
    bW1 = d1.T @ np.abs(Xb) + acc[0]
    bb1 = e1.sum(axis=0) + acc[1]        # b1 sums the unrounded dZ1
    bW2 = d2.T @ np.abs(H1) + acc[2]
    return [bW1, bb1, bW2] + [np.full_like(r, a) for r, a in zip(ref[3:], acc[3:])]


def test_loss_matches_oracle():
    NX, NY, NZ, B = 10, 9, 6, 300
    say("loss")
    T = torch()
    rng = np.random.default_rng(41)
    c0 = coarse_state(NX, NY, NZ, 1)
    c1 = [a + 0.5 * rng.standard_normal(a.shape) for a in c0]
    c1[2][:, :, -1] = 0.0
    tend = [0.1 * rng.standard_normal(a.shape) for a in c0]
    dt, scale = 2.0, [0.3, 0.2, 0.05, 0.01]
    rho = np.exp(-np.arange(NZ) / 5.0) * 1.2
    rhon = np.exp(-(np.arange(NZ) + 0.5) / 5.0) * 1.2
    cells = rng.integers(0, NX * NY * NZ, B).astype(np.int32)
    cells[:3] = [NZ - 1, 2 * NZ - 1, NX * NY * NZ - 1]          # lid cells
    Y4 = rng.standard_normal((4 * B, 4)).astype(np.float32)
    k = cells % NZ
    j = (cells // NZ) % NY
    i = cells // (NZ * NY)
    tgt = np.stack([((c1[q] - c0[q]) / dt - tend[q])[i + 2, j + 2, k] / scale[q]
                    for q in range(4)], axis=1)
    rh = np.stack([rhon[k] / rhon[0], rhon[k] / rhon[0], rho[k] / rho[0], rhon[k] / rhon[0]],
                  axis=1)
    mask = np.ones((B, 4))
    mask[k == NZ - 1, 2] = 0.0
    loss_ref, dY_ref = R.loss_and_grad(Y4.astype(np.float64), tgt, rh, mask)
    dY = T.zeros((4 * B, 4), dtype=T.float32, device=dev())
    loss = T.zeros(1, dtype=T.float32, device=dev())
    ws = T.zeros(M.monc_mlp_loss_workspace_bytes(B), dtype=T.uint8, device=dev())
    M.monc_mlp_loss(T.from_numpy(Y4).to(dev()), B, to_dev([cells])[0], to_dev(c0), to_dev(c1),
                    to_dev(tend), dt, scale, to_dev([np.zeros(NZ), rho, rhon]),
                    1.0 / mask.sum(), dY, loss, ws)
    T.cuda.synchronize()
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    d = dY.double().cpu().numpy()
    assert np.abs(d - dY_ref).max() <= 1e-5 * np.abs(dY_ref).max()


def test_adam_and_pack_match_oracle():
    say("adam")
    T = torch()
    rng = np.random.default_rng(77)
    p = rng.standard_normal(R.NPARAM).astype(np.float32)
    m1 = (0.01 * rng.standard_normal(R.NPARAM)).astype(np.float32)
    m2 = (1e-4 * rng.random(R.NPARAM)).astype(np.float32)
    g = (0.1 * rng.standard_normal(R.NPARAM)).astype(np.float32)
    pd, m1d, m2d, gd = (T.from_numpy(a.copy()).to(dev()) for a in (p, m1, m2, g))
    wp = T.zeros(M.MONC_MLP_WPACK, dtype=T.int16, device=dev())
    M.monc_mlp_adam(pd, m1d, m2d, gd, 3, 1e-3, 0.9, 0.999, 1e-8, wp)
    T.cuda.synchronize()
    pr, mr, vr = R.adam(p.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64),
                        g.astype(np.float64), 3, lr=1e-3)
    got = pd.double().cpu().numpy()
    # an FP32 update: the step is lr-sized, computed to FP32 relative accuracy
    assert np.abs(got - pr).max() <= 1e-6 * np.abs(pr).max()
    # moments: FP32 sums of two terms, bounded by a few FP32 ulps of the terms
    eps32 = np.finfo(np.float32).eps
    g64 = g.astype(np.float64)
    bound1 = 4 * eps32 * (0.9 * np.abs(m1) + 0.1 * np.abs(g64))
    bound2 = 4 * eps32 * (0.999 * m2 + 0.001 * g64 * g64)
    assert np.all(np.abs(m1d.double().cpu().numpy() - mr) <= bound1)
    assert np.all(np.abs(m2d.double().cpu().numpy() - vr) <= bound2)
    W1, _, W2, _, W3, _ = R.unpack(pd.double().cpu().numpy())
    packed = bf16_bits_to_f64(wp)
    n1, n2 = R.H * R.K, R.H * R.H
    np.testing.assert_array_equal(packed[:n1], R.bf16(W1).ravel())
    np.testing.assert_array_equal(packed[n1:n1 + n2], R.bf16(W2).ravel())
    w3 = packed[n1 + n2:].reshape(32, R.H)
    np.testing.assert_array_equal(w3[:4], R.bf16(W3))
    assert np.all(w3[4:] == 0.0)


def train_case(NX, NY, NZ, B, seed):
    """Coarse snapshots, tendencies, profiles and B cells (lid cells and one
    cell outside the grid included) for a training step."""
    rng = np.random.default_rng(seed)
    c0 = coarse_state(NX, NY, NZ, seed)
    c1 = [a + 0.5 * rng.standard_normal(a.shape) for a in c0]
    c1[2][:, :, -1] = 0.0
    tend = [0.1 * rng.standard_normal(a.shape) for a in c0]
    rho = np.exp(-np.arange(NZ) / 5.0) * 1.2
    rhon = np.exp(-(np.arange(NZ) + 0.5) / 5.0) * 1.2
    n = NX * NY * NZ
    cells = np.sort(rng.integers(0, n, B)).astype(np.int32)
    cells[:min(B, 2)] = [NZ - 1, n - 1][:min(B, 2)]          # lid cells
    if B > 3:
        cells[B // 2] = n                                     # outside the grid
    return c0, c1, tend, rho, rhon, cells


@pytest.mark.parametrize("shape,B", [((12, 10, 7), 5), ((12, 10, 7), 300),
                                     ((128, 128, 32), 8192), ((128, 128, 32), 20000)])
def test_fused_train_step_matches_oracle(shape, B):
    """monc_mlp_train_step against the oracle.  Its rows are the separate
    entry points' rows (features, forward, loss), so the oracle's gradient is
    taken from those kernels' activations and dY and the fused gradient must
    lie within backward_bounds of it; the loss within a float rounding of the
    separate loss and 1e-5 of the oracle's; the Adam step and the pack as in
    test_adam_and_pack_match_oracle.  B = 5 (one partial chunk: every row
    weighs on the gradient, so a wrong feature would show), 300 (ragged
    chunks), the 8192-cell training batch (two chunks per workgroup) and
    20000 cells (four or five chunks per workgroup)."""
    NX, NY, NZ = shape
    say(f"fused training step {shape} B={B}")
    T = torch()
    c0, c1, tend, rho, rhon, cells = train_case(NX, NY, NZ, B, 61 + B)
    n = NX * NY * NZ
    norm = [1.0, 3.0, -0.5, 2.0, 0.0, 0.7, 300.0, 0.5]
    dt, scale = 2.0, [0.3, 0.2, 0.05, 0.01]
    k = cells % NZ
    valid = cells < n
    nterm = float(4 * valid.sum() - np.sum(valid & (k == NZ - 1)))
    d0, d1, dte = to_dev(c0), to_dev(c1), to_dev(tend)
    prof = to_dev([np.zeros(NZ), rho, rhon])
    p = R.init_params(17).astype(np.float32)
    rng = np.random.default_rng(3)
    m1 = (0.01 * rng.standard_normal(R.NPARAM)).astype(np.float32)
    m2 = (1e-4 * rng.random(R.NPARAM)).astype(np.float32)

    # the separate entry points: features of x(i), x(i-1), y(j), y(j-1)
    # rows (an outside cell gives four zero rows), forward, loss
    ci = np.where(valid, cells, 0)
    i, j = ci // (NY * NZ), (ci // NZ) % NY
    xm = np.where(valid, (((i - 1) % NX) * NY + j) * NZ + k, n).astype(np.int32)
    ym = np.where(valid, (i * NY + (j - 1) % NY) * NZ + k, n).astype(np.int32)
    cx, cy, cd = to_dev([np.concatenate([cells, xm]), np.concatenate([cells, ym]), cells])
    m = 4 * B
    pd = T.from_numpy(p.copy()).to(dev())
    wp = T.zeros(M.MONC_MLP_WPACK, dtype=T.int16, device=dev())
    M.monc_mlp_pack(pd, wp)
    X = T.zeros((m, R.K), dtype=T.int16, device=dev())
    M.monc_mlp_features(d0, norm, 0, cx, X.narrow(0, 0, 2 * B))
    M.monc_mlp_features(d0, norm, 1, cy, X.narrow(0, 2 * B, 2 * B))
    Y = T.zeros((m, 4), dtype=T.float32, device=dev())
    H1 = T.zeros((m, 64), dtype=T.int16, device=dev())
    H2 = T.zeros_like(H1)
    Z1 = T.zeros((m, 64), dtype=T.float32, device=dev())
    Z2 = T.zeros_like(Z1)
    M.monc_mlp_forward(X, m, pd, wp, Y, H1, H2, Z1, Z2)
    dY = T.zeros((m, 4), dtype=T.float32, device=dev())
    loss_sep = T.zeros(1, dtype=T.float32, device=dev())
    wsl = T.zeros(M.monc_mlp_loss_workspace_bytes(B), dtype=T.uint8, device=dev())
    M.monc_mlp_loss(Y, B, cd, d0, d1, dte, dt, scale, prof, 1.0 / nterm, dY, loss_sep, wsl)

    # the fused step, twice from the same start (determinism)
    ws = T.zeros(M.monc_mlp_train_workspace_bytes(B), dtype=T.uint8, device=dev())
    runs = []
    for _ in range(2):
        pf = T.from_numpy(p.copy()).to(dev())
        m1f, m2f = T.from_numpy(m1.copy()).to(dev()), T.from_numpy(m2.copy()).to(dev())
        wpf = wp.clone()
        grad = T.full((R.NPARAM,), np.nan, dtype=T.float32, device=dev())
        loss = T.full((1,), np.nan, dtype=T.float32, device=dev())
        M.monc_mlp_train_step(d0, d1, dte, norm, cd, dt, scale, prof, 1.0 / nterm, pf, m1f, m2f,
                              3, 1e-3, 0.9, 0.999, 1e-8, wpf, grad, loss, ws)
        runs.append((pf, m1f, m2f, wpf, grad, loss))
    T.cuda.synchronize()
    for a, b in zip(runs[0], runs[1]):
        assert T.equal(a, b), "the fused step is not deterministic"
    pf, m1f, m2f, wpf, grad, loss = runs[0]

    # loss
    Yh = Y.double().cpu().numpy()
    ls, lf = float(loss_sep.item()), float(loss.item())
    assert abs(lf - ls) <= 2 * np.finfo(np.float32).eps * ls, (lf, ls)
    ii, jj = i + 2, j + 2
    tgt = np.stack([((c1[q] - c0[q]) / dt - tend[q])[ii, jj, k] / scale[q] for q in range(4)],
                   axis=1)
    rh = np.stack([rhon[k] / rhon[0], rhon[k] / rhon[0], rho[k] / rho[0], rhon[k] / rhon[0]],
                  axis=1)
    mask = np.ones((B, 4))
    mask[k == NZ - 1, 2] = 0.0
    mask[~valid] = 0.0
    loss_ref, _ = R.loss_and_grad(Yh, tgt, rh, mask)
    assert abs(lf - loss_ref) <= 1e-5 * loss_ref

    # gradient against the oracle from the separate kernels' activations
    _, b1, W2, b2, W3, b3 = R.unpack(p.astype(np.float64))
    cache = dict(Xb=bf16_bits_to_f64(X), Z1=Z1.double().cpu().numpy(), H1=bf16_bits_to_f64(H1),
                 Z2=Z2.double().cpu().numpy(), H2=bf16_bits_to_f64(H2), W2b=R.bf16(W2),
                 W3b=R.bf16(W3))
    dYh = dY.double().cpu().numpy()
    ref = R.backward(dYh, cache, emulate=True)
    g = grad.double().cpu().numpy()
    gb, rb = R.unpack(g), R.unpack(ref)
    bounds = backward_bounds(dYh, cache, rb)
    # b3's gradient, the sum of dY over the rows, is exactly 0 (a cell's four
    # rows cancel: a constant flux has no divergence); its FP32 sum is bounded
    # by the recursive-summation bound (m - 1) u sum |dY|
    bounds[5] = np.maximum(bounds[5], m * U32 * np.abs(dYh).sum(axis=0))
    for name, a, b, bd in zip(["W1", "b1", "W2", "b2", "W3", "b3"], gb, rb, bounds):
        worst = float(np.max(np.abs(a - b) / bd))
        say(f"  {name}: largest |error| / entry bound {worst:.3f}")
        assert np.all(np.abs(a - b) <= bd), (name, worst)
    assert np.all(gb[0][:, R.PAD] == 0.0)

    # Adam on that gradient, and the pack of the new weights
    pr, mr, vr = R.adam(p.astype(np.float64), m1.astype(np.float64), m2.astype(np.float64), g, 3,
                        lr=1e-3)
    got = pf.double().cpu().numpy()
    assert np.abs(got - pr).max() <= 1e-6 * np.abs(pr).max()
    eps32 = np.finfo(np.float32).eps
    assert np.all(np.abs(m1f.double().cpu().numpy() - mr) <=
                  4 * eps32 * (0.9 * np.abs(m1) + 0.1 * np.abs(g)))
    assert np.all(np.abs(m2f.double().cpu().numpy() - vr) <=
                  4 * eps32 * (0.999 * m2 + 0.001 * g * g))
    W1n, _, W2n, _, W3n, _ = R.unpack(got)
    packed = bf16_bits_to_f64(wpf)
    n1, n2 = R.H * R.K, R.H * R.H
    np.testing.assert_array_equal(packed[:n1], R.bf16(W1n).ravel())
    np.testing.assert_array_equal(packed[n1:n1 + n2], R.bf16(W2n).ravel())
    w3 = packed[n1 + n2:].reshape(32, R.H)
    np.testing.assert_array_equal(w3[:4], R.bf16(W3n))
    assert np.all(w3[4:] == 0.0)


def corrected_case(NX, NY, NZ, seed, theta_scale=1.0):
    rng = np.random.default_rng(seed)
    s = coarse_state(NX, NY, NZ, seed)
    # a smooth theta with small noise: both monotone faces (where the clamp
    # can act) and local extrema
    x = np.arange(NX + 4)[:, None, None]
    y = np.arange(NY + 4)[None, :, None]
    s[3] = 300.0 + np.sin(0.9 * x) * np.cos(0.7 * y) + 0.05 * rng.standard_normal(s[3].shape)
    tend = [0.1 * rng.standard_normal(a.shape) for a in s]
    gx = rng.standard_normal((NX * NY * NZ, 4)).astype(np.float32)
    gy = rng.standard_normal((NX * NY * NZ, 4)).astype(np.float32)
    gx[:, 3] *= theta_scale
    gy[:, 3] *= theta_scale
    rdz = 1.0 / np.linspace(40.0, 80.0, NZ)
    rho = 1.2 * np.exp(-np.arange(NZ) / 7.0)
    rhon = 1.2 * np.exp(-(np.arange(NZ) + 0.5) / 7.0)
    return s, tend, gx, gy, rdz, rho, rhon


def run_correct(s, tend, gx, gy, rdz, rho, rhon, scale, dt, growth, dx=200.0, dy=200.0):
    T = torch()
    NX, NY, NZ = s[0].shape[0] - 4, s[0].shape[1] - 4, s[0].shape[2]
    out = [T.full(a.shape, np.nan, dtype=T.float64, device=dev()) for a in s]
    flags = T.zeros(4, dtype=T.int32, device=dev())
    ws = T.zeros(M.monc_correct_step_workspace_bytes(NX, NY, NZ), dtype=T.uint8, device=dev())
    M.monc_correct_step(to_dev(s), to_dev(tend), T.from_numpy(gx).to(dev()),
                        T.from_numpy(gy).to(dev()), out, dx, dy, scale,
                        to_dev([rdz, rho, rhon]), dt, growth, flags, ws)
    T.cuda.synchronize()
    return [o.cpu().numpy() for o in out], flags.cpu().numpy()


def oracle_correct(s, tend, gx, gy, rdz, rho, rhon, scale, dt, growth, dx=200.0, dy=200.0):
    return R.corrected_step([I.interior(a) for a in s], [I.interior(a) for a in tend], gx, gy,
                            dx, dy, scale, rdz, rho, rhon, dt, growth)


@pytest.mark.parametrize("shape,theta_scale", [((9, 7, 5), 1.0), ((16, 12, 8), 0.05),
                                               ((32, 32, 32), 0.3), ((128, 128, 32), 0.3)])
def test_corrected_step_matches_oracle_and_conserves(shape, theta_scale):
    NX, NY, NZ = shape
    say(f"correct_step {shape} theta_scale={theta_scale}")
    s, tend, gx, gy, rdz, rho, rhon = corrected_case(NX, NY, NZ, 3 + NX, theta_scale)
    scale, dt = [0.3, 0.2, 0.05, 0.01], 2.0
    out, flags = run_correct(s, tend, gx, gy, rdz, rho, rhon, scale, dt, 1e300)
    ref, (nonfin, grown, nclamp) = oracle_correct(s, tend, gx, gy, rdz, rho, rhon, scale, dt,
                                                  1e300)
    say(f"  clamped theta faces: gpu {flags[3]}, oracle {nclamp} of {2 * NX * NY * NZ}")
    assert flags[1] == 0 and flags[2] == 0 and nonfin == 0 and grown == 0
    # a face whose corrected value sits on the interval's end to within
    # rounding may be counted on one side or the other
    assert abs(int(flags[3]) - nclamp) <= 2 + 2e-6 * (2 * NX * NY * NZ)
    assert 0 < nclamp < 2 * NX * NY * NZ
    for q in range(4):
        a = I.interior(out[q])
        err = np.abs(a - ref[q]).max() / np.abs(ref[q]).max()
        assert err <= 1e-14, (q, err)
        # the correction adds no mass
        plain = I.interior(s[q]) + dt * I.interior(tend[q])
        w = (rho if q == 2 else rhon) / rdz
        dm = (a - plain) * w[None, None, :]
        if q == 2:
            dm = dm[:, :, :-1]
        assert abs(dm.sum()) <= 1e-12 * np.abs(dm).sum() + 1e-300


def test_corrected_step_falls_back_on_nonfinite_fluxes():
    NX, NY, NZ = 8, 8, 4
    say("correct_step non-finite fallback")
    s, tend, gx, gy, rdz, rho, rhon = corrected_case(NX, NY, NZ, 4)
    gx[17, 2] = np.nan
    out, flags = run_correct(s, tend, gx, gy, rdz, rho, rhon, [1.0] * 4, 2.0, 1e300)
    assert flags[1] == 1 and flags[2] == 0 and flags[3] == 0
    for q in range(4):
        ref = I.interior(s[q]) + 2.0 * I.interior(tend[q])
        if q == 2:
            ref[:, :, -1] = 0.0
        np.testing.assert_array_equal(I.interior(out[q]), ref)


def test_corrected_step_growth_guard():
    NX, NY, NZ = 12, 10, 6
    say("correct_step growth guard")
    s, tend, gx, gy, rdz, rho, rhon = corrected_case(NX, NY, NZ, 5)
    scale = [0.3, 0.2, 0.05, 0.01]
    for growth in (1e-6, 1e300):
        out, flags = run_correct(s, tend, gx, gy, rdz, rho, rhon, scale, 2.0, growth)
        ref, fl = oracle_correct(s, tend, gx, gy, rdz, rho, rhon, scale, 2.0, growth)
        assert flags[2] == fl[1] == (1 if growth < 1 else 0)
        for q in range(4):
            a = I.interior(out[q])
            assert np.abs(a - ref[q]).max() <= 1e-14 * np.abs(ref[q]).max()


def test_training_lowers_held_out_loss():
    """A short training run on restricted fine runs lowers the loss on a
    held-out run below that of the untrained network and of no correction."""
    from paper_2009_12850_amd import learned as L
    say("training")
    d = dev()
    train = [L.fine_series(s, 64, 64, 32, steps=24, every=4, dt=0.5, dx=50.0, device=d)
             for s in (11, 12)]
    held = L.fine_series(13, 64, 64, 32, steps=24, every=4, dt=0.5, dx=50.0, device=d)
    norm, scale = L.statistics(train)
    model = L.Correction(d, seed=3, norm=norm, scale=scale, batch=2048)
    T = torch()

    def held_loss(mdl):
        rng = np.random.default_rng(99)
        return np.mean([mdl.evaluate_loss(held, n, rng) for n in range(len(held.tend))])

    zero = L.Correction(d, seed=3, norm=norm, scale=scale, batch=2048)
    zero.params.zero_()
    M.monc_mlp_pack(zero.params, zero.wpack)
    base = held_loss(zero)
    before = held_loss(model)
    hist = L.train(model, train, steps=300, seed=1, lr=1e-3, log=say)
    after = held_loss(model)
    T.cuda.synchronize()
    say(f"  held-out loss: zero {base:.4f}, untrained {before:.4f}, trained {after:.4f}")
    assert np.isfinite(after)
    assert after < 0.9 * base and after < before


def test_experiment_driver_small():
    """The end-to-end driver (fine runs, restriction, training, held-out
    coarse runs plain and learned, timings) on a small grid."""
    from paper_2009_12850_amd import learned as L
    say("experiment driver, 64x64x32")
    r = L.run_experiment(nx=64, ny=64, nz=32, seeds=range(30, 34), n_train=3, steps=24,
                         train_steps=150, batch=1024, coarse_steps=6, device=dev(), log=say)
    say(f"  {r}")
    assert r["coarse"] == [16, 16, 8] and r["coarse_steps"] == 6
    assert all(np.isfinite(r["err_plain"])) and all(np.isfinite(r["err_learned"]))
    assert r["held_out_loss_trained"] < r["held_out_loss_no_correction"]
    # the trained correction lowers the multi-step coarse error of u, v and w
    # against the restricted fine solution; theta's error is reported, not
    # asserted (on the full-size experiment its correction changes it by less
    # than 0.1 %, with or without the clamp)
    for q, name in enumerate("uvw"):
        assert r["err_learned"][q] < r["err_plain"][q], (name, r["err_learned"], r["err_plain"])
    say(f"  theta: plain {r['err_plain'][3]:.4f}, learned {r['err_learned'][3]:.4f}")
    assert r["fallback_nonfinite"] == 0
    assert r["t_fine_ms"] > 0 and r["t_coarse_learned_ms"] > 0 and r["mlp_tflops"] > 0


@pytest.mark.parametrize("shape", [(12, 10, 7), (8, 12, 32), (6, 4, 32), (128, 128, 32)])
def test_inference_of_both_orientations_equals_each_alone(shape):
    """orient 2 (both face orientations; on staged grids from one staged tile
    per 128 rows) gives bitwise the x-face outputs of orient 0 followed by
    the y-face outputs of orient 1."""
    NX, NY, NZ = shape
    say(f"infer both {shape}")
    T = torch()
    s = to_dev(coarse_state(NX, NY, NZ, 70 + NZ))
    norm = [1.0, 3.0, -0.5, 2.0, 0.0, 0.7, 300.0, 0.5]
    p = T.from_numpy(R.init_params(17).astype(np.float32)).to(dev())
    p[R.H * R.K:R.H * R.K + R.H] = 0.05
    wp = T.zeros(M.MONC_MLP_WPACK, dtype=T.int16, device=dev())
    M.monc_mlp_pack(p, wp)
    n = NX * NY * NZ
    Y0 = T.full((n, 4), float("nan"), dtype=T.float32, device=dev())
    Y1 = T.full((n, 4), float("nan"), dtype=T.float32, device=dev())
    Y2 = T.full((2 * n, 4), float("nan"), dtype=T.float32, device=dev())
    M.monc_mlp_infer(s, norm, 0, p, wp, Y0)
    M.monc_mlp_infer(s, norm, 1, p, wp, Y1)
    M.monc_mlp_infer(s, norm, 2, p, wp, Y2)
    T.cuda.synchronize()
    assert T.equal(Y2[:n], Y0) and T.equal(Y2[n:], Y1)


@pytest.mark.parametrize("shape", [(12, 10, 7), (16, 16, 8), (5, 3, 33), (8, 12, 32), (3, 32, 4),
                                   (6, 4, 32), (128, 128, 32)])
@pytest.mark.parametrize("orient", [0, 1])
def test_fused_inference_equals_features_then_forward(shape, orient):
    """The fused gather + MLP kernel gives bitwise the outputs of the feature
    gather followed by the forward pass, over every cell.  Grids of 32 levels
    with ny a multiple of 4 take the LDS-staged gather, the others the direct
    one; (6, 4, 32) stages more columns than the grid has (periodic
    duplicates); (128, 128, 32) is the learned form's coarse grid."""
    NX, NY, NZ = shape
    say(f"infer {shape} orient={orient}")
    T = torch()
    s = to_dev(coarse_state(NX, NY, NZ, 60 + NZ))
    norm = [1.0, 3.0, -0.5, 2.0, 0.0, 0.7, 300.0, 0.5]
    p = T.from_numpy(R.init_params(13).astype(np.float32)).to(dev())
    p[R.H * R.K:R.H * R.K + R.H] = 0.05
    wp = T.zeros(M.MONC_MLP_WPACK, dtype=T.int16, device=dev())
    M.monc_mlp_pack(p, wp)
    n = NX * NY * NZ
    X = T.zeros((n, R.K), dtype=T.int16, device=dev())
    M.monc_mlp_features(s, norm, orient, None, X)
    Y1 = T.zeros((n, 4), dtype=T.float32, device=dev())
    M.monc_mlp_forward(X, n, p, wp, Y1)
    Y2 = T.full((n, 4), float("nan"), dtype=T.float32, device=dev())
    M.monc_mlp_infer(s, norm, orient, p, wp, Y2)
    T.cuda.synchronize()
    assert T.equal(Y1, Y2)
