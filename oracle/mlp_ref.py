"""FP64 NumPy oracle of the learned coarse-grid flux correction.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product library.

The correction is a small MLP that maps the 5 x 5 x 3 neighbourhood of
(u, v, w, theta) around a coarse cell (300 standardised values) through two
64-unit GELU layers to 4 outputs: correction fluxes of u, v, w, theta through
one face of the cell.  x-faces use the neighbourhood as it is; y-faces use the
same network on the neighbourhood with x and y exchanged (and u, v swapped in
both inputs and outputs).  The correction tendency of field q at cell (i,j,k) is
    c_q = -[ g^x_q(i) - g^x_q(i-1) + g^y_q(j) - g^y_q(j-1) ] / rhohat_q(k),
a discrete flux divergence, so the correction conserves sum(rho_q c_q).  The
network is trained in BF16 with FP32 accumulation on the GPU; this oracle runs in
FP64 and, when `emulate` is set, rounds to BF16 exactly where the GPU kernels
do: the input features, the weights, the hidden activations, and the
back-propagated pre-activation gradients that feed matrix products.

Feature order: index f*80 + (a*5 + b)*3 + c for field f (u, v, w, theta),
a = offset along the face normal + 2, b = tangential offset + 2, c = vertical
offset + 1; periodic in x and y, edge-replicated in z; each field's slots
75..79 are 0 (300 values in 320 slots).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NIN, K, H, NOUT = 300, 320, 64, 4
FSTRIDE = 80                      # slots per field; 75 used
NPARAM = H * K + H + H * H + H + NOUT * H + NOUT
SWAP = [1, 0, 2, 3]
USED = np.array([f * FSTRIDE + p for f in range(4) for p in range(75)])
PAD = np.array([f * FSTRIDE + p for f in range(4) for p in range(75, FSTRIDE)])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * K].reshape(H, K); o += H * K
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + NOUT * H].reshape(NOUT, H); o += NOUT * H
    b3 = p[o:o + NOUT]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def init_params(seed):
    """Weights ~ N(0, 1/fan_in), biases 0; padded input columns zero."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, K)) / math.sqrt(NIN)
    W1[:, PAD] = 0.0
    W2 = rng.standard_normal((H, H)) / math.sqrt(H)
    W3 = rng.standard_normal((NOUT, H)) / math.sqrt(H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), W3, np.zeros(NOUT))


def features(state, norm, orient, cells):
    """state: 4 interior arrays (NX, NY, NZ) of u, v, w, theta; norm: [mean0,
    std0, ..., mean3, std3]; orient 0 (x-faces) or 1 (y-faces); cells: linear
    indices (i*NY + j)*NZ + k.  Returns [len(cells), 320]."""
    NX, NY, NZ = state[0].shape
    cells = np.asarray(cells)
    k = cells % NZ
    j = (cells // NZ) % NY
    i = cells // (NZ * NY)
    X = np.zeros((len(cells), K))
    for f in range(4):
        src = state[SWAP[f]] if orient == 1 else state[f]
        mean, std = norm[2 * SWAP[f] if orient == 1 else 2 * f], norm[2 * SWAP[f] + 1 if orient == 1 else 2 * f + 1]
        for a in range(5):
            for b in range(5):
                for c in range(3):
                    if orient == 0:
                        di, dj = a - 2, b - 2
                    else:
                        di, dj = b - 2, a - 2
                    ii = (i + di) % NX
                    jj = (j + dj) % NY
                    kk = np.clip(k + c - 1, 0, NZ - 1)
                    X[:, f * FSTRIDE + (a * 5 + b) * 3 + c] = (src[ii, jj, kk] - mean) / std
    return X


def forward(X, p, emulate=True):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    r = bf16 if emulate else (lambda x: np.asarray(x, dtype=np.float64))
    Xb, W1b, W2b, W3b = r(X), r(W1), r(W2), r(W3)
    Z1 = Xb @ W1b.T + b1
    H1 = r(gelu(Z1))
    Z2 = H1 @ W2b.T + b2
    H2 = r(gelu(Z2))
    Y = H2 @ W3b.T + b3
    return Y, dict(Xb=Xb, Z1=Z1, H1=H1, Z2=Z2, H2=H2, W1b=W1b, W2b=W2b, W3b=W3b)


def backward(dY, cache, emulate=True):
    r = bf16 if emulate else (lambda x: np.asarray(x, dtype=np.float64))
    Xb, Z1, H1, Z2, H2 = cache["Xb"], cache["Z1"], cache["H1"], cache["Z2"], cache["H2"]
    W2b, W3b = cache["W2b"], cache["W3b"]
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = dY @ W3b
    dZ2 = dH2 * gelu_grad(Z2)
    db2 = dZ2.sum(axis=0)
    dZ2b = r(dZ2)
    dW2 = dZ2b.T @ H1
    dH1 = dZ2b @ W2b
    dZ1 = dH1 * gelu_grad(Z1)
    db1 = dZ1.sum(axis=0)
    dZ1b = r(dZ1)
    dW1 = dZ1b.T @ Xb
    return pack(dW1, db1, dW2, db2, dW3, db3)


def correction(Yxp, Yxm, Yyp, Yym, rhohat):
    """c = -(gx(i) - gx(i-1) + gy(j) - gy(j-1)) / rhohat, y outputs swapped back."""
    return -(Yxp - Yxm + Yyp[:, SWAP] - Yym[:, SWAP]) / rhohat


def loss_and_grad(Y4, target, rhohat, mask):
    """Y4: [4B, 4] outputs ordered x(i), x(i-1), y(j), y(j-1) blocks of B rows;
    target, rhohat, mask: [B, 4].  Loss = sum(mask*(c - target)^2)/sum(mask)."""
    B = target.shape[0]
    Yxp, Yxm, Yyp, Yym = Y4[:B], Y4[B:2 * B], Y4[2 * B:3 * B], Y4[3 * B:]
    c = correction(Yxp, Yxm, Yyp, Yym, rhohat)
    err = (c - target) * mask
    n = mask.sum()
    loss = (err * err).sum() / n
    dc = 2.0 * err / n
    g = dc / rhohat
    dY = np.concatenate([-g, g, (-g)[:, SWAP], g[:, SWAP]])
    return loss, dY


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def _ultimate_interval(pU, pC, pD, c):
    """Admissible face values of the ULTIMATE universal limiter in normalised
    variables (Leonard 1991): with t = (phi - pU)/(pD - pU), a face whose
    upwind cell is not monotone between its neighbours (tC outside (0, 1))
    takes the upwind value; otherwise tC <= t_f <= min(1, tC/c).  Returns the
    QUICKEST face value limited to that range, and the range (lo, hi) in
    physical values, lo <= hi."""
    delta = pD - pU
    safe = np.where(delta != 0.0, delta, 1.0)
    tC = np.where(delta != 0.0, (pC - pU) / safe, -1.0)
    mono = (tC > 0.0) & (tC < 1.0)
    csafe = np.where(c > 0.0, c, 1.0)
    t_hi = np.where(c > 0.0, np.minimum(1.0, tC / csafe), 1.0)
    # QUICKEST: the centred value minus the upwind-biased Courant term and the
    # curvature term (1 - c^2)/6 * (pD - 2 pC + pU)
    quick = 0.5 * (pC + pD) - 0.5 * c * (pD - pC) - (1.0 - c * c) / 6.0 * (pD - 2.0 * pC + pU)
    tq = (quick - pU) / safe
    tf = np.clip(tq, tC, t_hi)
    f = np.where(mono, pU + tf * delta, pC)
    a, b = pU + tC * delta, pU + t_hi * delta
    lo = np.where(mono, np.minimum(a, b), pC)
    hi = np.where(mono, np.maximum(a, b), pC)
    return f, lo, hi


def _theta_face_correction(a, th_m1, th_0, th_p1, th_p2, dt_over_h, rhon_k, G):
    """Clamped theta correction flux through faces with normal velocity a,
    between cells 0 and +1 (neighbours -1 and +2 for the far-upwind values)."""
    c = np.abs(a) * dt_over_h
    pos = a >= 0.0
    pU = np.where(pos, th_m1, th_p2)
    pC = np.where(pos, th_0, th_p1)
    pD = np.where(pos, th_p1, th_0)
    f, lo, hi = _ultimate_interval(pU, pC, pD, c)
    moving = a != 0.0
    amass = np.where(moving, rhon_k * a, 1.0)
    trial = f + G / amass
    f_new = np.clip(trial, lo, hi)
    Geff = np.where(moving, amass * (f_new - f), 0.0)
    clamped = np.where(moving, (trial < lo) | (trial > hi), G != 0.0)
    return Geff, clamped


def corrected_step(state, tend, gx, gy, dx, dy, scale, rdz, rho, rhon, dt, growth):
    """The guarded corrected coarse step in FP64.

    state, tend: 4 interior arrays (NX, NY, NZ) of u, v, w, theta and their
    plain source terms; gx, gy: [NX*NY*NZ, 4] face outputs (gy in the exchanged
    frame).  u, v, w: c_q = -scale_q (div of g) / rhohat_q.  theta: face fluxes
    G = h rhon(0) scale_3 g clamped to the ULTIMATE admissible face values,
    then their divergence.  Plain step if any output is not finite, or if the
    kinetic energy or the mass-weighted theta variance of the corrected state
    exceeds `growth` times the plain one.  Returns (out, (nonfinite, grown,
    n_clamped_faces))."""
    NX, NY, NZ = state[0].shape
    plain = [state[q] + dt * tend[q] for q in range(4)]
    plain[2] = plain[2].copy()
    plain[2][:, :, -1] = 0.0
    if not (np.all(np.isfinite(gx)) and np.all(np.isfinite(gy))):
        return plain, (1, 0, 0)
    Gx = np.asarray(gx, np.float64).reshape(NX, NY, NZ, 4)
    Gy = np.asarray(gy, np.float64).reshape(NX, NY, NZ, 4)[..., SWAP]
    rh = [rhon / rhon[0], rhon / rhon[0], rho / rho[0]]
    out = []
    for q in range(3):
        div = Gx[..., q] - np.roll(Gx[..., q], 1, axis=0) + Gy[..., q] - np.roll(Gy[..., q], 1, axis=1)
        c = -scale[q] * div / rh[q][None, None, :]
        out.append(state[q] + dt * (tend[q] + c))
    th, u, v = state[3], state[0], state[1]
    rk = rhon[None, None, :]
    r = lambda f, s, ax: np.roll(f, -s, axis=ax)        # r(f, s, ax)[i] = f[i + s]
    Fx, cx = _theta_face_correction(u, r(th, -1, 0), th, r(th, 1, 0), r(th, 2, 0), dt / dx, rk,
                                    dx * rhon[0] * scale[3] * Gx[..., 3])
    Fy, cy = _theta_face_correction(v, r(th, -1, 1), th, r(th, 1, 1), r(th, 2, 1), dt / dy, rk,
                                    dy * rhon[0] * scale[3] * Gy[..., 3])
    cth = -((Fx - np.roll(Fx, 1, axis=0)) / dx + (Fy - np.roll(Fy, 1, axis=1)) / dy) / rk
    out.append(th + dt * (tend[3] + cth))
    out[2][:, :, -1] = 0.0
    m = (rhon / rdz)[None, None, :]
    mw = np.where(np.arange(NZ) < NZ - 1, rho / rdz, 0.0)[None, None, :]

    def ke(s):
        return np.sum(m * (s[0] ** 2 + s[1] ** 2)) + np.sum(mw * s[2] ** 2)

    def var(t):
        M = np.sum(m * np.ones_like(t))
        mean = np.sum(m * t) / M
        return np.sum(m * (t - mean) ** 2) / M

    nclamp = int(cx.sum() + cy.sum())
    if not (ke(out) <= growth * ke(plain) and var(out[3]) <= growth * var(plain[3])):
        return plain, (0, 1, nclamp)
    return out, (0, 0, nclamp)
