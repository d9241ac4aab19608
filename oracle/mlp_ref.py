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

Feature order: index ((f*5 + a)*5 + b)*3 + c for field f (u, v, w, theta),
a = offset along the face normal + 2, b = tangential offset + 2, c = vertical
offset + 1; periodic in x and y, edge-replicated in z; indices 300..319 are 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NIN, K, H, NOUT = 300, 320, 64, 4
NPARAM = H * K + H + H * H + H + NOUT * H + NOUT
SWAP = [1, 0, 2, 3]


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
    """Weights ~ N(0, 1/fan_in), biases 0; padded input columns 300..319 zero."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, K)) / math.sqrt(NIN)
    W1[:, NIN:] = 0.0
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
                    X[:, ((f * 5 + a) * 5 + b) * 3 + c] = (src[ii, jj, kk] - mean) / std
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
