"""Float64 reference of the precision selector's features and network.

TEST INFRASTRUCTURE ONLY (imported by tests, never by the library).

The selector is not part of the paper; what is fixed here is its definition,
written out plainly so the device kernels can be compared with it:

* ``features(a)``: the 16 O(n^2) matrix features (list below).
* ``mlp_forward`` / ``mlp_loss_grad``: the 16 -> 64 -> 64 -> 3 network with
  ReLU hidden layers and a linear output, the mean squared error over the
  batch and the three outputs, and its exact gradient by the chain rule.
* ``adam_step``: one Adam update with bias correction.

Parameter vector layout (5443 float values): W1 (64 x 16, row-major), b1 (64),
W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3).
"""

from __future__ import annotations

import numpy as np

NFEAT = 16
H = 64
NOUT = 3
NPARAM = H * NFEAT + H + H * H + H + NOUT * H + NOUT  # 5443


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    w1 = p[o:o + H * NFEAT].reshape(H, NFEAT); o += H * NFEAT
    b1 = p[o:o + H]; o += H
    w2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + NOUT * H].reshape(NOUT, H); o += NOUT * H
    b3 = p[o:o + NOUT]; o += NOUT
    assert o == NPARAM
    return w1, b1, w2, b2, w3, b3


def _log10(x, floor=1e-30):
    return float(np.log10(max(float(x), floor)))


def features(a):
    """The 16 selector features of a square real or complex matrix.

    With F = ||A||_F, rms = F / sqrt(n), r_i = sum_{j != i} |a_ij| (Gershgorin
    radius), row/column norms and sums of |a_ij|:
      0  log2(n) / 10
      1  1 if A equals its transpose (conjugate transpose for complex) exactly
      2  log10(||A - A^T||_F / F + 1e-16) / 16   (A^H for complex)
      3  log10(max_i |a_ii| / rms)
      4  log10(min_i |a_ii| / rms)                (floor 1e-30)
      5  fraction of i with Re a_ii <= 0
      6  g / (1 + |g|),  g = min_i (Re a_ii - r_i) / rms
      7  fraction of i with Re a_ii - r_i <= 0
      8  log10(max row 2-norm / min row 2-norm)
      9  log10(max column 2-norm / min column 2-norm)
      10 log10(||A||_1 / F)
      11 log10(||A||_inf / F)
      12 log10(1 + n F^2 / |tr A|^2)
      13 Re tr(A^2) / F^2
      14 Re tr(A) / (sqrt(n) F)
      15 log10(max_i |a_ii| / min_i |a_ii|)      (floor 1e-30 on the minimum)
    """
    a = np.asarray(a)
    n = a.shape[0]
    az = a.astype(np.complex128)
    absa = np.abs(az)
    fro = float(np.sqrt(np.sum(absa ** 2)))
    rms = fro / np.sqrt(n)
    d = np.diag(az)
    ad = np.abs(d)
    is_c = np.iscomplexobj(a)
    at = az.conj().T if is_c else az.T
    sym = 1.0 if np.array_equal(az, at) else 0.0
    asym = float(np.sqrt(np.sum(np.abs(az - at) ** 2)))
    rad = absa.sum(axis=1) - ad
    g = float(np.min(d.real - rad)) / rms
    rown = np.sqrt((absa ** 2).sum(axis=1))
    coln = np.sqrt((absa ** 2).sum(axis=0))
    tr = complex(np.sum(d))
    tra2 = float(np.real(np.sum(az * az.T)))
    f = np.zeros(NFEAT)
    f[0] = np.log2(n) / 10.0
    f[1] = sym
    f[2] = np.log10(asym / fro + 1e-16) / 16.0
    f[3] = _log10(ad.max() / rms)
    f[4] = _log10(ad.min() / rms)
    f[5] = float(np.mean(d.real <= 0))
    f[6] = g / (1.0 + abs(g))
    f[7] = float(np.mean(d.real - rad <= 0))
    f[8] = _log10(rown.max() / max(rown.min(), 1e-300))
    f[9] = _log10(coln.max() / max(coln.min(), 1e-300))
    f[10] = _log10(absa.sum(axis=0).max() / fro)
    f[11] = _log10(absa.sum(axis=1).max() / fro)
    f[12] = np.log10(1.0 + n * fro ** 2 / max(abs(tr) ** 2, 1e-300))
    f[13] = tra2 / fro ** 2
    f[14] = tr.real / (np.sqrt(n) * fro)
    f[15] = _log10(ad.max() / max(ad.min(), 1e-30))
    return f


def relu(x):
    return np.maximum(x, 0.0)


def mlp_forward(p, x):
    """x: (B, 16) -> (h1, h2, out) with out (B, 3)."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = relu(x @ w1.T + b1)
    h2 = relu(h1 @ w2.T + b2)
    out = h2 @ w3.T + b3
    return h1, h2, out


def mlp_loss_grad(p, x, y):
    """Mean squared error over batch and outputs, and its gradient."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    bsz = x.shape[0]
    h1, h2, out = mlp_forward(p, x)
    diff = out - y
    loss = float(np.sum(diff ** 2) / (bsz * NOUT))
    dout = 2.0 * diff / (bsz * NOUT)
    gw3 = dout.T @ h2
    gb3 = dout.sum(axis=0)
    d2 = (dout @ w3) * (h2 > 0)
    gw2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ w2) * (h1 > 0)
    gw1 = d1.T @ x
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3])
    return loss, g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
