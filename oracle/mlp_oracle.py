"""FP64 NumPy oracle of the column MLP (test infrastructure only).

Network y = W3 s(W2 s(W1 x + b1) + b2) + b3 with SiLU s(z) = z / (1 + e^-z),
parameters flattened in the order W1 [256][400], b1, W2 [256][256], b2,
W3 [192][256], b3; mean-squared-error loss; Adam (Kingma & Ba 2015) with
bias correction.  Column features and targets follow the definition used
by the library: per-field RMS scaling, linear resampling to 64 canonical
levels z_c = z_0 + H c / 63.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 400, 256, 192
SHAPES = [(HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)]


def unflatten(w):
    out, off = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(w[off:off + n], dtype=np.float64).reshape(s))
        off += n
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(w, x):
    W1, b1, W2, b2, W3, b3 = unflatten(w)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (x, z1, h1, z2, h2)


def backward(w, cache, dy):
    """Gradient of sum(y * dy) with respect to the flattened parameters."""
    W1, b1, W2, b2, W3, b3 = unflatten(w)
    x, z1, h1, z2, h2 = cache
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * dsilu(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return flatten([gW1, gb1, gW2, gb2, gW3, gb3])


def mse(y, t):
    return ((y - t) ** 2).mean()


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def column_features(b, lb, z, alpha):
    """b, lb: arrays [3][n_z][ncol] of (rho', w, theta') of the right-hand
    side and of L_v b; z: lattice levels.  Returns features [ncol][400] and
    the per-field scales [ncol][3]."""
    nz, ncol = b.shape[1], b.shape[2]
    # per-field scale: RMS over the column of b_f together with the
    # first-order correction alpha (L_v b)_f
    s = np.sqrt((b ** 2).mean(axis=1) + ((alpha * lb) ** 2).mean(axis=1)) + 1e-30   # [3][ncol]
    zc = z[0] + (z[-1] - z[0]) * np.arange(64) / 63.0
    feat = np.zeros((ncol, IN))
    for f in range(3):
        for c in range(ncol):
            feat[c, f * 64:(f + 1) * 64] = np.interp(zc, z, b[f, :, c]) / s[f, c]
            feat[c, 192 + f * 64:192 + (f + 1) * 64] = alpha * np.interp(zc, z, lb[f, :, c]) / s[f, c]
    feat[:, 384:387] = np.log10(s.T)
    feat[:, 387] = alpha / 10.0
    return feat, s.T


def column_targets(b, x, z, s):
    zc = z[0] + (z[-1] - z[0]) * np.arange(64) / 63.0
    ncol = b.shape[2]
    t = np.zeros((ncol, OUT))
    for f in range(3):
        for c in range(ncol):
            t[c, f * 64:(f + 1) * 64] = (np.interp(zc, z, x[f, :, c]) - np.interp(zc, z, b[f, :, c])) / s[c, f]
    return t
