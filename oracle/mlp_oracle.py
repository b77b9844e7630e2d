"""FP64 NumPy oracle of the column MLP (test infrastructure only).

Network y = W3 s(W2 s(W1 x + b1) + b2) + b3 + S x with SiLU
s(z) = z / (1 + e^-z) and a linear bypass S, parameters flattened in the
order W1 [256][208], b1, W2 [256][256], b2, W3 [256][256], b3, S [256][208];
mean-squared-error loss; Adam (Kingma & Ba 2015) with bias correction.

Column features, targets and the guess follow the definition used by the
library (the learned-guess design is this project's own; the paper has no
learned part):
  * fields (rho', w, theta') are made dimensionless level by level with the
    reference state: rho'/rho0, w/c0 (c0 = sqrt(gamma p0 / rho0)), theta'/theta0;
  * the default start x0 = b leaves the residual r = b - (I - alpha L_v) b
    = alpha L_v b, and the exact correction is x - b = (I - alpha L_v)^-1 r:
    a linear function of r alone.  The features are r (dimensionless)
    divided by one scale per column, s = RMS of the dimensionless r over the
    column's 3 n_z values, so that the correction is predicted relative to
    its own size and not to the size of b;
  * the canonical column is the 65 LGL nodes of 16 equal order-4 elements
    on the normalised height (z - z_0) / H; lattice data are resampled to it
    linearly in z, and the predicted correction back to the lattice levels
    the same way.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 208, 256, 256
NC = 65          # canonical levels
NF = 3 * NC      # used outputs (rho', w, theta' on the canonical levels)
SHAPES = [(HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,), (OUT, IN)]


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
    W1, b1, W2, b2, W3, b3, S = unflatten(w)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3 + x @ S.T
    return y, (x, z1, h1, z2, h2)


def backward(w, cache, dy):
    """Gradient of sum(y * dy) with respect to the flattened parameters."""
    W1, b1, W2, b2, W3, b3, S = unflatten(w)
    x, z1, h1, z2, h2 = cache
    gS = dy.T @ x
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * dsilu(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return flatten([gW1, gb1, gW2, gb2, gW3, gb3, gS])


def mse(y, t):
    return ((y - t) ** 2).mean()


def mse_grad(y, t):
    """Gradient of mse(y, t) with respect to y."""
    return 2.0 * (y - t) / y.size


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, ndecay=0):
    """Adam with bias correction; the first ndecay parameters also take
    decoupled weight decay wd (Loshchilov & Hutter 2019, AdamW):
    w - lr (m_hat / (sqrt(v_hat) + eps) + wd w)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    u = mh / (np.sqrt(vh) + eps)
    d = np.zeros_like(w)
    d[:ndecay] = wd * w[:ndecay]
    return w - lr * (u + d), m, v


def canonical_levels():
    """Normalised heights of the canonical column: LGL nodes of order 4 in
    each of 16 equal elements, shared element faces counted once."""
    from .oracle import lgl
    xi = np.asarray(lgl(4)[0], dtype=np.float64)
    zc = np.zeros(NC)
    for k in range(NC):
        e = min(k // 4, 15)
        zc[k] = (e + (xi[k - 4 * e] + 1.0) / 2.0) / 16.0
    return zc


def dimension_factors(rho0, p0, theta0, gamma):
    """Per-level factors D [3][n_z] that make (rho', w, theta') dimensionless."""
    c0 = np.sqrt(gamma * np.asarray(p0) / np.asarray(rho0))
    return np.stack([np.asarray(rho0, dtype=np.float64), c0, np.asarray(theta0, dtype=np.float64)])


def column_features(b, lb, z, alpha, D):
    """b, lb: arrays [3][n_z][ncol] of (rho', w, theta') of the right-hand
    side and of L_v b; z: lattice levels; D: dimension factors [3][n_z].
    Returns features [ncol][208] and the column scales s [ncol]: the
    dimensionless residual alpha L_v b / (D s) of the default start on the
    canonical levels (entries 0 .. 194), the scalars alpha / 10,
    100 alpha c0(z_0) / H, log10 H / 5 (195 .. 197), zeros to 207.  s is not
    a feature: the correction is homogeneous of degree one in r, so once r
    is divided by s the map does not depend on s."""
    nz, ncol = b.shape[1], b.shape[2]
    lh = alpha * lb / D[:, :, None]
    s = np.sqrt((lh ** 2).sum(axis=(0, 1)) / (3 * nz)) + 1e-300
    H = z[-1] - z[0]
    zc = z[0] + H * canonical_levels()
    feat = np.zeros((ncol, IN))
    for f in range(3):
        for c in range(ncol):
            feat[c, f * NC:(f + 1) * NC] = np.interp(zc, z, lh[f, :, c]) / s[c]
    feat[:, NF] = alpha / 10.0
    feat[:, NF + 1] = 100.0 * alpha * D[1, 0] / H
    feat[:, NF + 2] = np.log10(H) / 5.0
    return feat, s


def column_targets(b, x, z, D, s):
    """Scaled dimensionless correction (x - b) / (D s) on the canonical levels
    [ncol][256] (entries past 3 x 65 are zero)."""
    zc = z[0] + (z[-1] - z[0]) * canonical_levels()
    ncol = b.shape[2]
    d = (x - b) / D[:, :, None]
    t = np.zeros((ncol, OUT))
    for f in range(3):
        for c in range(ncol):
            t[c, f * NC:(f + 1) * NC] = np.interp(zc, z, d[f, :, c]) / s[c]
    return t


def column_guess(b, y, z, D, s):
    """Initial guess x0 = b + D s resample(y) on the lattice levels; the w
    correction is zero on the bottom and top levels (walls)."""
    zh = (z - z[0]) / (z[-1] - z[0])
    zc = canonical_levels()
    x0 = np.array(b, dtype=np.float64, copy=True)
    for f in range(3):
        for c in range(b.shape[2]):
            d = np.interp(zh, zc, y[c, f * NC:(f + 1) * NC])
            if f == 1:
                d[0] = 0.0
                d[-1] = 0.0
            x0[f, :, c] += D[f] * s[c] * d
    return x0
