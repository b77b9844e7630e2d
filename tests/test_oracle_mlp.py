"""Pins of the MLP oracle: backward against central differences, Adam's
first step against its closed form, features against hand-built columns."""
import numpy as np

from oracle import mlp_oracle as MO


def _small_params(rng, scale=0.05):
    return rng.normal(scale=scale, size=sum(int(np.prod(s)) for s in MO.SHAPES))


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    w = _small_params(rng, 0.1)
    x = rng.normal(size=(5, MO.IN))
    t = rng.normal(size=(5, MO.OUT))
    y, cache = MO.forward(w, x)
    dy = 2 * (y - t) / y.size
    g = MO.backward(w, cache, dy)
    idx = rng.choice(w.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (MO.mse(MO.forward(wp, x)[0], t) - MO.mse(MO.forward(wm, x)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    w = rng.normal(size=50); g = rng.normal(size=50)
    w1, m, v = MO.adam(w, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    # bias-corrected first step moves every weight by lr * sign(g)
    np.testing.assert_allclose(w1, w - 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(MO.dsilu(z), (MO.silu(z + h) - MO.silu(z - h)) / (2 * h), atol=1e-8)


def test_column_features_on_linear_profiles():
    z = np.linspace(0, 1000.0, 17)
    ncol = 3
    b = np.zeros((3, 17, ncol)); lb = np.zeros_like(b)
    for f in range(3):
        for c in range(ncol):
            b[f, :, c] = (f + 1) * (c + 1) * (1.0 + z / 1000.0)
            lb[f, :, c] = -b[f, :, c]
    feat, s = MO.column_features(b, lb, z, alpha=2.0)
    zc = np.arange(64) / 63.0
    for f in range(3):
        for c in range(ncol):
            # scale = RMS of (b, alpha L_v b) = sqrt(1 + alpha^2) RMS(b) for lb = -b
            rms = np.sqrt(5.0) * np.sqrt((b[f, :, c] ** 2).mean())
            np.testing.assert_allclose(s[c, f], rms, rtol=1e-15)
            np.testing.assert_allclose(feat[c, f * 64:(f + 1) * 64], (f + 1) * (c + 1) * (1 + zc) / rms, rtol=1e-14)
            np.testing.assert_allclose(feat[c, 192 + f * 64:192 + (f + 1) * 64],
                                       -2.0 * (f + 1) * (c + 1) * (1 + zc) / rms, rtol=1e-14)
    assert np.all(feat[:, 388:] == 0) and np.allclose(feat[:, 387], 0.2)
    t = MO.column_targets(b, 2 * b, z, s)
    np.testing.assert_allclose(t, feat[:, :192], rtol=1e-14)


def test_column_features_bounded_when_a_field_vanishes():
    """w = 0 in b (a state at rest in the vertical) while L_v b has a w
    component: the w scale is that of alpha L_v b, every feature is O(1)."""
    z = np.linspace(0, 1000.0, 17)
    b = np.zeros((3, 17, 1)); lb = np.zeros_like(b)
    b[0, :, 0] = 1e-3 * np.cos(z / 300.0)
    b[2, :, 0] = 0.5 * np.sin(z / 200.0)
    lb[1, :, 0] = 2e-3 * np.sin(z / 250.0)
    feat, s = MO.column_features(b, lb, z, alpha=3.0)
    assert np.isclose(s[0, 1], 3.0 * np.sqrt((lb[1, :, 0] ** 2).mean()), rtol=1e-14)
    rows = np.sqrt(17.0)  # |v| / RMS(v) <= sqrt(n)
    assert np.all(np.abs(feat[:, :384]) <= rows + 1e-12)
