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


def test_adamw_first_step_closed_form():
    """Decoupled weight decay on the first ndecay parameters: the first
    bias-corrected step moves those by lr (sign(g) + wd w), the rest by
    lr sign(g) (Loshchilov & Hutter 2019)."""
    rng = np.random.default_rng(2)
    w = rng.normal(size=40); g = rng.normal(size=40)
    w1, m, v = MO.adam(w, g, np.zeros(40), np.zeros(40), 1, lr=1e-3, eps=0.0, wd=0.25, ndecay=25)
    ref = w - 1e-3 * np.sign(g)
    ref[:25] -= 1e-3 * 0.25 * w[:25]
    np.testing.assert_allclose(w1, ref, rtol=0, atol=1e-15)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(MO.dsilu(z), (MO.silu(z + h) - MO.silu(z - h)) / (2 * h), atol=1e-8)


def test_canonical_levels():
    """65 points: element faces at e/16, interior points at the order-4 LGL
    nodes (0, +-sqrt(3/7)) of each element, increasing from 0 to 1."""
    zc = MO.canonical_levels()
    assert zc.size == 65 and zc[0] == 0.0 and zc[-1] == 1.0 and np.all(np.diff(zc) > 0)
    r = np.sqrt(3.0 / 7.0)
    for e in range(16):
        np.testing.assert_allclose(zc[4 * e:4 * e + 4],
                                   (e + (np.array([-1.0, -r, 0.0, r]) + 1.0) / 2.0) / 16.0, rtol=0, atol=1e-15)


def _dims(nz, rho=1.2, c=340.0, th=300.0, gamma=1.4):
    p0 = np.full(nz, c * c * rho / gamma)
    return MO.dimension_factors(np.full(nz, rho), p0, np.full(nz, th), gamma)


def test_column_features_on_linear_profiles():
    """Linear profiles survive the linear resampling exactly; the scale is
    the RMS of the dimensionless alpha L_v b (the default start's residual)
    alone, b itself enters only the targets."""
    z = np.linspace(0, 1000.0, 17)
    ncol = 3
    D = _dims(17)
    np.testing.assert_allclose(D[1], 340.0, rtol=1e-14)
    b = np.zeros((3, 17, ncol)); lb = np.zeros_like(b)
    for f in range(3):
        for c in range(ncol):
            b[f, :, c] = 1e3 * D[f] * (f + 1) * (c + 1) * (1.0 + z / 1000.0)
            lb[f, :, c] = -1e-3 * b[f, :, c]
    feat, s = MO.column_features(b, lb, z, alpha=2.0, D=D)
    zc = MO.canonical_levels()
    prof = 1.0 + z / 1000.0
    for c in range(ncol):
        # alpha L_v b / D = -2 (f+1)(c+1) prof: sum over fields of
        # 4 ((f+1)(c+1))^2 mean(prof^2), over 3 n_z values
        s_ref = np.sqrt(4.0 * (c + 1) ** 2 * (1 + 4 + 9) * (prof ** 2).mean() / 3.0)
        np.testing.assert_allclose(s[c], s_ref, rtol=1e-14)
        for f in range(3):
            np.testing.assert_allclose(feat[c, f * 65:(f + 1) * 65], -2.0 * (f + 1) * (c + 1) * (1 + zc) / s_ref,
                                       rtol=1e-13)
    assert feat.shape == (ncol, 208) and np.all(feat[:, 198:] == 0) and np.allclose(feat[:, 195], 0.2)
    np.testing.assert_allclose(feat[:, 196], 100.0 * 2.0 * 340.0 / 1000.0, rtol=1e-14)
    np.testing.assert_allclose(feat[:, 197], 3.0 / 5.0, rtol=1e-14)
    # x = b + 1e-3 b: the correction is 1e-3 b = -lb, i.e. -feat / alpha on the canonical levels
    t = MO.column_targets(b, b - lb, z, D, s)
    np.testing.assert_allclose(t[:, :195], -feat[:, :195] / 2.0, rtol=1e-13)
    assert np.all(t[:, 195:] == 0)


def test_column_guess_inverts_targets_on_the_canonical_grid():
    """On a column whose levels are the canonical ones, resampling is the
    identity: the guess built from the exact targets is the solution (the w
    correction vanishing on the walls, as L_v keeps w fixed there)."""
    H = 20e3
    z = 100.0 + H * MO.canonical_levels()
    rng = np.random.default_rng(4)
    D = _dims(65)
    b = rng.normal(size=(3, 65, 4)) * D[:, :, None]
    x = b + 0.1 * rng.normal(size=b.shape) * D[:, :, None]
    x[1, 0] = b[1, 0]
    x[1, -1] = b[1, -1]
    lb = rng.normal(size=b.shape)
    feat, s = MO.column_features(b, lb, z, 0.5, D)
    t = MO.column_targets(b, x, z, D, s)
    np.testing.assert_allclose(MO.column_guess(b, t, z, D, s), x, rtol=1e-12, atol=0)


def test_column_features_bounded_when_a_field_vanishes():
    """A residual with no w component and a tiny rho' one: one common scale
    keeps every feature O(1) and the ratios between the fields intact; a
    zero residual (b already the solution) gives zero features."""
    z = np.linspace(0, 1000.0, 17)
    D = _dims(17)
    b = np.zeros((3, 17, 2)); lb = np.zeros_like(b)
    b[1, :, 0] = 3.0
    lb[0, :, 0] = 1e-3 * np.cos(z / 300.0)
    lb[2, :, 0] = 0.5 * np.sin(z / 200.0)
    feat, s = MO.column_features(b, lb, z, alpha=3.0, D=D)
    assert np.all(np.abs(feat[:, :195]) <= np.sqrt(3 * 17.0) + 1e-12)
    k = 30
    np.testing.assert_allclose(feat[0, k] / feat[0, 2 * 65 + k],
                               np.interp(MO.canonical_levels()[k] * 1000.0, z, lb[0, :, 0] / D[0]) /
                               np.interp(MO.canonical_levels()[k] * 1000.0, z, lb[2, :, 0] / D[2]), rtol=1e-12)
    assert np.all(feat[0, 65:130] == 0)
    assert np.all(feat[1, :195] == 0) and np.all(np.isfinite(feat))


def test_exact_targets_are_one_linear_map_of_the_features(oracle_mod):
    """On a column grid equal to the canonical one (16 equal order-4
    elements, so the resampling is the identity) the exact target of every
    column is the same matrix applied to its features: the dimensionless
    (I - alpha L_v)^-1, from the oracle's own L_v and LAPACK solves, for
    right-hand sides of very different sizes and shapes."""
    from paper_2504_08157_amd import workloads as W
    ph = W.Physics(g=W.G)
    mesh = W.MeshSpec((1, 1, 16), 4, W.uniform_edges(0, 40e3, 1), W.uniform_edges(0, 40e3, 1),
                      W.uniform_edges(0, 20e3, 16), (True, True))
    o = oracle_mod.Oracle(mesh, ph)
    x, y, z = o.lattice_coords()
    rho0, th0 = W.constant_n_reference(z)
    o.set_reference(rho0, th0)
    Lm = oracle_mod.column_matrix(o)
    nz = o.nz
    assert nz == 65
    alpha = 2.0 * 0.29289321881345254
    A = np.eye(3 * nz) - alpha * Lm
    rng = np.random.default_rng(3)
    ncol = 6
    B = rng.normal(size=(3 * nz, ncol)) * np.logspace(-6, 3, ncol)[None, :]
    B[nz] = B[2 * nz - 1] = 0.0          # w right-hand side zero on the walls
    X = np.linalg.solve(A, B)
    LB = Lm @ B
    col = lambda M: M.reshape(3, nz, ncol)
    # dimension factors: any positive per-level factors serve the identity
    D = np.stack([rho0, np.full(nz, 340.0) * (1 + z / 4e4), th0])
    feat, s = MO.column_features(col(B), col(LB), z, alpha, D)
    T = MO.column_targets(col(B), col(X), z, D, s)
    Dv = D.reshape(-1)
    M = (np.linalg.inv(A) @ np.diag(Dv)) / Dv[:, None]     # D^-1 (I - alpha L)^-1 D
    for c in range(ncol):
        np.testing.assert_allclose(T[c, :195], M @ feat[c, :195], rtol=0,
                                   atol=1e-10 * np.abs(T[c, :195]).max())


def test_forward_closed_form():
    """A network with a handful of nonzero weights, evaluated by hand with
    sigmoid(ln 3) = 3/4, so silu(ln 3) = (3/4) ln 3 and silu(-ln 3) =
    -(1/4) ln 3.  Hidden unit 3 reads input 7 (W1[3, 7]: row = unit, column
    = input), unit 5 of layer 2 reads unit 3 (W2[5, 3]) with a bias that
    brings it back to ln 3, output 9 reads unit 5 of layer 2 (W3[9, 5]) and,
    through the bypass, input 7 (S[9, 7]); output 10 is a bias only, output
    11 a negative pre-activation.  A transposed operand, a dropped bias or
    bypass moves or changes these values."""
    ln3 = np.log(3.0)
    W1, b1, W2, b2, W3, b3, S = [np.zeros(s) for s in MO.SHAPES]
    W1[3, 7] = 1.0
    W1[4, 7] = -1.0
    W2[5, 3] = 1.0
    b2[5] = 0.25 * ln3                      # (3/4) ln 3 + (1/4) ln 3 = ln 3
    W3[9, 5] = 2.0
    b3[9] = 0.1
    S[9, 7] = -1.0
    b3[10] = 0.7
    W2[6, 4] = 4.0                          # 4 silu(-ln 3) = -ln 3
    W3[11, 6] = 1.0
    w = MO.flatten([W1, b1, W2, b2, W3, b3, S])
    x = np.zeros((2, MO.IN))
    x[0, 7] = ln3
    x[1, 2] = 5.0                           # reaches nothing
    y, (xc, z1, h1, z2, h2) = MO.forward(w, x)
    np.testing.assert_allclose(h1[0, 3], 0.75 * ln3, rtol=1e-15)
    np.testing.assert_allclose(h1[0, 4], -0.25 * ln3, rtol=1e-15)
    want = np.zeros(MO.OUT)
    want[9] = 2.0 * 0.75 * ln3 + 0.1 - ln3
    want[10] = 0.7
    want[11] = -0.25 * ln3                  # silu(-ln 3)
    np.testing.assert_allclose(y[0], want, rtol=1e-14, atol=1e-15)
    # row 1: every layer-1 unit is silu(0) = 0, so unit 5 of layer 2 sees
    # only its bias, silu((1/4) ln 3), and unit 6 is silu(0) = 0
    want1 = np.zeros(MO.OUT)
    zb = 0.25 * ln3
    want1[9] = 2.0 * zb / (1.0 + np.exp(-zb)) + 0.1
    want1[10] = 0.7
    np.testing.assert_allclose(y[1], want1, rtol=1e-14, atol=1e-15)


def test_mse_gradient_central_differences():
    rng = np.random.default_rng(2)
    y = rng.normal(size=(4, 7))
    t = rng.normal(size=(4, 7))
    g = MO.mse_grad(y, t)
    h = 1e-6
    for i in np.ndindex(y.shape):
        yp = y.copy(); yp[i] += h
        ym = y.copy(); ym[i] -= h
        fd = (MO.mse(yp, t) - MO.mse(ym, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-9, (i, fd, g[i])


def test_adam_second_step_closed_forms():
    """Constant gradient: the bias-corrected moments equal g and g^2 at every
    step, so each step moves by lr sign(g).  Gradient g then -g: the second
    step's corrected moments are -(1 - b1)/(1 + b1) g and g^2, a move of
    +lr (1 - b1)/(1 + b1) sign(g)."""
    rng = np.random.default_rng(3)
    w = rng.normal(size=40); g = rng.normal(size=40)
    lr, b1, b2 = 1e-2, 0.9, 0.999
    m = v = np.zeros(40)
    w1, m1, v1 = MO.adam(w, g, m, v, 1, lr, b1, b2, eps=0.0)
    w2, _, _ = MO.adam(w1, g, m1, v1, 2, lr, b1, b2, eps=0.0)
    np.testing.assert_allclose(w2, w - 2 * lr * np.sign(g), rtol=0, atol=1e-14)
    w2b, _, _ = MO.adam(w1, -g, m1, v1, 2, lr, b1, b2, eps=0.0)
    np.testing.assert_allclose(w2b, w1 + lr * (1 - b1) / (1 + b1) * np.sign(g), rtol=0, atol=1e-14)
