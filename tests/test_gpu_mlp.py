"""GPU column-MLP kernels against the FP64 NumPy oracle (same FP16-rounded
weights and inputs): forward, backward, training, features, and the HEVI
initial-guess hook."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO
from paper_2504_08157_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _mlp_with_random_params(seed=3, B=128):
    import torch
    from paper_2504_08157_amd import nhsem
    rng = np.random.default_rng(seed)
    m = nhsem.ColumnMLP(max_batch=256)
    w = rng.normal(scale=0.08, size=m.nparam).astype(np.float32)
    m.nh_mlp_set_params(torch.from_numpy(w).cuda())
    x = rng.normal(size=(B, MO.IN)).astype(np.float16)
    # oracle uses the FP16 copies of the weights and FP32 biases
    parts = MO.unflatten(w.astype(np.float64))
    for i in (0, 2, 4, 6):   # W1, W2, W3 and the bypass S are used in FP16
        parts[i] = parts[i].astype(np.float16).astype(np.float64)
    wo = MO.flatten(parts)
    return m, torch, w, wo, x


def test_forward_matches_oracle():
    m, torch, w, wo, x = _mlp_with_random_params()
    y = m.nh_mlp_forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yo, _ = MO.forward(wo, x.astype(np.float64))
    assert _rel(y, yo) <= 5e-3, _rel(y, yo)


def test_backward_matches_oracle():
    m, torch, w, wo, x = _mlp_with_random_params(seed=4)
    rng = np.random.default_rng(9)
    dy = rng.normal(size=(x.shape[0], MO.OUT)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    m.nh_mlp_forward(xd)
    m.nh_mlp_backward(xd, torch.from_numpy(dy).cuda())
    _, g = m.nh_mlp_params()
    g = g.cpu().numpy().astype(np.float64)
    _, cache = MO.forward(wo, x.astype(np.float64))
    go = MO.backward(wo, cache, dy.astype(np.float64))
    for i, (a, b) in enumerate(zip(MO.unflatten(g), MO.unflatten(go))):
        assert _rel(a, b) <= 5e-3, (i, _rel(a, b))


def test_training_reduces_loss():
    import torch
    from paper_2504_08157_amd import nhsem
    rng = np.random.default_rng(5)
    m = nhsem.ColumnMLP(max_batch=512, seed=7)
    X = rng.normal(size=(512, MO.IN)).astype(np.float16)
    A = rng.normal(scale=0.05, size=(MO.IN, MO.OUT))
    T = (X.astype(np.float64) @ A).astype(np.float32)
    xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    first = None
    for it in range(300):
        m.nh_mlp_train_step(xd, td, lr=2e-3, loss=loss)
        if it == 0:
            first = loss.item()
    last = loss.item()
    assert last < 0.2 * first, (first, last)


def test_features_match_oracle(oracle_mod):
    import torch
    from paper_2504_08157_amd import nhsem
    ph = W.Physics()
    mesh = W.MeshSpec((3, 2, 4), 4, W.uniform_edges(0, 30e3, 3), W.uniform_edges(0, 20e3, 2),
                      W.stretched_edges(0, 15e3, 4, seed=8), (True, True))
    ctx = nhsem.Context(mesh, ph)
    orc = oracle_mod.Oracle(mesh, ph)
    g = ctx.nh_lattice_coords(); o = orc.lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    orc.set_reference(*W.constant_n_reference(o[2]))
    bq = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=2, walls=(False, False))
    xq = 1.3 * bq
    m = nhsem.ColumnMLP(max_batch=64)
    feat, scale, tgt = m.nh_mlp_samples(ctx, 0.7, torch.from_numpy(bq).cuda(), torch.from_numpy(xq).cuda())
    lb = orc.lv_apply(bq)
    sel = lambda a: np.stack([a[0], a[3], a[4]]).reshape(3, orc.nz, -1)
    rho0, th0 = W.constant_n_reference(o[2])
    D = MO.dimension_factors(rho0, orc.reference_pressure(), th0, ph.cp / ph.cv)
    fo, so = MO.column_features(sel(bq), sel(lb), o[2], 0.7, D)
    to = MO.column_targets(sel(bq), sel(xq), o[2], D, so)
    np.testing.assert_allclose(scale.cpu().numpy(), so, rtol=1e-12)
    assert _rel(feat.cpu().numpy().astype(np.float64), fo) <= 2e-3
    assert _rel(tgt.cpu().numpy(), to) <= 1e-6


def test_samples_of_a_given_start_match_oracle(oracle_mod):
    """nh_mlp_samples with a start x0 (the samples of a refinement pass):
    features of the residual b - (I - alpha L_v) x0 and targets x - x0,
    against the oracle's residual (its own L_v) and feature and target
    definitions."""
    import torch
    from paper_2504_08157_amd import nhsem
    ph = W.Physics()
    mesh = W.MeshSpec((3, 2, 4), 4, W.uniform_edges(0, 30e3, 3), W.uniform_edges(0, 20e3, 2),
                      W.stretched_edges(0, 15e3, 4, seed=8), (True, True))
    ctx = nhsem.Context(mesh, ph)
    orc = oracle_mod.Oracle(mesh, ph)
    g = ctx.nh_lattice_coords(); o = orc.lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    orc.set_reference(*W.constant_n_reference(o[2]))
    rho0, th0 = W.constant_n_reference(o[2])
    bq = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=2, walls=(False, False))
    xq = 1.3 * bq
    sel = lambda a: np.stack([a[0], a[3], a[4]]).reshape(3, orc.nz, -1)
    rng = np.random.default_rng(5)
    x0 = sel(bq) * (1.0 + 0.01 * rng.normal(size=sel(bq).shape))
    alpha = 0.7
    m = nhsem.ColumnMLP(max_batch=64)
    feat, scale, tgt = m.nh_mlp_samples(ctx, alpha, torch.from_numpy(bq).cuda(), torch.from_numpy(xq).cuda(),
                                        x0=torch.from_numpy(np.ascontiguousarray(x0.reshape(-1))).cuda())
    full = np.zeros_like(bq)
    full[0], full[3], full[4] = (x0[f].reshape(bq[0].shape) for f in range(3))
    r = sel(bq) - x0 + alpha * sel(orc.lv_apply(full))
    D = MO.dimension_factors(rho0, orc.reference_pressure(), th0, ph.cp / ph.cv)
    fo, so = MO.column_features(x0, r / alpha, o[2], alpha, D)
    to = MO.column_targets(x0, sel(xq), o[2], D, so)
    np.testing.assert_allclose(scale.cpu().numpy(), so, rtol=1e-10)
    assert _rel(feat.cpu().numpy().astype(np.float64), fo) <= 2e-3
    assert _rel(tgt.cpu().numpy(), to) <= 1e-6


@pytest.mark.parametrize("nelz,tol", [(4, 5e-3), (17, 1e-12)], ids=["residual_in_kernel", "residual_from_lv"])
def test_fused_guess_matches_separate_kernels(oracle_mod, nelz, tol):
    """The one-kernel inference of nh_mlp_guess (features, network and
    resampling in LDS) against the separate L_v, feature and forward kernels
    followed by the oracle's resampling, on a ragged column count (117).
    Columns of at most 65 levels (n_z = 17 here) compute their residual
    inside the inference kernel and keep it as FP32 between the walk and
    the resampling, so a feature can round to the neighbouring FP16 value:
    the correction agrees to that rounding.  Taller columns (n_z = 69) read
    L_v b from the separate kernel: the same arithmetic, to 1e-12."""
    import torch
    from paper_2504_08157_amd import nhsem
    ph = W.Physics()
    mesh = W.MeshSpec((3, 2, nelz), 4, W.uniform_edges(0, 30e3, 3), W.uniform_edges(0, 20e3, 2),
                      W.stretched_edges(0, 15e3, nelz, seed=8), (True, True))
    ctx = nhsem.Context(mesh, ph)
    orc = oracle_mod.Oracle(mesh, ph)
    g = ctx.nh_lattice_coords(); o = orc.lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    orc.set_reference(*W.constant_n_reference(o[2]))
    bq = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=4, walls=(False, False))
    ncol = ctx.nx * ctx.ny
    m = nhsem.ColumnMLP(max_batch=128)
    rng = np.random.default_rng(12)
    m.nh_mlp_set_params(torch.from_numpy(rng.normal(scale=0.03, size=m.nparam).astype(np.float32)).cuda())
    alpha = 0.9
    bd = torch.from_numpy(bq).cuda()
    x0 = m.nh_mlp_guess(ctx, alpha, bd).cpu().numpy().reshape(3, orc.nz, ncol)
    feat, scale, _ = m.nh_mlp_samples(ctx, alpha, bd)
    fpad = torch.zeros((128, MO.IN), dtype=torch.float16, device="cuda")
    fpad[:ncol] = feat
    y = m.nh_mlp_forward(fpad).cpu().numpy()[:ncol].astype(np.float64)
    sel = lambda a: np.stack([a[0], a[3], a[4]]).reshape(3, orc.nz, -1)
    rho0, th0 = W.constant_n_reference(o[2])
    D = MO.dimension_factors(rho0, orc.reference_pressure(), th0, ph.cp / ph.cv)
    ref = MO.column_guess(sel(bq), y, o[2], D, scale.cpu().numpy())
    corr, corr_ref = x0 - sel(bq), ref - sel(bq)
    assert np.linalg.norm(corr_ref) > 1e-3 * np.linalg.norm(sel(bq))   # the network changes the guess
    assert _rel(corr, corr_ref) <= tol, _rel(corr, corr_ref)


def test_fused_guess_and_forward_repeatable():
    """The same input three times: the fused guess (16,384 columns, 256
    workgroups of the inference kernel) and the forward GEMMs return the
    same bits every time."""
    import torch
    from paper_2504_08157_amd import nhsem
    w = W.cfg_hevi()
    w.mesh = W._tc_mesh(32, 32, 6)
    ctx = nhsem.Context(w.mesh, w.phys)
    g = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.reference_profiles(w, g[2]))
    assert ctx.nx * ctx.ny == 16384
    m = nhsem.ColumnMLP(max_batch=16384)
    rng = np.random.default_rng(21)
    m.nh_mlp_set_params(torch.from_numpy(rng.normal(scale=0.05, size=m.nparam).astype(np.float32)).cuda())
    b = torch.from_numpy(W.smooth_random_state(*g, *W.reference_profiles(w, g[2]), seed=5,
                                               walls=(False, False))).cuda()
    x = torch.from_numpy(rng.normal(size=(16384, MO.IN)).astype(np.float16)).cuda()
    ref_g = m.nh_mlp_guess(ctx, 0.7, b).clone()
    ref_y = m.nh_mlp_forward(x).clone()
    assert torch.isfinite(ref_g).all() and torch.isfinite(ref_y).all()
    for _ in range(2):
        assert torch.equal(m.nh_mlp_guess(ctx, 0.7, b), ref_g)
        assert torch.equal(m.nh_mlp_forward(x), ref_y)


def test_untrained_guess_equals_default(oracle_mod):
    import torch
    from paper_2504_08157_amd import nhsem
    w = W.cfg_hevi()
    w.mesh = W._tc_mesh(4, 4, 4)
    ctx = nhsem.Context(w.mesh, w.phys)
    g = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    ctx.nh_hevi_attach()
    q0 = torch.from_numpy(W.initial_state(w, *g)).cuda()
    ctx.nh_set_state(q0)
    st0 = ctx.nh_hevi_step(0.0, 2.0)
    a = ctx.nh_get_state().cpu().numpy()
    m = nhsem.ColumnMLP(max_batch=64)  # last layer zero: guess = right-hand side
    ctx.nh_set_state(q0)
    st1 = ctx.nh_hevi_step(0.0, 2.0, guess=m)
    b = ctx.nh_get_state().cpu().numpy()
    assert st0.iters_total == st1.iters_total
    np.testing.assert_array_equal(a, b)


def test_learned_guess_reduces_iterations():
    """Train on solves the method generates (a small TC mesh, the first ten
    steps of the evaluation mesh, random column right-hand sides on its
    grid, then a fine-tune on that grid with hidden-path decay and
    refinement-pass samples), evaluate on the 100 held-out steps that
    follow (steps 11-110): fewer Arnoldi steps per solve with one network
    pass and far fewer with three, final states equal to the solver
    tolerance.  (Wall time is measured by the hevi bench on the full case;
    on this 12 x 12 x 16 mesh a step is launch-bound.)"""
    from paper_2504_08157_amd import learned_guess as LG
    from paper_2504_08157_amd import nhsem
    mlp = nhsem.ColumnMLP(max_batch=16384, seed=7)
    wtr = W.cfg_hevi(); wtr.mesh = W._tc_mesh(16, 16, 6)
    wev = W.cfg_hevi(); wev.mesh = W._tc_mesh(12, 12, 16)
    wr = W.cfg_hevi(); wr.mesh = W._tc_mesh(32, 32, 16)   # the same column grid, 16384 columns per batch
    tr = LG.fit(mlp, wev, 2.0, 10, [(wtr, 1, 2.0)], epochs=40, batch=1024, lr=1e-3, random_grid=wr,
                random_batches=24, finetune_epochs=60, finetune_batch=4096, finetune_decay=3.0,
                refine_random_batches=8)
    print("training", tr)
    assert tr["loss_last"] < 0.01 * tr["loss_untrained"], tr
    res = LG.compare(mlp, wev, warm=10, held=100, dt=2.0, restart=10, refine_passes=3)
    print({k: res[k]["iters_per_solve"] for k in ("default", "mlp", "mlp_refined")})
    assert res["mlp"]["iters_per_solve"] < res["default"]["iters_per_solve"], res
    assert res["mlp_refined"]["iters_per_solve"] < 0.85 * res["default"]["iters_per_solve"], res
    assert res["state_rel_diff_stacked"] < 1e-8, res
    assert res["state_rel_diff_stacked_refined"] < 1e-8, res


def test_train_step_matches_oracle():
    """One nh_mlp_train_step against the oracle's forward, MSE gradient and
    backward on the same FP16-rounded weights and inputs (loss and every
    gradient tensor to 5e-3, the FP16 forward's accuracy), and its Adam
    update against the oracle's Adam applied to the step's own gradient
    (FP32 arithmetic: 1e-5 of the update)."""
    m, torch, w, wo, x = _mlp_with_random_params(seed=11)
    rng = np.random.default_rng(12)
    t = rng.normal(scale=0.5, size=(x.shape[0], MO.OUT)).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    m.nh_mlp_train_step(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), lr=lr, b1=b1, b2=b2, eps=eps,
                        loss=loss)
    w1, g = m.nh_mlp_params()
    w1, g = w1.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    yo, cache = MO.forward(wo, x.astype(np.float64))
    to = t.astype(np.float64)
    lo = MO.mse(yo, to)
    assert abs(loss.item() - lo) <= 5e-3 * lo, (loss.item(), lo)
    go = MO.backward(wo, cache, MO.mse_grad(yo, to))
    for i, (a, b) in enumerate(zip(MO.unflatten(g), MO.unflatten(go))):
        assert _rel(a, b) <= 5e-3, (i, _rel(a, b))
    w0 = w.astype(np.float64)
    z = np.zeros_like(w0)
    wa, _, _ = MO.adam(w0, g, z, z, 1, lr, b1, b2, eps)
    assert np.linalg.norm(w1 - wa) <= 1e-5 * np.linalg.norm(wa - w0)


def test_adam_step_matches_oracle():
    """nh_mlp_adam_step three times on the gradient of one backward pass
    against the oracle's Adam over the same three steps (FP32 moments)."""
    m, torch, w, wo, x = _mlp_with_random_params(seed=13)
    rng = np.random.default_rng(14)
    dy = rng.normal(size=(x.shape[0], MO.OUT)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    m.nh_mlp_forward(xd)
    m.nh_mlp_backward(xd, torch.from_numpy(dy).cuda())
    lr, b1, b2, eps = 2e-3, 0.8, 0.99, 1e-6
    wa = w.astype(np.float64)
    _, g = m.nh_mlp_params()
    g = g.cpu().numpy().astype(np.float64)
    mo = vo = np.zeros_like(wa)
    for step in range(1, 4):
        m.nh_mlp_adam_step(lr, b1, b2, eps)
        wa, mo, vo = MO.adam(wa, g, mo, vo, step, lr, b1, b2, eps)
    w3, _ = m.nh_mlp_params()
    w3 = w3.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(w3 - wa) <= 1e-5 * np.linalg.norm(wa - w.astype(np.float64))
    # bad hyper-parameters are refused
    from paper_2504_08157_amd import nhsem
    with pytest.raises(nhsem.NHError):
        m.nh_mlp_adam_step(lr=-1.0)


def test_adam_step_with_hidden_path_decay_matches_oracle():
    """nh_mlp_set_decay: three Adam steps with decoupled weight decay on the
    hidden path (every parameter before the bypass S) against the oracle's
    AdamW on the same gradient; the bypass takes plain Adam."""
    m, torch, w, wo, x = _mlp_with_random_params(seed=15)
    rng = np.random.default_rng(16)
    dy = rng.normal(size=(x.shape[0], MO.OUT)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    m.nh_mlp_forward(xd)
    m.nh_mlp_backward(xd, torch.from_numpy(dy).cuda())
    lr, b1, b2, eps, wd = 2e-3, 0.8, 0.99, 1e-6, 0.5
    m.nh_mlp_set_decay(wd)
    nd = w.size - MO.OUT * MO.IN
    wa = w.astype(np.float64)
    _, g = m.nh_mlp_params()
    g = g.cpu().numpy().astype(np.float64)
    mo = vo = np.zeros_like(wa)
    for step in range(1, 4):
        m.nh_mlp_adam_step(lr, b1, b2, eps)
        wa, mo, vo = MO.adam(wa, g, mo, vo, step, lr, b1, b2, eps, wd=wd, ndecay=nd)
    w3, _ = m.nh_mlp_params()
    w3 = w3.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(w3 - wa) <= 1e-5 * np.linalg.norm(wa - w.astype(np.float64))
    # the decay reaches the hidden path and only it
    wplain, _, _ = MO.adam(w.astype(np.float64), g, 0 * g, 0 * g, 1, lr, b1, b2, eps)
    assert not np.allclose(wa[:nd], wplain[:nd])
    from paper_2504_08157_amd import nhsem
    with pytest.raises(nhsem.NHError):
        m.nh_mlp_set_decay(-1.0)


def _canonical_column_case(oracle_mod, nel=(2, 2, 16)):
    """A context and oracle with nel[2] equal order-4 elements in z over
    20 km; with 16 the column grid is the canonical one and feature
    resampling is the identity."""
    from paper_2504_08157_amd import nhsem
    w = W.cfg_hevi()
    mesh = W.MeshSpec(nel, 4, W.uniform_edges(0, 40e3, nel[0]), W.uniform_edges(0, 40e3, nel[1]),
                      W.uniform_edges(0, 20e3, nel[2]), (True, True))
    ctx = nhsem.Context(mesh, w.phys)
    orc = oracle_mod.Oracle(mesh, w.phys)
    g = ctx.nh_lattice_coords(); o = orc.lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    orc.set_reference(*W.constant_n_reference(o[2]))
    ctx.nh_hevi_attach()
    return ctx, orc, o, w.phys


def _exact_map_params(m, orc, o, ph, alpha, oracle_mod):
    """Network parameters whose hidden path is zero and whose bypass is the
    dimensionless (I - alpha L_v)^-1 of the oracle on features 0 .. 194: the
    exact correction map in FP16."""
    Lm = oracle_mod.column_matrix(orc)
    nz = orc.nz
    rho0, th0 = W.constant_n_reference(o[2])
    D = MO.dimension_factors(rho0, orc.reference_pressure(), th0, ph.cp / ph.cv).reshape(-1)
    M = (np.linalg.inv(np.eye(3 * nz) - alpha * Lm) * D[None, :]) / D[:, None]
    parts = [np.zeros(s) for s in MO.SHAPES]
    parts[6][:3 * nz, :3 * nz] = M
    return MO.flatten(parts).astype(np.float32)


@pytest.mark.parametrize("nelz", [16, 17], ids=["residual_in_kernel", "residual_walk_kernel"])
def test_refinement_pass_matches_oracle(oracle_mod, nelz):
    """Second pass of nh_mlp_guess (the network on the residual of its first
    guess) against the oracle: the residual from the oracle's L_v, features,
    the GPU forward on them, the oracle's resampling; random parameters,
    the pass-2 correction to FP16 rounding of the features.  n_z = 65: the
    residual computed inside the inference kernel; n_z = 69: by the
    residual form of the L_v walk, then the inference kernel."""
    import torch
    from paper_2504_08157_amd import nhsem
    ctx, orc, o, ph = _canonical_column_case(oracle_mod, nel=(3, 2, nelz))
    m = nhsem.ColumnMLP(max_batch=128)
    rng = np.random.default_rng(21)
    m.nh_mlp_set_params(torch.from_numpy(rng.normal(scale=0.03, size=m.nparam).astype(np.float32)).cuda())
    bq = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=6, walls=(False, False))
    bd = torch.from_numpy(bq).cuda()
    alpha = 0.6
    ncol = ctx.nx * ctx.ny
    sel = lambda a: np.stack([a[0], a[3], a[4]]).reshape(3, orc.nz, -1)
    x1 = m.nh_mlp_guess(ctx, alpha, bd).cpu().numpy().reshape(3, orc.nz, ncol)
    m.nh_mlp_set_passes(2)
    x2 = m.nh_mlp_guess(ctx, alpha, bd).cpu().numpy().reshape(3, orc.nz, ncol)
    # the oracle's residual of x1 and the features of the second pass
    full = np.zeros_like(bq)
    full[0], full[3], full[4] = (x1[f].reshape(bq[0].shape) for f in range(3))
    r1 = sel(bq) - x1 + alpha * sel(orc.lv_apply(full))
    rho0, th0 = W.constant_n_reference(o[2])
    D = MO.dimension_factors(rho0, orc.reference_pressure(), th0, ph.cp / ph.cv)
    fo, so = MO.column_features(x1, r1 / alpha, o[2], alpha, D)
    fpad = torch.zeros((128, MO.IN), dtype=torch.float16, device="cuda")
    fpad[:ncol] = torch.from_numpy(fo.astype(np.float16)).cuda()
    y = m.nh_mlp_forward(fpad).cpu().numpy()[:ncol].astype(np.float64)
    ref = MO.column_guess(x1, y, o[2], D, so)
    assert np.linalg.norm(ref - x1) > 1e-3 * np.linalg.norm(x1 - sel(bq))   # pass 2 changes the guess
    assert _rel(x2 - x1, ref - x1) <= 5e-3, _rel(x2 - x1, ref - x1)
    with pytest.raises(RuntimeError):
        m.nh_mlp_set_passes(0)
    with pytest.raises(RuntimeError):
        m.nh_mlp_set_passes(5)


def test_refinement_pass_with_the_exact_map(oracle_mod):
    """With the exact correction map as the network (bypass = the
    dimensionless (I - alpha L_v)^-1 in FP16), one pass leaves the FP16
    rounding of the map, a residual about 1e-3 of the default start's, and
    each refinement pass multiplies it by about that factor again."""
    import torch
    from paper_2504_08157_amd import nhsem
    ctx, orc, o, ph = _canonical_column_case(oracle_mod)
    alpha = 0.6
    m = nhsem.ColumnMLP(max_batch=64)
    m.nh_mlp_set_params(torch.from_numpy(_exact_map_params(m, orc, o, ph, alpha, oracle_mod)).cuda())
    bq = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=8, walls=(False, False))
    bd = torch.from_numpy(bq).cuda()
    ncol = ctx.nx * ctx.ny
    sel = lambda a: np.stack([a[0], a[3], a[4]]).reshape(3, orc.nz, -1)

    def resid(x):
        full = np.zeros_like(bq)
        full[0], full[3], full[4] = (x[f].reshape(bq[0].shape) for f in range(3))
        return np.linalg.norm(sel(bq) - x + alpha * sel(orc.lv_apply(full)))

    r = [resid(sel(bq))]
    for passes in (1, 2, 3):
        m.nh_mlp_set_passes(passes)
        r.append(resid(m.nh_mlp_guess(ctx, alpha, bd).cpu().numpy().reshape(3, orc.nz, ncol)))
    print("residuals", r)
    assert r[1] < 1e-2 * r[0] and r[2] < 1e-2 * r[1] and r[3] < r[2], r
