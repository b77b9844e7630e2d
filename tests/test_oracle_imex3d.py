"""Pins of the oracle's 3D-IMEX pieces (Sec. 2.3 with the linear operator
taken over all three directions): the 3D linear operator against a central
difference of the nonlinear right-hand side, its implicit absorbing-layer
term, its reduction to the vertical operator, and the ARK2 step built on it
(second order in time, stable for acoustic Courant numbers far above the
explicit limit)."""
import numpy as np

from paper_2504_08157_amd import workloads as W


def _box(oracle_mod, nel=(3, 3, 3), N=3, per=(True, False), ph=None):
    ph = ph or W.Physics()
    mesh = W.MeshSpec(nel, N, W.uniform_edges(0, 30e3, nel[0]), W.uniform_edges(0, 24e3, nel[1]),
                      W.stretched_edges(0, 9e3, nel[2], seed=4), per)
    o = oracle_mod.Oracle(mesh, ph)
    x, y, z = o.lattice_coords()
    o.set_reference(*W.constant_n_reference(z))
    return o, x, y, z


def _perturbation(o, x, y, z, seed, walls):
    ref = W.constant_n_reference(z)
    q = W.smooth_random_state(x, y, z, *ref, seed=seed, walls=walls)
    return q


def test_l3_is_linearisation_of_s(oracle_mod):
    """f = 0 and no sponge: S linearised about rest (central difference of
    the nonlinear RHS: nonlinear EOS, momentum and mass fluxes, total-theta
    gradient) equals L on every field, for a 3D perturbation with all five
    fields nonzero."""
    o, x, y, z = _box(oracle_mod)
    xv = _perturbation(o, x, y, z, seed=1, walls=(False, True))
    Lx = o.l3_apply(xv)
    eps = 1e-6
    fd = (o.rhs(0.0, eps * xv) - o.rhs(0.0, -eps * xv)) / (2 * eps)
    for f in range(5):
        scale = np.abs(Lx[f]).max()
        assert scale > 0
        assert np.abs(fd[f] - Lx[f]).max() < 1e-7 * scale, f


def test_l3_absorbing_layer_and_vertical_part(oracle_mod):
    """With the sponge on, L gains -tau(z) w on the w row only (interior
    levels); for horizontally uniform fields with u = v = 0 it reduces to the
    vertical operator of the 1D split plus that term."""
    ph = W.Physics(sponge_z0=5e3, sponge_tau=0.05)
    o, x, y, z = _box(oracle_mod, ph=ph)
    o0, *_ = _box(oracle_mod)
    xv = _perturbation(o, x, y, z, seed=2, walls=(False, True))
    d = o.l3_apply(xv) - o0.l3_apply(xv)
    tau = np.where(z >= 5e3, 0.05 * np.sin(0.5 * np.pi * (z - 5e3) / (9e3 - 5e3)) ** 2, 0.0)
    want = -tau[:, None, None] * xv[3]
    want[0] = want[-1] = 0.0
    assert np.abs(d[[0, 1, 2, 4]]).max() == 0.0
    assert np.abs(d[3] - want).max() <= 1e-13 * np.abs(want).max()
    col = np.zeros((5, o.nz))
    rng = np.random.default_rng(3)
    col[0] = 1e-3 * rng.normal(size=o.nz)
    col[3] = rng.normal(size=o.nz)
    col[4] = 0.5 * rng.normal(size=o.nz)
    xu = np.broadcast_to(col[:, :, None, None], (5,) + o.shape).copy()
    L3, Lv = o.l3_apply(xu), o.lv_apply(xu)
    extra = -tau[:, None, None] * xu[3]
    extra[0] = extra[-1] = 0.0
    Lv[3] += extra
    assert np.abs(L3 - Lv).max() <= 1e-12 * np.abs(Lv).max()


def test_imex3d_second_order_and_acoustic_stability(oracle_mod):
    """The 3D-IMEX ARK2 step with direct stage solves: errors against a
    fine explicit reference fall as dt^2; at an acoustic Courant number of
    about 10 (far beyond the explicit limit) the step stays bounded."""
    o, x, y, z = _box(oracle_mod, nel=(2, 2, 2), N=3, per=(True, True))
    q0 = 0.2 * _perturbation(o, x, y, z, seed=5, walls=(False, False))
    Lm = oracle_mod.l3_matrix(o)
    T = 4.0
    ref = o.rk3(0.0, T / 800, 800, q0.copy()).reshape(q0.shape)
    errs = []
    for n in (4, 8, 16):
        dt = T / n
        q = q0.copy()
        for k in range(n):
            q = oracle_mod.imex3d_step(o, Lm, k * dt, dt, q)
        errs.append(max(np.abs(q[f] - ref[f]).max() / np.abs(ref[f]).max() for f in range(5)))
    p = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (p > 1.7).all(), (errs, p)
    # acoustic Courant number c dt / dx_min ~ 10 with the smallest LGL spacing
    dxmin = np.diff(x).min()
    dt = 10 * dxmin / 350.0
    q = q0.copy()
    for k in range(20):
        q = oracle_mod.imex3d_step(o, Lm, k * dt, dt, q)
    assert np.isfinite(q).all() and np.abs(q).max() < 10 * np.abs(q0).max()
