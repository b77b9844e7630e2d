"""Pins of the oracle's HEVI pieces (Sec. 2.3): the vertical linear operator
L_v, the ARK2 tableau and step, and the direct column solve."""
import numpy as np
import pytest

from paper_2504_08157_amd import workloads as W


def _tc(oracle_mod, nel=(2, 2, 4), N=4):
    ph = W.Physics(g=W.G)
    mesh = W.MeshSpec(nel, N, W.uniform_edges(0, 40e3, nel[0]), W.uniform_edges(0, 40e3, nel[1]),
                      W.stretched_edges(0, 12e3, nel[2], seed=4), (True, True))
    o = oracle_mod.Oracle(mesh, ph)
    x, y, z = o.lattice_coords()
    rho0, th0 = W.constant_n_reference(z)
    o.set_reference(rho0, th0)
    return o, x, y, z


def test_lv_is_linearisation_of_s(oracle_mod):
    """For horizontally uniform perturbations with u = v = 0 (f = 0, no
    sponge) the full nonlinear S linearised about rest equals L_v: pinned by
    a central difference of the oracle's S (a different code path: the
    nonlinear EOS, the momentum flux and the total-theta gradient)."""
    o, x, y, z = _tc(oracle_mod)
    rng = np.random.default_rng(0)
    col = np.zeros((5, o.nz))
    col[0] = 1e-3 * rng.normal(size=o.nz)
    col[3] = rng.normal(size=o.nz); col[3][0] = col[3][-1] = 0
    col[4] = 0.5 * rng.normal(size=o.nz)
    xv = np.broadcast_to(col[:, :, None, None], (5,) + o.shape).copy()
    Lx = o.lv_apply(xv)
    eps = 1e-5
    fd = (o.rhs(0.0, eps * xv) - o.rhs(0.0, -eps * xv)) / (2 * eps)
    for f in (0, 3, 4):
        scale = np.abs(Lx[f]).max()
        assert np.abs(fd[f] - Lx[f]).max() < 1e-7 * scale, f
    assert np.abs(Lx[1]).max() == 0 and np.abs(Lx[2]).max() == 0
    # every column carries the same operator
    assert np.abs(Lx - Lx[:, :, :1, :1]).max() < 1e-12 * np.abs(Lx).max()


def test_ark2_tableau_order_conditions(oracle_mod):
    A, At, b, c = oracle_mod.hevi_coefficients()
    one = np.ones(3)
    for T in (A, At):
        np.testing.assert_allclose(T @ one, c, atol=1e-15)     # row sums = abscissae
        assert abs(b @ one - 1) < 1e-15                        # order 1
        assert abs(b @ (T @ one) - 0.5) < 1e-15                # order 2
    assert np.all(np.triu(A) == 0)                             # explicit
    assert np.all(np.triu(At, 1) == 0) and At[0, 0] == 0       # singly diagonally implicit


def test_ark2_second_order_on_split_ode(oracle_mod):
    """y' = lam_e y + lam_i y, explicit/implicit split: global error O(dt^2)
    against the exact exponential."""
    lam_e, lam_i = -0.7 + 1.3j, -2.0
    S = lambda t, y: (lam_e + lam_i) * y
    L = lambda y: lam_i * y
    solve = lambda a, r: r / (1 - a * lam_i)
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = np.array([1.0 + 0j])
        for k in range(n):
            y = oracle_mod.ark2_generic(S, L, solve, k * dt, dt, y)
        errs.append(abs(y[0] - np.exp(lam_e + lam_i)))
    p = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (p > 1.9).all() and (p < 2.2).all(), p
    # L = 0 reduces to the explicit tableau: stability polynomial
    A, At, b, c = oracle_mod.hevi_coefficients()
    zz = 0.3 + 0.2j
    y = oracle_mod.ark2_generic(lambda t, y: zz * y, lambda y: 0 * y, lambda a, r: r, 0.0, 1.0,
                                np.array([1.0 + 0j]))
    one = np.ones(3)
    R = 1 + zz * (b @ one) + zz ** 2 * (b @ A @ one) + zz ** 3 * (b @ A @ A @ one)
    assert abs(y[0] - R) < 1e-15


def test_column_solve_and_hevi_step(oracle_mod):
    o, x, y, z = _tc(oracle_mod, nel=(2, 2, 3), N=3)
    Lm = oracle_mod.column_matrix(o)
    n = 3 * o.nz
    assert Lm.shape == (n, n)
    # L_v rows of w at z = 0, H vanish
    assert np.all(Lm[o.nz] == 0) and np.all(Lm[2 * o.nz - 1] == 0)
    # columns of the assembled matrix reproduce lv_apply on a random column state
    rng = np.random.default_rng(3)
    xv = rng.normal(size=(5,) + o.shape)
    xv[1:3] = 0
    Lx = o.lv_apply(xv)
    X = np.concatenate([xv[0].reshape(o.nz, -1), xv[3].reshape(o.nz, -1), xv[4].reshape(o.nz, -1)])
    Y = Lm @ X
    np.testing.assert_allclose(Y[:o.nz], Lx[0].reshape(o.nz, -1), atol=1e-12 * np.abs(Lx[0]).max())
    np.testing.assert_allclose(Y[o.nz:2 * o.nz], Lx[3].reshape(o.nz, -1), atol=1e-12 * np.abs(Lx[3]).max())
    # a HEVI step from rest stays at rest; mass is conserved for a perturbed state
    q0 = np.zeros((5,) + o.shape)
    assert np.all(oracle_mod.ark2_step(o, Lm, 0.0, 5.0, q0) == 0)
    w = W.cfg_hevi(); w.mesh = o.mesh
    q = W.smooth_random_state(x, y, z, *W.constant_n_reference(z), seed=2, walls=(False, False), amp=0.3)
    M = o.mass()
    q1 = oracle_mod.ark2_step(o, Lm, 0.0, 2.0, q)
    rho0 = W.constant_n_reference(z)[0][:, None, None]
    assert abs((M * q1[0]).sum() - (M * q[0]).sum()) < 1e-13 * (M * rho0).sum()
