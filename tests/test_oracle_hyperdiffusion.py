"""Pins of the hyper-diffusion oracle (section on tensor-based
hyper-diffusion: H_q = -(div tau grad)^2 q, tau from the eigendecomposition
of the metric tensor, nu_i scaled by element size and time step) against
closed forms, invariants and a Fourier mode."""
import numpy as np
import pytest

from oracle import hyperdiffusion as HD
from paper_2504_08157_amd import workloads as W


def _geo(oracle_mod, nel, per, xe=None, ye=None, ze=None, N=4):
    xe = W.uniform_edges(0, 80e3, nel[0]) if xe is None else xe
    ye = W.uniform_edges(0, 60e3, nel[1]) if ye is None else ye
    ze = W.uniform_edges(0, 8e3, nel[2]) if ze is None else ze
    mesh = W.MeshSpec(nel, N, xe, ye, ze, per)
    orc = oracle_mod.Oracle(mesh, W.Physics())
    return HD.ElementGeometry(orc), orc


def test_tau_box_closed_form():
    """Box element of edges (10, 8, 1) km: the principal axes are x, y, z in
    that order of decreasing extent, so tau = diag(nu_1, nu_2, nu_3) with
    nu_i = sqrt(c_i) h_i^2 / sqrt(dt)."""
    h = np.array([10e3, 8e3, 1e3])
    c = np.array([0.01, 0.02, 0.05])
    dt = 3.0
    tau = HD.viscosity_tensor(np.diag(h / 2), c, dt)
    nu = np.sqrt(c) * h ** 2 / np.sqrt(dt)
    np.testing.assert_allclose(tau, np.diag(nu), rtol=1e-14, atol=1e-9 * nu.max())
    # a tall element: z is now the largest extent and takes nu_1
    h2 = np.array([1e3, 2e3, 5e3])
    tau2 = HD.viscosity_tensor(np.diag(h2 / 2), c, dt)
    nu2 = np.sqrt(c[[2, 1, 0]]) * h2 ** 2 / np.sqrt(dt)
    np.testing.assert_allclose(np.diag(tau2), nu2, rtol=1e-14)


def test_tau_rotated_element():
    """A box rotated about z: G has distinct eigenvalues, eigh finds the
    rotated axes, and tau = R diag(nu) R^T."""
    th = 0.3
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    h = np.array([10e3, 6e3, 1e3])
    J = R @ np.diag(h / 2)
    c = np.array([0.01, 0.02, 0.05])
    tau = HD.viscosity_tensor(J, c, 2.0)
    nu = np.sqrt(c) * h ** 2 / np.sqrt(2.0)
    np.testing.assert_allclose(tau, R @ np.diag(nu) @ R.T, rtol=1e-12, atol=1e-9 * nu.max())


def test_laplacian_invariants(oracle_mod):
    """Constants are in the kernel; the operator is symmetric and negative
    semi-definite in the mass inner product and conserves the mass-weighted
    sum (walls and periodic directions, stretched z)."""
    geo, orc = _geo(oracle_mod, (3, 2, 3), (True, False), ze=W.stretched_edges(0, 8e3, 3, seed=2))
    c, dt = (0.02, 0.03, 0.05), 2.0
    M = orc.mass().reshape(-1)
    one = HD.weak_laplacian(geo, np.ones((1, orc.U)), c, dt)
    rng = np.random.default_rng(4)
    u, v = rng.normal(size=(2, 1, orc.U))
    Lu, Lv = HD.weak_laplacian(geo, u, c, dt), HD.weak_laplacian(geo, v, c, dt)
    scale = np.abs(Lu).max()
    assert np.abs(one).max() <= 1e-12 * scale
    assert abs((M * u * Lv).sum() - (M * Lu * v).sum()) <= 1e-12 * np.abs(M * u * Lv).sum()
    assert (M * u * Lu).sum() < 0
    assert abs((M * Lu).sum()) <= 1e-13 * np.abs(M * Lu).sum()
    H = HD.hyperdiffusion(geo, u, c, dt)
    assert (M * u * H).sum() < 0                      # dissipative
    assert abs((M * H).sum()) <= 1e-12 * np.abs(M * H).sum()


def _mode(oracle_mod, nel, xe, ye, axis, c, dt):
    mesh = W.MeshSpec(nel, 4, xe, ye, W.uniform_edges(0, 1e3, 1), (True, True))
    orc = oracle_mod.Oracle(mesh, W.Physics())
    geo = HD.ElementGeometry(orc)
    x, y, z = orc.lattice_coords()
    X = np.broadcast_to(x[None, None, :] if axis == 0 else y[None, :, None], orc.shape)
    k = 2 * np.pi / 80e3
    q = np.sin(k * X).reshape(1, -1)
    return geo, q, k


@pytest.mark.parametrize("axis", [0, 1])
def test_fourier_mode_tie(oracle_mod, axis):
    """A resolved periodic mode q = sin(2 pi s / L) (s = x or y) on 10 km
    square elements: x and y tie as principal axes and take nu_1, nu_2 in
    that order, so (div tau grad) q = -nu_(axis+1) k^2 q to the accuracy of
    order-4 elements at 8 per period, and H_q = -nu^2 k^4 q to 3 % (the
    second application amplifies the first one's error, which sits at high
    wavenumbers near element faces, by about (k_max / k)^2)."""
    c, dt = (0.02, 0.03, 0.05), 2.0
    geo, q, k = _mode(oracle_mod, (8, 8, 1), W.uniform_edges(0, 80e3, 8), W.uniform_edges(0, 80e3, 8), axis, c, dt)
    tau = np.sqrt(c[axis]) * 10e3 ** 2 / np.sqrt(dt)
    L = HD.weak_laplacian(geo, q, c, dt)
    assert np.linalg.norm(L + tau * k ** 2 * q) <= 1e-4 * np.linalg.norm(tau * k ** 2 * q)
    H = HD.hyperdiffusion(geo, q, c, dt)
    assert np.linalg.norm(H + tau ** 2 * k ** 4 * q) <= 3e-2 * np.linalg.norm(tau ** 2 * k ** 4 * q)


def test_fourier_mode_convergence(oracle_mod):
    """Elements of 40 km in y and 80/n km in x: y is the largest extent and
    takes nu_1, x takes nu_2; the error of (div tau grad) sin(2 pi x / L)
    against -nu_2 k^2 sin falls by more than 12 from n = 8 to n = 16
    (measured 15.6: fourth order, set by the lumped LGL mass)."""
    c, dt = (0.02, 0.03, 0.05), 2.0
    err = []
    for n in (8, 16):
        geo, q, k = _mode(oracle_mod, (n, 2, 1), W.uniform_edges(0, 80e3, n), W.uniform_edges(0, 80e3, 2), 0, c, dt)
        tau = np.sqrt(c[1]) * (80e3 / n) ** 2 / np.sqrt(dt)
        L = HD.weak_laplacian(geo, q, c, dt)
        err.append(np.linalg.norm(L + tau * k ** 2 * q) / np.linalg.norm(tau * k ** 2 * q))
    assert err[0] <= 1e-4 and err[1] <= err[0] / 12, err


def _walled_state(orc, seed):
    x, y, z = orc.lattice_coords()
    q = W.smooth_random_state(x, y, z, *W.constant_n_reference(z), seed=seed, walls=(True, True))
    # wall-normal velocities exactly zero (sin(pi) is not)
    q[1][:, :, [0, -1]] = 0.0
    q[2][:, [0, -1], :] = 0.0
    q[3][[0, -1]] = 0.0
    return q.reshape(5, -1)


def test_wall_mask_matches_rhs_walls(oracle_mod):
    """The mask zeroes exactly the rows the C oracle's right-hand side zeroes
    after its DSS (an independent implementation of the no-flux walls):
    masking its output changes nothing, and the mask of a tendency of ones
    removes 2 n_y n_z u rows, 2 n_x n_z v rows and 2 n_x n_y w rows."""
    geo, orc = _geo(oracle_mod, (3, 2, 2), (False, False), N=3)
    orc.set_reference(*W.constant_n_reference(orc.lattice_coords()[2]))
    q = _walled_state(orc, 11)
    R = orc.rhs(0.0, q).reshape(5, -1)
    assert np.array_equal(HD.wall_mask(orc, R), R)
    ones = HD.wall_mask(orc, np.ones((5, orc.U)))
    nz, ny, nx = orc.shape
    assert (ones == 0).sum(axis=1).tolist() == [0, 2 * ny * nz, 2 * nx * nz, 2 * nx * ny, 0]
    # periodic x and y: only w keeps its rows at bottom and top
    _, orp = _geo(oracle_mod, (3, 2, 2), (True, True), N=3)
    onesp = HD.wall_mask(orp, np.ones((5, orp.U)))
    assert (onesp == 0).sum(axis=1).tolist() == [0, 0, 0, 2 * orp.nx * orp.ny, 0]


def test_masked_tendency_keeps_walls_and_mass(oracle_mod):
    """Three SSP-RK3 steps of dq/dt = S + H_q with the wall rows of H_q
    zeroed keep u, v on the side walls and w at the bottom and top exactly
    zero and the mass-weighted sum of rho' constant to 1e-13 of its size.
    Adding H_q unmasked instead puts velocity on the walls, and the mass then
    drifts by far more (the divergence's sum is the boundary flux)."""
    geo, orc = _geo(oracle_mod, (3, 2, 2), (False, False), N=3)
    orc.set_physics(W.Physics(f=5e-5))
    orc.set_reference(*W.constant_n_reference(orc.lattice_coords()[2]))
    c, hdt, dt = (1e-6, 2e-6, 5e-6), 1.0, 0.5
    M = orc.mass().reshape(-1)
    q0 = _walled_state(orc, 12)

    def run(masked):
        def F(t, y):
            H = HD.hyperdiffusion(geo, y, c, hdt)
            H = HD.wall_mask(orc, H) if masked else H
            return orc.rhs(t, y).reshape(5, -1) + H
        y = q0.copy()
        for s in range(3):
            t = s * dt
            y1 = y + dt * F(t, y)
            y2 = 0.75 * y + 0.25 * (y1 + dt * F(t + dt, y1))
            y = y / 3.0 + 2.0 / 3.0 * (y2 + dt * F(t + 0.5 * dt, y2))
        return y.reshape((5,) + orc.shape)

    m0 = (M * q0[0]).sum()
    scale = (M * np.abs(q0[0])).sum()
    y = run(True)
    assert np.all(y[1][:, :, [0, -1]] == 0.0) and np.all(y[2][:, [0, -1], :] == 0.0)
    assert np.all(y[3][[0, -1]] == 0.0)
    assert abs((M * y[0].reshape(-1)).sum() - m0) <= 1e-13 * scale
    yu = run(False)
    assert np.abs(yu[1][:, :, [0, -1]]).max() > 1e-6
    assert abs((M * yu[0].reshape(-1)).sum() - m0) > 1e-9 * scale
