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
