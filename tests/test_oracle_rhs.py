"""Pins of the oracle's right-hand side, DSS and SSP-RK3 (Eq. governing,
Eq. governing:matrix, Algorithms 1-3) against exact results: rest states,
polynomial exactness, closed forms, conservation, symmetry, convergence."""
import mpmath
import numpy as np
import pytest

from paper_2504_08157_amd import workloads as W


def _setup(oracle_mod, mesh, phys, reference="isentropic"):
    o = oracle_mod.Oracle(mesh, phys)
    x, y, z = o.lattice_coords()
    if reference == "isentropic":
        rho0, th0 = W.isentropic_reference(z, phys=phys)
    elif reference == "constant":
        rho0 = np.full(z.size, 1.1); th0 = np.full(z.size, 300.0)
    else:
        rho0, th0 = W.constant_n_reference(z, phys=phys)
    o.set_reference(rho0, th0)
    return o, x, y, z, rho0, th0


def _cube(nel=(4, 4, 4), N=4, periodic=(False, False), stretch=False, L=1000.0):
    if stretch:
        e = [W.stretched_edges(0.0, L, n, seed=s) for n, s in zip(nel, (11, 12, 13))]
    else:
        e = [W.uniform_edges(0.0, L, n) for n in nel]
    return W.MeshSpec(tuple(nel), N, e[0], e[1], e[2], periodic)


@pytest.mark.parametrize("periodic", [(False, False), (True, True)])
@pytest.mark.parametrize("ref", ["isentropic", "constant_n"])
def test_rest_state_is_exactly_steady(oracle_mod, periodic, ref):
    ph = W.Physics(f=5e-5, sponge_z0=600.0, sponge_tau=0.02)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, _cube(periodic=periodic, stretch=True), ph, ref)
    R = o.rhs(0.0, np.zeros((5,) + o.shape))
    assert np.all(R == 0.0)
    # EOS of the reference equals the closed-form hydrostatic pressure p_a pi0^(cp/R)
    p0 = o.reference_pressure()
    pi0 = W.exner_isentropic(z) if ref == "isentropic" else W.exner_constant_n(z)
    np.testing.assert_allclose(p0, ph.p_a * pi0 ** (ph.cp / ph.R), rtol=1e-13)


def _poly(coef, X, Y, Z, L=1000.0):
    """Tensor polynomial sum c_abc (X/L)^a (Y/L)^b (Z/L)^c and its gradient."""
    xs, ys, zs = X / L, Y / L, Z / L
    f = np.zeros_like(X); fx = np.zeros_like(X); fy = np.zeros_like(X); fz = np.zeros_like(X)
    for (a, b, c), v in coef.items():
        f += v * xs ** a * ys ** b * zs ** c
        if a: fx += v * a * xs ** (a - 1) * ys ** b * zs ** c / L
        if b: fy += v * b * xs ** a * ys ** (b - 1) * zs ** c / L
        if c: fz += v * c * xs ** a * ys ** b * zs ** (c - 1) / L
    return f, fx, fy, fz


def _walls(R, periodic):
    R = R.copy()
    if not periodic[0]:
        R[1][:, :, 0] = 0; R[1][:, :, -1] = 0
    if not periodic[1]:
        R[2][:, 0, :] = 0; R[2][:, -1, :] = 0
    R[3][0] = 0; R[3][-1] = 0
    return R


@pytest.mark.parametrize("N", [3, 4])
def test_polynomial_exactness_advection(oracle_mod, N):
    """g = 0, constant reference, rho' = theta' = 0 (so p' = 0 exactly) and
    velocities of degree <= N: the DSS'd derivatives are exact at the nodes,
    on a stretched mesh, so R equals the analytic tendency."""
    ph = W.Physics(g=0.0)
    mesh = _cube(nel=(3, 2, 3), N=N, stretch=True)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph, "constant")
    X, Y, Z = W.grid3(x, y, z)
    rng = np.random.default_rng(N)

    def rnd():
        return {(a, b, c): rng.normal() for a in range(N + 1) for b in range(N + 1) for c in range(N + 1)
                if a + b + c <= N + 1}
    u = _poly(rnd(), X, Y, Z); v = _poly(rnd(), X, Y, Z); w = _poly(rnd(), X, Y, Z)
    q = np.zeros((5,) + o.shape); q[1], q[2], q[3] = u[0], v[0], w[0]
    R = o.rhs(0.0, q)
    ex = np.zeros_like(R)
    ex[0] = -1.1 * (u[1] + v[2] + w[3])
    for f, F in ((1, u), (2, v), (3, w)):
        ex[f] = -(u[0] * F[1] + v[0] * F[2] + w[0] * F[3])
    ex = _walls(ex, mesh.periodic)
    for f in range(4):
        scale = np.abs(ex[f]).max()
        assert np.abs(R[f] - ex[f]).max() < 1e-12 * scale, f
    # theta tendency: -u . grad(theta0) = 0 up to rounding of D applied to a constant
    assert np.abs(R[4]).max() < 1e-11


@pytest.mark.parametrize("N", [3, 4])
def test_polynomial_exactness_pressure_and_eos(oracle_mod, N):
    """u = 0 and rho' constructed in 40-digit arithmetic so that
    p' = EOS(rho0+rho', theta0+theta') - EOS(rho0, theta0) is a polynomial P
    of degree <= N: then R_u,v,w = -(1/rho) grad P exactly.  Pins the
    equation of state, the pressure-gradient term and the metric terms."""
    ph = W.Physics(g=0.0)
    mesh = _cube(nel=(2, 3, 2), N=N, stretch=True)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph, "constant")
    X, Y, Z = W.grid3(x, y, z)
    rng = np.random.default_rng(10 + N)
    P = _poly({(a, b, c): 40.0 * rng.normal() for a in range(N + 1) for b in range(N + 1)
               for c in range(N + 1) if a + b + c <= N}, X, Y, Z)
    thp = 0.3 * np.sin(X / 300.0) * np.cos(Y / 400.0)
    mpmath.mp.dps = 40
    gam = mpmath.mpf(ph.cp) / mpmath.mpf(ph.cv)
    R_ = mpmath.mpf(ph.R); pa = mpmath.mpf(ph.p_a)
    r0 = mpmath.mpf(1.1); t0 = mpmath.mpf(300.0)
    p0 = pa * (r0 * R_ * t0 / pa) ** gam
    rhop = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        th = t0 + mpmath.mpf(thp[idx])
        p = p0 + mpmath.mpf(P[0][idx])
        rho = pa / (R_ * th) * (p / pa) ** (1 / gam)
        rhop[idx] = float(rho - r0)
    q = np.zeros((5,) + o.shape); q[0] = rhop; q[4] = thp
    R = o.rhs(0.0, q)
    rho = 1.1 + rhop
    ex = np.zeros_like(R)
    ex[1] = -P[1] / rho; ex[2] = -P[2] / rho; ex[3] = -P[3] / rho
    ex = _walls(ex, mesh.periodic)
    for f in (1, 2, 3):
        scale = np.abs(ex[f]).max()
        assert np.abs(R[f] - ex[f]).max() < 1e-11 * scale, f
    assert np.abs(R[0]).max() == 0.0


def test_pointwise_sources_and_forcing_interpolation(oracle_mod):
    """Coriolis, sponge and the time-interpolated forcing act pointwise:
    for a horizontally uniform state with w = 0 the tendency is exactly the
    pointwise source (checked against the sponge profile reading
    tau = tau_max sin^2(pi/2 (z - z_s)/(H - z_s)))."""
    ph = W.Physics(f=1e-3, sponge_z0=400.0, sponge_tau=0.05)
    mesh = _cube(nel=(2, 2, 3), N=3, periodic=(True, True))
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph, "isentropic")
    X, Y, Z = W.grid3(x, y, z)
    q = np.zeros((5,) + o.shape)
    q[1] = 3.0 + 0 * X; q[2] = -2.0 + 0 * X
    tau = np.where(z >= 400.0, 0.05 * np.sin(0.5 * np.pi * (z - 400.0) / 600.0) ** 2, 0.0)[:, None, None]
    rng = np.random.default_rng(0)
    F0 = rng.normal(size=o.shape); F1 = rng.normal(size=o.shape)
    o.set_forcing(4, [0.0, 10.0], np.stack([F0, F1]))
    for t, lam in ((2.5, 0.25), (-1.0, 0.0), (20.0, 1.0), (10.0, 1.0)):
        R = o.rhs(t, q)
        np.testing.assert_allclose(R[1], 1e-3 * q[2] - tau * q[1], atol=1e-13)
        np.testing.assert_allclose(R[2], -1e-3 * q[1] - tau * q[2], atol=1e-13)
        np.testing.assert_allclose(R[4], (1 - lam) * F0 + lam * F1, atol=1e-13)
        assert np.abs(R[0]).max() < 1e-13 and np.abs(R[3]).max() < 1e-13


def test_rk3_amplification_factor_coriolis(oracle_mod):
    """Spatially uniform (u, v) on an f-plane rotate: d(u+iv)/dt = -i f (u+iv).
    SSP-RK3 must reproduce the stability polynomial 1+z+z^2/2+z^3/6 exactly."""
    f = 2e-3
    # g = 0 with a constant reference and a 1000 km box keeps rounding noise
    # far inside the acoustic stability limit at this time step
    ph = W.Physics(f=f, g=0.0)
    mesh = _cube(nel=(2, 2, 2), N=3, periodic=(True, True), L=1.0e6)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph, "constant")
    q = np.zeros((5,) + o.shape); q[1] = 4.0; q[2] = 1.5
    dt, n = 20.0, 7
    out = o.rk3(0.0, dt, n, q)
    zz = -1j * f * dt
    amp = (1 + zz + zz ** 2 / 2 + zz ** 3 / 6) ** n
    ex = amp * (4.0 + 1.5j)
    np.testing.assert_allclose(out[1], ex.real, atol=1e-12)
    np.testing.assert_allclose(out[2], ex.imag, atol=1e-12)


def test_rk3_sponge_decay(oracle_mod):
    ph = W.Physics(sponge_z0=3.0e5, sponge_tau=0.1, g=0.0)
    mesh = _cube(nel=(1, 1, 4), N=4, periodic=(True, True), L=1.0e6)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph, "constant")
    q = np.zeros((5,) + o.shape)
    q[1] = (1.0 + z / 1.0e6)[:, None, None] + 0 * q[1]
    dt, n = 0.5, 5
    out = o.rk3(0.0, dt, n, q)
    tau = np.where(z >= 3.0e5, 0.1 * np.sin(0.5 * np.pi * (z - 3.0e5) / 7.0e5) ** 2, 0.0)
    zz = -tau * dt
    ex = (1 + zz + zz ** 2 / 2 + zz ** 3 / 6) ** n * (1.0 + z / 1.0e6)
    np.testing.assert_allclose(out[1][:, 0, 0], ex, rtol=1e-14)


def test_dss_conservation(oracle_mod):
    mesh = _cube(nel=(3, 2, 2), N=3, periodic=(True, False), stretch=True)
    o, *_ = _setup(oracle_mod, mesh, W.Physics())
    rng = np.random.default_rng(1)
    E = rng.normal(size=(2, o.L))
    out = o.dss(E, mode=0)
    np.testing.assert_allclose(out.sum(axis=1), E.sum(axis=1), rtol=1e-13)
    # mass-weighted average: sum M out = sum wJ in
    xi, w, _ = oracle_mod.lgl(3)
    n1 = 4
    wJ = np.zeros(o.L)
    e = 0
    for ez in range(2):
        for ey in range(2):
            for ex in range(3):
                J = ((mesh.xe[ex + 1] - mesh.xe[ex]) * (mesh.ye[ey + 1] - mesh.ye[ey])
                     * (mesh.ze[ez + 1] - mesh.ze[ez]) / 8)
                wJ[e * 64:(e + 1) * 64] = (w[None, None, :] * w[None, :, None] * w[:, None, None] * J).ravel()
                e += 1
    avg = o.dss(E, mode=1)
    M = o.mass().ravel()
    np.testing.assert_allclose((avg * M).sum(axis=1), (E * wJ).sum(axis=1), rtol=1e-13)
    # scatter then average of a continuous field returns it
    Uv = rng.normal(size=(1, o.U))
    np.testing.assert_allclose(o.dss(o.scatter(Uv), mode=1), Uv, rtol=1e-13)
    cnt = o.dss(np.ones((1, o.L)), mode=0)
    assert set(np.unique(cnt)) <= {1.0, 2.0, 4.0, 8.0}


def test_mass_conservation_bubble(oracle_mod):
    w = W.cfg_bubble()
    o, x, y, z, rho0, th0 = _setup(oracle_mod, w.mesh, w.phys)
    q = W.initial_state(w, x, y, z)
    M = o.mass()
    m0 = (M * q[0]).sum()
    out = o.rk3(0.0, w.dt, w.steps, q)
    total = (M * (rho0[:, None, None] + q[0])).sum()
    assert abs((M * out[0]).sum() - m0) < 1e-13 * total
    # the bubble rises: positive w above the centre
    assert out[3][np.argmin(np.abs(z - 500.0)), 8, 8] > 0


def test_mass_conservation_periodic_with_heating(oracle_mod):
    w = W.cfg_tc_small()
    w.mesh = W._tc_mesh(4, 4, 3)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, w.mesh, w.phys, "constant_n")
    q = W.initial_state(w, x, y, z)
    t, Q = W.heating(w, x, y, z)
    o.set_forcing(4, t, Q)
    M = o.mass()
    m0 = (M * q[0]).sum()
    out = o.rk3(0.0, 0.5, 4, q)
    total = (M * (rho0[:, None, None] + q[0])).sum()
    assert abs((M * out[0]).sum() - m0) < 1e-13 * total


def test_bubble_mirror_symmetry(oracle_mod):
    w = W.cfg_bubble()
    o, x, y, z, rho0, th0 = _setup(oracle_mod, w.mesh, w.phys)
    q = W.initial_state(w, x, y, z)
    out = o.rk3(0.0, w.dt, w.steps, q)
    # velocity components share one scale (|u|, |v| << |w| for the young bubble)
    scale = np.abs(out).reshape(5, -1).max(axis=1)
    scale[1:4] = scale[1:4].max()
    flipx = out[:, :, :, ::-1]
    sign = np.array([1, -1, 1, 1, 1])[:, None, None, None]
    assert (np.abs(flipx * sign - out).reshape(5, -1).max(axis=1) <= 1e-12 * scale + 1e-300).all()
    flipy = out[:, :, ::-1, :]
    sign = np.array([1, 1, -1, 1, 1])[:, None, None, None]
    assert (np.abs(flipy * sign - out).reshape(5, -1).max(axis=1) <= 1e-12 * scale + 1e-300).all()
    sw = out.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
    assert (np.abs(sw - out).reshape(5, -1).max(axis=1) <= 1e-12 * scale + 1e-300).all()


def test_rhs_sample_equals_full_rhs(oracle_mod):
    """The sampled evaluation used at full size is the full right-hand side
    restricted to the sample, bit for bit, with repeated and boundary nodes."""
    ph = W.Physics(f=1e-4, sponge_z0=500.0, sponge_tau=0.02)
    mesh = _cube(nel=(3, 4, 3), N=3, periodic=(True, False), stretch=True)
    o, x, y, z, rho0, th0 = _setup(oracle_mod, mesh, ph)
    q = W.smooth_random_state(x, y, z, rho0, th0, seed=12, walls=(False, True))
    rng = np.random.default_rng(3)
    F = rng.normal(size=(2,) + o.shape)
    o.set_forcing(4, [0.0, 5.0], F)
    R = o.rhs(1.5, q).reshape(5, -1)
    nodes = np.concatenate([rng.integers(0, o.U, 300), [0, o.U - 1, 7, 7, 7]])
    np.testing.assert_array_equal(o.rhs_sample(1.5, q, nodes), R[:, nodes])
    with pytest.raises(ValueError):
        o.rhs_sample(1.5, q, [o.U])
