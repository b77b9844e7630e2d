"""GPU tensor hyper-diffusion against the oracle (section on tensor-based
hyper-diffusion): H_q on several meshes, SSP-RK3 steps with H_q added to
the tendency, the unsupported case and switching it off."""
import numpy as np
import pytest

from oracle import hyperdiffusion as HD
from paper_2504_08157_amd import workloads as W

pytestmark = pytest.mark.gpu

C = (0.02, 0.03, 0.05)
DT = 1.0

CASES = {
    "walls_stretched_N4": ((4, 3, 3), 4, (False, False), True),
    "periodic_N4": ((3, 4, 2), 4, (True, True), False),
    "mixed_N3": ((5, 2, 3), 3, (True, False), True),
    "periodic_x1_N5": ((1, 3, 2), 5, (True, True), True),
    # 68 x 21 lattice columns: two 64 x 16 tiles each way, ragged in both
    "multi_tile_N4": ((17, 5, 2), 4, (True, False), True),
    "walls_N2": ((9, 7, 3), 2, (False, False), False),
    "periodic_y_N6": ((3, 2, 2), 6, (False, True), True),
    # 71 x 20 columns, walls in x: two tiles each way for the one-walk form
    "multi_tile_walls_N2": ((35, 10, 3), 2, (False, True), True),
    # 70 x 19 columns, walls everywhere, ragged tiles
    "multi_tile_walls_N3": ((23, 6, 2), 3, (False, False), True),
}


def _pair(oracle_mod, nel, N, per, stretched, H=6e3):
    from paper_2504_08157_amd import nhsem
    ze = W.stretched_edges(0, H, nel[2], seed=5) if stretched else W.uniform_edges(0, H, nel[2])
    mesh = W.MeshSpec(nel, N, W.uniform_edges(0, 40e3, nel[0]), W.uniform_edges(0, 36e3, nel[1]), ze, per)
    ph = W.Physics(f=5e-5)
    ctx = nhsem.Context(mesh, ph)
    orc = oracle_mod.Oracle(mesh, ph)
    g = ctx.nh_lattice_coords(); o = orc.lattice_coords()
    ctx.nh_set_reference(*W.constant_n_reference(g[2]))
    orc.set_reference(*W.constant_n_reference(o[2]))
    return ctx, orc, g, o


@pytest.mark.parametrize("case", list(CASES))
def test_hyperdiffusion_parity(oracle_mod, case):
    import torch
    nel, N, per, stretched = CASES[case]
    ctx, orc, g, o = _pair(oracle_mod, nel, N, per, stretched)
    ctx.nh_set_hyperdiffusion(C, DT)
    q = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=3, walls=(not per[0], not per[1]))
    Hg = ctx.nh_hyperdiffusion(torch.from_numpy(q).cuda()).cpu().numpy().reshape(5, -1)
    Ho = HD.hyperdiffusion_tendency(HD.ElementGeometry(orc), q.reshape(5, -1), C, DT)
    for f in range(5):
        err = np.linalg.norm(Hg[f] - Ho[f]) / np.linalg.norm(Ho[f])
        assert err <= 1e-12, (case, f, err)
    # the wall-normal rows are zero exactly, as the mask leaves them
    assert np.array_equal(Hg[Ho == 0.0], Ho[Ho == 0.0]), case


# order 4 takes the running-sum form of the accumulating launch, order 6 the
# register-window form
RK_CASES = {"N4": ((4, 3, 3), 4), "N6": ((3, 2, 2), 6)}


@pytest.mark.parametrize("case", list(RK_CASES))
def test_rk3_with_hyperdiffusion(oracle_mod, case):
    """Two SSP-RK3 steps with H_q in the tendency against the oracle's
    right-hand side plus its H_q, stepped in the Shu-Osher form.  The
    coefficients are small enough for the explicit step (nu scales with the
    element extent, so the largest eigenvalue of H_q is ~ c (pi N)^4 / dt)."""
    import torch
    nel, N = RK_CASES[case]
    ctx, orc, g, o = _pair(oracle_mod, nel, N, (True, False), True)
    c_step = (1e-6, 2e-6, 5e-6)
    ctx.nh_set_hyperdiffusion(c_step, DT)
    q = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=6, walls=(False, True))
    ctx.nh_set_state(torch.from_numpy(q).cuda())
    dt = 0.5
    ctx.nh_rk_step(0.0, dt, 2)
    got = ctx.nh_get_state().cpu().numpy().reshape(5, -1)
    geo = HD.ElementGeometry(orc)

    def F(t, y):
        return orc.rhs(t, y.reshape((5,) + orc.shape)).reshape(5, -1) + HD.hyperdiffusion_tendency(geo, y, c_step, DT)

    y = q.reshape(5, -1)
    for s in range(2):
        t = s * dt
        y1 = y + dt * F(t, y)
        y2 = 0.75 * y + 0.25 * (y1 + dt * F(t + dt, y1))
        y = y / 3.0 + 2.0 / 3.0 * (y2 + dt * F(t + 0.5 * dt, y2))
    plain0 = orc.rk3(0.0, dt, 2, q).reshape(5, -1)
    for f in range(5):
        err = np.linalg.norm(got[f] - y[f]) / np.linalg.norm(y[f])
        assert err <= 1e-12, (f, err)
    # the term changes the result by far more than the tolerance
    assert np.linalg.norm(y - plain0) > 1e-8 * np.linalg.norm(y)
    # switched off: the plain step again
    ctx.nh_set_hyperdiffusion(None, 0.0)
    ctx.nh_set_state(torch.from_numpy(q).cuda())
    ctx.nh_rk_step(0.0, dt, 1)
    plain = orc.rk3(0.0, dt, 1, q).reshape(5, -1)
    got = ctx.nh_get_state().cpu().numpy().reshape(5, -1)
    for f in range(5):
        assert np.linalg.norm(got[f] - plain[f]) <= 1e-12 * np.linalg.norm(plain[f])


def test_walls_and_mass_with_hyperdiffusion(oracle_mod):
    """SSP-RK3 steps with H_q on a mesh walled in x and y: the wall-normal
    velocities (u on the x walls, v on the y walls, w at the bottom and top)
    stay exactly zero and the mass-weighted sum of rho' is conserved to 1e-13
    of its size, as without the term; the state matches the oracle's steps
    with the masked tendency."""
    import torch
    ctx, orc, g, o = _pair(oracle_mod, (4, 3, 3), 4, (False, False), True)
    c_step = (1e-6, 2e-6, 5e-6)
    ctx.nh_set_hyperdiffusion(c_step, DT)
    q = W.smooth_random_state(*o, *W.constant_n_reference(o[2]), seed=7, walls=(True, True))
    q[1][:, :, [0, -1]] = 0.0
    q[2][:, [0, -1], :] = 0.0
    q[3][[0, -1]] = 0.0
    ctx.nh_set_state(torch.from_numpy(q).cuda())
    M = orc.mass().reshape(-1)
    m0, scale = (M * q[0].reshape(-1)).sum(), (M * np.abs(q[0]).reshape(-1)).sum()
    dt = 0.5
    ctx.nh_rk_step(0.0, dt, 4)
    got = ctx.nh_get_state().cpu().numpy().reshape((5,) + orc.shape)
    assert np.all(got[1][:, :, [0, -1]] == 0.0) and np.all(got[2][:, [0, -1], :] == 0.0)
    assert np.all(got[3][[0, -1]] == 0.0)
    assert abs((M * got[0].reshape(-1)).sum() - m0) <= 1e-13 * scale
    geo = HD.ElementGeometry(orc)

    def F(t, y):
        return orc.rhs(t, y.reshape((5,) + orc.shape)).reshape(5, -1) + HD.hyperdiffusion_tendency(geo, y, c_step, DT)

    y = q.reshape(5, -1)
    for s in range(4):
        t = s * dt
        y1 = y + dt * F(t, y)
        y2 = 0.75 * y + 0.25 * (y1 + dt * F(t + dt, y1))
        y = y / 3.0 + 2.0 / 3.0 * (y2 + dt * F(t + 0.5 * dt, y2))
    got = got.reshape(5, -1)
    for f in range(5):
        assert np.linalg.norm(got[f] - y[f]) <= 1e-12 * np.linalg.norm(y[f]), f


def test_unsupported_when_extent_order_changes(oracle_mod):
    """A z layer taller than the horizontal elements swaps the principal
    axes in that layer: tau is not separable per direction."""
    from paper_2504_08157_amd import nhsem
    ze = np.array([0.0, 1e3, 2e3, 15e3])        # last layer 13 km > 10 km horizontal
    mesh = W.MeshSpec((2, 2, 3), 4, W.uniform_edges(0, 20e3, 2), W.uniform_edges(0, 20e3, 2), ze, (True, True))
    ctx = nhsem.Context(mesh, W.Physics())
    with pytest.raises(nhsem.NHError) as e:
        ctx.nh_set_hyperdiffusion(C, DT)
    assert e.value.code == nhsem.NH_EUNSUPPORTED


def test_full_size_tc_share_properties():
    """The 128 x 128 x 20 element (N = 4) share in the launch configuration
    the benchmark times, through properties that hold at any size: H_q of
    constant fields vanishes, the mass-weighted sum of H_q is conserved, H_q
    is dissipative, and a horizontal Fourier mode is an eigenfunction with
    eigenvalue -(tau k^2)^2 to the discretisation's accuracy (square
    elements: x takes c_1)."""
    import torch
    from paper_2504_08157_amd import nhsem
    w = W.cfg_tc_large()
    ctx = nhsem.Context(w.mesh, w.phys)
    x, y, z = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.reference_profiles(w, z))
    c = (1e-6, 2e-6, 5e-6)
    ctx.nh_set_hyperdiffusion(c, w.dt)
    M = ctx.nh_mass().reshape(-1)
    shape = (5,) + ctx.shape
    # constants
    one = torch.ones(shape, dtype=torch.float64, device="cuda")
    H1 = ctx.nh_hyperdiffusion(one)
    q0 = torch.from_numpy(W.initial_state(w, x, y, z)).cuda()
    Hq = ctx.nh_hyperdiffusion(q0)
    scale = Hq.abs().max().item()
    assert H1.abs().max().item() <= 1e-12 * scale
    # conservation and dissipation per field (fields with variation)
    Hf, qf = Hq.reshape(5, -1), q0.reshape(5, -1)
    for f in range(5):
        s = (M * Hf[f]).sum().item()
        a = (M * Hf[f].abs()).sum().item()
        if a == 0:
            continue
        assert abs(s) <= 1e-10 * a, f
        assert (M * qf[f] * Hf[f]).sum().item() < 0, f
    # Fourier mode along x
    Lx = float(w.mesh.xe[-1] - w.mesh.xe[0])
    k = 2 * np.pi / Lx
    hx = Lx / w.mesh.nel[0]
    tau = np.sqrt(c[0]) * hx ** 2 / np.sqrt(w.dt)
    X = torch.from_numpy(np.broadcast_to(x[None, None, :], ctx.shape).copy()).cuda()
    m = torch.zeros(shape, dtype=torch.float64, device="cuda")
    m[4] = torch.sin(k * X)
    Hm = ctx.nh_hyperdiffusion(m)[4]
    want = -(tau * k * k) ** 2 * m[4]
    err = (Hm - want).norm().item() / want.norm().item()
    # fourth order in k h (lumped LGL mass), k h = 2 pi / 128: measured 5.7e-5
    assert err <= 1e-4, err
