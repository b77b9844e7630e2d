"""Parity of the gfx950 library (through the C ABI) with the FP64 oracle.

Both sides build their own node coordinates, evaluate the shared workload
generators there, and are compared field by field with the relative L2 norm
||gpu - oracle|| / ||oracle|| (FP64 path: <= 1e-12).
"""
import numpy as np
import pytest

from paper_2504_08157_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _rel(a, b):
    a = np.asarray(a).reshape(5, -1)
    b = np.asarray(b).reshape(5, -1)
    return np.array([np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), 1e-300) for f in range(5)])


def _pair(oracle_mod, mesh, phys, reference="isentropic", precision=0):
    import torch
    from paper_2504_08157_amd import nhsem
    ctx = nhsem.Context(mesh, phys, precision=precision)
    orc = oracle_mod.Oracle(mesh, phys)
    gx, gy, gz = ctx.nh_lattice_coords()
    ox, oy, oz = orc.lattice_coords()
    np.testing.assert_allclose(gx, ox, rtol=0, atol=1e-9 * (abs(ox).max() + 1))
    np.testing.assert_allclose(gz, oz, rtol=0, atol=1e-9 * (abs(oz).max() + 1))
    prof = W.isentropic_reference if reference == "isentropic" else W.constant_n_reference
    ctx.nh_set_reference(*prof(gz, phys=phys))
    orc.set_reference(*prof(oz, phys=phys))
    return ctx, orc, (gx, gy, gz), (ox, oy, oz), prof, torch


def _mesh(nel, N, periodic, L=(1000.0, 1000.0, 1000.0), stretch=False):
    if stretch:
        e = [W.stretched_edges(0.0, l, n, seed=s) for n, l, s in zip(nel, L, (21, 22, 23))]
    else:
        e = [W.uniform_edges(0.0, l, n) for n, l in zip(nel, L)]
    return W.MeshSpec(tuple(nel), N, e[0], e[1], e[2], periodic)


RHS_CASES = [
    ("walls_N4", (4, 4, 4), 4, (False, False), False),
    ("walls_stretched_N3", (5, 3, 4), 3, (False, False), True),
    ("periodic_ragged_N4", (5, 7, 3), 4, (True, True), False),
    ("mixed_stretched_N5", (3, 4, 2), 5, (True, False), True),
    ("periodic_N2", (9, 8, 3), 2, (True, True), True),
    ("walls_N6", (2, 3, 2), 6, (False, False), False),
    ("one_element_periodic_N4", (1, 2, 1), 4, (True, True), False),
]


@pytest.mark.parametrize("name,nel,N,per,stretch", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_rhs_parity(oracle_mod, name, nel, N, per, stretch):
    ph = W.Physics(f=1e-3, sponge_z0=600.0, sponge_tau=0.05)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh(nel, N, per, stretch=stretch), ph)
    walls = (not per[0], not per[1])
    qg = W.smooth_random_state(*g, *prof(g[2]), seed=7, walls=walls)
    qo = W.smooth_random_state(*o, *prof(o[2]), seed=7, walls=walls)
    dq = ctx.nh_rhs(0.0, torch.from_numpy(qg).cuda()).cpu().numpy()
    ref = orc.rhs(0.0, qo)
    err = _rel(dq, ref)
    print(name, err)
    assert (err <= TOL64).all(), err


# the node-class form of the stage kernel (tile variant 2, order 4): every
# order-4 case above plus a mesh of several tiles with ragged edges in x and
# y and an odd number of element layers (the bottom/top plane slots swap
# roles every layer)
CLS_CASES = [c for c in RHS_CASES if c[2] == 4] + [
    ("multi_tile_ragged_N4", (11, 5, 3), 4, (True, False), True),
    ("walls_tall_N4", (3, 2, 7), 4, (False, False), True),
]


@pytest.mark.parametrize("name,nel,N,per,stretch", CLS_CASES, ids=[c[0] for c in CLS_CASES])
def test_rhs_parity_class_kernel(oracle_mod, name, nel, N, per, stretch):
    ph = W.Physics(f=1e-3, sponge_z0=600.0, sponge_tau=0.05)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh(nel, N, per, stretch=stretch), ph)
    ctx.nh_set_tile(2)
    walls = (not per[0], not per[1])
    qg = W.smooth_random_state(*g, *prof(g[2]), seed=7, walls=walls)
    qo = W.smooth_random_state(*o, *prof(o[2]), seed=7, walls=walls)
    dq = ctx.nh_rhs(0.0, torch.from_numpy(qg).cuda()).cpu().numpy()
    ref = orc.rhs(0.0, qo)
    err = _rel(dq, ref)
    print(name, err)
    assert (err <= TOL64).all(), err


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_mixed"])
def test_rk3_class_kernel_tc_with_heating(oracle_mod, precision):
    """Ten SSP-RK3 steps of the heated vortex through the node-class stage
    kernel, FP64 to 1e-12 and FP32-mixed to the FP32 tolerances."""
    w = W.cfg_tc_small()
    w.mesh = W._tc_mesh(9, 5, 3)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys, reference="constant_n", precision=precision)
    ctx.nh_set_tile(2)
    tg, Qg = W.heating(w, *g)
    to, Qo = W.heating(w, *o)
    Qdev = torch.from_numpy(Qg.reshape(len(tg), -1)).cuda()
    ctx.nh_set_forcing(4, tg - 1500.0, Qdev)
    orc.set_forcing(4, to - 1500.0, Qo)
    ctx.nh_set_state(torch.from_numpy(W.initial_state(w, *g)).cuda())
    ctx.nh_rk_step(0.0, 2.0, 10)
    got = ctx.nh_get_state().cpu().numpy()
    ref = orc.rk3(0.0, 2.0, 10, W.initial_state(w, *o))
    err = _rel(got, ref)
    print("class kernel", precision, err)
    assert (err <= (TOL64 if precision == 0 else TOL32_RK)).all(), err


def test_rest_state_exactly_zero(oracle_mod):
    ph = W.Physics(f=5e-5, sponge_z0=500.0, sponge_tau=0.02)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((5, 4, 3), 4, (True, False), stretch=True), ph,
                                        reference="constant_n")
    q = torch.zeros((5,) + ctx.shape, dtype=torch.float64, device="cuda")
    dq = ctx.nh_rhs(0.0, q)
    assert torch.count_nonzero(dq).item() == 0


def test_rk3_parity_bubble(oracle_mod):
    w = W.cfg_bubble()
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys)
    ctx.nh_set_state(torch.from_numpy(W.initial_state(w, *g)).cuda())
    ctx.nh_rk_step(0.0, w.dt, w.steps)
    got = ctx.nh_get_state().cpu().numpy()
    ref = orc.rk3(0.0, w.dt, w.steps, W.initial_state(w, *o))
    err = _rel(got, ref)
    # u, v of the young bubble are tiny: compare velocities against the velocity norm
    vel = np.linalg.norm(ref[1:4])
    err_v = np.array([np.linalg.norm(got[f] - ref[f]) / vel for f in (1, 2, 3)])
    print(err, err_v)
    assert err[0] <= TOL64 and err[4] <= TOL64 and (err_v <= TOL64).all()


def test_rk3_parity_tc_with_heating(oracle_mod):
    w = W.cfg_tc_small()
    w.mesh = W._tc_mesh(6, 5, 4)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys, reference="constant_n")
    tg, Qg = W.heating(w, *g)
    to, Qo = W.heating(w, *o)
    # shift the window so the bursts are active during the test steps
    Qdev = torch.from_numpy(Qg.reshape(len(tg), -1)).cuda()
    ctx.nh_set_forcing(4, tg - 1500.0, Qdev)
    orc.set_forcing(4, to - 1500.0, Qo)
    ctx.nh_set_state(torch.from_numpy(W.initial_state(w, *g)).cuda())
    ctx.nh_rk_step(0.0, 2.0, 10)
    got = ctx.nh_get_state().cpu().numpy()
    ref = orc.rk3(0.0, 2.0, 10, W.initial_state(w, *o))
    err = _rel(got, ref)
    print(err)
    assert (err <= TOL64).all(), err


def test_forcing_on_every_field(oracle_mod):
    ph = W.Physics()
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((3, 3, 2), 4, (True, True)), ph)
    rng = np.random.default_rng(5)
    F = rng.normal(size=(5, 2) + ctx.shape)
    keep = []
    for f in range(5):
        d = torch.from_numpy(F[f].reshape(2, -1).copy()).cuda()
        keep.append(d)
        ctx.nh_set_forcing(f, [0.0, 4.0], d)
        orc.set_forcing(f, [0.0, 4.0], F[f])
    qg = W.smooth_random_state(*g, *prof(g[2]), seed=3, walls=(False, False))
    qo = W.smooth_random_state(*o, *prof(o[2]), seed=3, walls=(False, False))
    for t in (-1.0, 1.0, 9.0):
        dq = ctx.nh_rhs(t, torch.from_numpy(qg).cuda()).cpu().numpy()
        err = _rel(dq, orc.rhs(t, qo))
        assert (err <= TOL64).all(), (t, err)


def test_dss_scatter_mass_parity(oracle_mod):
    ph = W.Physics()
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((3, 4, 2), 3, (True, False), stretch=True), ph)
    rng = np.random.default_rng(11)
    E = rng.normal(size=(3, ctx.L))
    Ed = torch.from_numpy(E).cuda()
    s = ctx.nh_dss(Ed, 0).cpu().numpy()
    np.testing.assert_array_equal(s, orc.dss(E, 0))  # same summation order
    a = ctx.nh_dss(Ed, 1).cpu().numpy()
    np.testing.assert_allclose(a, orc.dss(E, 1), rtol=1e-14, atol=0)
    Uv = rng.normal(size=(2, ctx.U))
    sc = ctx.nh_scatter(torch.from_numpy(Uv).cuda()).cpu().numpy()
    np.testing.assert_array_equal(sc, orc.scatter(Uv))
    M = ctx.nh_mass().cpu().numpy()
    np.testing.assert_allclose(M, orc.mass(), rtol=1e-14)


def test_mass_conservation_and_diagnostics(oracle_mod):
    w = W.cfg_tc_small()
    w.mesh = W._tc_mesh(5, 5, 4)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys, reference="constant_n")
    q = W.initial_state(w, *g)
    ctx.nh_set_state(torch.from_numpy(q).cuda())
    d0 = ctx.nh_diagnostics()
    ctx.nh_rk_step(0.0, 1.0, 20)
    d1 = ctx.nh_diagnostics()
    M = ctx.nh_mass().cpu().numpy()
    total = (M * prof(g[2])[0][:, None, None]).sum()
    assert abs(d1[0] - d0[0]) < 1e-13 * total
    assert d1[7] == 0 and ctx.nh_check_finite() == 0
    np.testing.assert_allclose(d0[1], np.abs(q[1]).max(), rtol=1e-15)
    np.testing.assert_allclose(d0[0], (M * q[0]).sum(), rtol=1e-12)


def test_nonfinite_detected(oracle_mod):
    ph = W.Physics()
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((2, 2, 2), 4, (True, True)), ph)
    q = torch.zeros((5,) + ctx.shape, dtype=torch.float64, device="cuda")
    q[3, 1, 2, 3] = float("nan")
    ctx.nh_set_state(q)
    from paper_2504_08157_amd import nhsem
    assert ctx.nh_check_finite() == nhsem.NH_ENONFINITE
    assert "non-finite" in ctx.nh_last_error()


# FP32-mixed path against the FP64 oracle, relative L2 per field (rho', u, v,
# w, theta'): about ten times the measured errors (rhs: 2.3e-7, 1.1e-7,
# 1.2e-7, 1.2e-7, 9.7e-8; ten steps: 3.7e-8, 5.3e-10, 6.9e-10, 4.1e-7,
# 9.3e-10), for one tendency of a smooth random state and for ten SSP-RK3
# steps of the heated vortex
TOL32_RHS = np.array([2e-6, 2e-6, 2e-6, 2e-6, 2e-6])
TOL32_RK = np.array([5e-7, 1e-8, 1e-8, 5e-6, 1e-8])


def test_fp32_mixed_rhs_close(oracle_mod):
    """FP32 contractions with FP64 EOS, DSS and RK: one tendency of a smooth
    state against the FP64 oracle (TOL32_RHS per field)."""
    ph = W.Physics(f=1e-4)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((4, 4, 3), 4, (True, True)), ph, precision=1)
    qg = W.smooth_random_state(*g, *prof(g[2]), seed=9, walls=(False, False))
    qo = W.smooth_random_state(*o, *prof(o[2]), seed=9, walls=(False, False))
    dq = ctx.nh_rhs(0.0, torch.from_numpy(qg).cuda()).cpu().numpy()
    err = _rel(dq, orc.rhs(0.0, qo))
    print("fp32 rhs", err)
    assert (err <= TOL32_RHS).all(), err


def test_fp32_mixed_rk3_steps(oracle_mod):
    """Ten SSP-RK3 steps of the heated vortex (6 x 5 x 4 elements, N = 4)
    in FP32-mixed against the FP64 oracle: every stage's combination
    a q^n + b q^s + c R runs, in FP64, after FP32 contractions
    (TOL32_RK per field; w, small and driven by the heating, has the
    largest relative error)."""
    w = W.cfg_tc_small()
    w.mesh = W._tc_mesh(6, 5, 4)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys, reference="constant_n", precision=1)
    tg, Qg = W.heating(w, *g)
    to, Qo = W.heating(w, *o)
    Qdev = torch.from_numpy(Qg.reshape(len(tg), -1)).cuda()
    ctx.nh_set_forcing(4, tg - 1500.0, Qdev)
    orc.set_forcing(4, to - 1500.0, Qo)
    ctx.nh_set_state(torch.from_numpy(W.initial_state(w, *g)).cuda())
    ctx.nh_rk_step(0.0, 2.0, 10)
    got = ctx.nh_get_state().cpu().numpy()
    ref = orc.rk3(0.0, 2.0, 10, W.initial_state(w, *o))
    err = _rel(got, ref)
    print("fp32 rk3", err)
    assert (err <= TOL32_RK).all(), err


def test_rhs_parity_both_eos_branches(oracle_mod):
    """A state with a 30 K warm core and a 9 % density deficit elsewhere:
    the EOS argument s = (1 + rho'/rho0)(1 + theta'/theta0) - 1 passes 1/16
    in both directions at some nodes (the expm1/log1p branch) and stays
    below it at most others (the series), FP64 <= 1e-12 per field."""
    ph = W.Physics(f=1e-4)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((4, 4, 3), 4, (False, False)), ph)

    def state(c):
        x, y, z = c
        rho0, th0 = prof(z)
        q = W.smooth_random_state(x, y, z, rho0, th0, seed=13, walls=(True, True))
        X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
        X, Y, Z = (a.transpose(2, 1, 0) for a in (X, Y, Z))
        warm = np.exp(-((X - 300.0) ** 2 + (Y - 600.0) ** 2 + (Z - 400.0) ** 2) / 200.0 ** 2)
        light = np.exp(-((X - 700.0) ** 2 + (Y - 300.0) ** 2 + (Z - 600.0) ** 2) / 200.0 ** 2)
        q[4] += 30.0 * warm
        q[0] -= 0.09 * rho0[:, None, None] * light
        return q, rho0, th0

    qo, rho0, th0 = state(o)
    s = (1 + qo[0] / rho0[:, None, None]) * (1 + qo[4] / th0[:, None, None]) - 1
    assert (s >= 1 / 16).sum() > 20 and (s <= -1 / 16).sum() > 20 and (np.abs(s) < 1 / 16).mean() > 0.5
    qg = state(g)[0]
    dq = ctx.nh_rhs(0.0, torch.from_numpy(qg).cuda()).cpu().numpy()
    err = _rel(dq, orc.rhs(0.0, qo))
    print("eos branches", err)
    assert (err <= TOL64).all(), err


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_tile_variants_bitwise_equal(oracle_mod, N):
    from paper_2504_08157_amd import nhsem
    ph = W.Physics(f=1e-4, sponge_z0=500.0, sponge_tau=0.01)
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, _mesh((7, 5, 3), N, (True, False)), ph)
    q = torch.from_numpy(W.smooth_random_state(*g, *prof(g[2]), seed=4, walls=(False, True))).cuda()
    outs = []
    # variant 2 is another tile of the same arithmetic except at order 4
    # (node-class form, equal to rounding: covered by the class-kernel tests)
    for v in ((0, 1, 2) if N != 4 else (0, 1)):
        ctx.nh_set_tile(v)
        outs.append(ctx.nh_rhs(0.0, q).cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_array_equal(outs[0], o)
    with pytest.raises(nhsem.NHError):
        ctx.nh_set_tile(3)


def test_full_size_sampled_rhs_parity(oracle_mod):
    """Tropical-cyclone box at its benchmark size (128 x 128 x 20 elements,
    N = 4, 21.3 M unique nodes) with the heating bursts, both tile variants
    (the benchmark times the faster one): the GPU tendency at 4096 seeded
    sample nodes plus corner and edge classes against the oracle evaluated at
    those nodes only.

    Two states.  A smooth random state: relative L2 <= 1e-12 per field.  The
    balanced vortex: there the tendencies are residues of cancelling terms
    (div(rho u) and u.grad(theta') of a rotational wind, gradient-wind and
    hydrostatic balance), up to ~1e6 times smaller than the terms, so each
    field is measured against the size of its terms: the tendency with only
    the x or only the y wind component, and the buoyancy g rho'/rho."""
    w = W.cfg_tc_large()
    ctx, orc, g, o, prof, torch = _pair(oracle_mod, w.mesh, w.phys, reference="constant_n")
    # one set of inputs (on the oracle's lattice) feeds both sides: at this
    # size generating them twice would dominate the test
    to, Qo = W.heating(w, *o)
    Qdev = torch.from_numpy(Qo.reshape(len(to), -1)).cuda()
    ctx.nh_set_forcing(4, to - 1500.0, Qdev)
    orc.set_forcing(4, to - 1500.0, Qo)
    del Qo
    rng = np.random.default_rng(2024)
    nx, ny, nz = ctx.shape[2], ctx.shape[1], ctx.shape[0]
    ix = np.concatenate([rng.integers(0, nx, 4096), [0, nx - 1, 0, nx - 1, 1, 4, 5]])
    iy = np.concatenate([rng.integers(0, ny, 4096), [0, 0, ny - 1, ny - 1, 4, 1, 8]])
    iz = np.concatenate([rng.integers(0, nz, 4096), [0, nz - 1, 4, 0, nz - 1, 5, 8]])
    nodes = (iz * ny + iy) * nx + ix
    nd = torch.from_numpy(nodes).cuda()
    t = 1600.0

    def gpu(q, v):
        ctx.nh_set_tile(v)
        return ctx.nh_rhs(t, torch.from_numpy(q).cuda()).reshape(5, -1)[:, nd].cpu().numpy()

    qr = W.smooth_random_state(*o, *prof(o[2]), seed=8, walls=(False, False))
    ref = orc.rhs_sample(t, qr, nodes)
    for v in (0, 1, 2):
        err = _rel(gpu(qr, v), ref)
        print("random, tile", v, err)
        assert (err <= TOL64).all(), (v, err)
    del qr

    qv = W.initial_state(w, *o)
    ref = orc.rhs_sample(t, qv, nodes)
    # size of the terms that cancel in the balanced vortex: the tendency with
    # only the x (v = 0) or only the y (u = 0) wind component, and buoyancy
    scale = np.linalg.norm(ref, axis=1)
    for comp in (1, 2):
        qs = qv.copy()
        qs[3 - comp] = 0.0
        scale = np.maximum(scale, np.linalg.norm(orc.rhs_sample(t, qs, nodes), axis=1))
        del qs
    rho0, th0 = prof(o[2])
    rp = qv[0].reshape(-1)[nodes]
    inner = (iz > 0) & (iz < nz - 1)
    scale[3] = max(scale[3], np.linalg.norm(w.phys.g * rp[inner] / (rho0[iz][inner] + rp[inner])))
    # The oracle advects total theta = theta0 + theta' (its literal reading):
    # its horizontal stencil sums terms of size theta0 (2/h) |D| u, so its own
    # rounding is a few eps times that, ~1e-12 of the small u.grad(theta') of
    # the vortex; the theta' error is allowed 1e-15 (~5 eps) of the summands.
    Dm = np.asarray(oracle_mod.lgl(w.mesh.order)[2]).reshape(w.mesh.order + 1, -1)
    hx = (w.mesh.xe[-1] - w.mesh.xe[0]) / w.mesh.nel[0]
    wind = np.abs(qv[1].reshape(-1)[nodes]) + np.abs(qv[2].reshape(-1)[nodes])
    summands = th0[iz] * (2.0 / hx) * np.abs(Dm).sum(axis=1).max() * wind
    scale[4] = max(scale[4], 1e-3 * np.linalg.norm(summands))
    for v in (0, 1, 2):
        err = np.linalg.norm(gpu(qv, v) - ref, axis=1) / scale
        print("vortex, tile", v, err, "scales", scale)
        assert (err <= TOL64).all(), (v, err)
