"""GPU RI-velocity diagnostic against the oracle (section on the RI velocity):
centroids, strip counts (bit-exact) and means, u_RI and its location, the
maximum horizontal speed; edge cases and argument errors."""
import numpy as np
import pytest

from oracle import ri_velocity as RI
from paper_2504_08157_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _vortex_state(orc, xc, yc, vm=20.0, rm=8e3, seed=0):
    """Axisymmetric vortex about (xc, yc), tilted with height, plus seeded
    smooth noise in u, v, w."""
    x, y, z = orc.lattice_coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    H = max(float(z[-1]), 1.0)
    cx = xc + 2e3 * Z / H
    cy = yc - 1e3 * Z / H
    dx, dy = X - cx, Y - cy
    r = np.sqrt(dx * dx + dy * dy)
    V = vm * (r / rm) * np.exp((1 - (r / rm) ** 2) / 2) * (1.0 - 0.5 * Z / H)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(r > 0, V / r, 0.0)
    rng = np.random.default_rng(seed)
    a = rng.normal(size=6)
    L = float(x[-1] - x[0]) + 1.0
    q = np.zeros((5,) + orc.shape)
    q[1] = -s * dy + 0.3 * np.sin(2 * np.pi * (X / L + a[0])) * np.cos(2 * np.pi * (Y / L + a[1]))
    q[2] = s * dx + 0.3 * np.cos(2 * np.pi * (X / L + a[2])) * np.sin(2 * np.pi * (Y / L + a[3]))
    q[3] = 0.5 * np.sin(np.pi * Z / H) * np.cos(2 * np.pi * (X / L + a[4]))
    q[0] = 1e-3 * a[5]
    q[4] = 0.2
    return q


MESHES = {
    "periodic_N4": ((6, 5, 3), 4, (60e3, 50e3, 6e3), (True, True), False),
    "walls_stretched_N3": ((5, 6, 4), 3, (50e3, 60e3, 8e3), (False, False), True),
    "mixed_N5_ragged": ((7, 3, 2), 5, (70e3, 30e3, 4e3), (True, False), False),
}


def _mesh(oracle_mod, nel, N, ext, per, stretched):
    from paper_2504_08157_amd import nhsem
    ze = W.stretched_edges(0, ext[2], nel[2], seed=4) if stretched else W.uniform_edges(0, ext[2], nel[2])
    mesh = W.MeshSpec(nel, N, W.uniform_edges(0, ext[0], nel[0]), W.uniform_edges(0, ext[1], nel[1]), ze, per)
    return nhsem.Context(mesh, W.Physics()), oracle_mod.Oracle(mesh, W.Physics())


def _compare(got, want, loc_check=True):
    import torch  # noqa: F401
    assert got["count"].cpu().numpy().tolist() == want["count"].tolist()
    ub = got["ubar"].cpu().numpy()
    scale = max(np.abs(want["ubar"]).max(), 1e-300)
    assert np.abs(ub - want["ubar"]).max() <= TOL * scale
    res = got["result"].cpu().numpy()
    assert abs(res[0] - want["u_ri"]) <= TOL * max(abs(want["u_ri"]), 1e-300)
    assert abs(res[3] - want["umax"]) <= TOL * max(want["umax"], 1e-300)
    if loc_check:
        # the location is unique unless another populated strip comes within rounding of the maximum
        flat = np.where(want["count"] > 0, want["ubar"], -np.inf).ravel()
        second = np.sort(flat)[-2] if flat.size > 1 else -np.inf
        if want["u_ri"] - second > 1e-9 * max(want["u_ri"], 1e-300):
            assert res[1] == want["r_ri"] and res[2] == want["z_ri"]


@pytest.mark.parametrize("case", list(MESHES))
def test_ri_parity(oracle_mod, case):
    import torch
    nel, N, ext, per, st = MESHES[case]
    ctx, orc = _mesh(oracle_mod, nel, N, ext, per, st)
    q = _vortex_state(orc, 0.45 * ext[0], 0.55 * ext[1], seed=list(MESHES).index(case))
    qd = torch.from_numpy(q).cuda()
    rmax = 0.5 * min(ext[0], ext[1])
    want = RI.ri_velocity(orc, q, nstrips=50, rmax=rmax)
    got = ctx.nh_ri_velocity(qd, nstrips=50, rmax=rmax)
    cen = got["center"].cpu().numpy()
    assert np.abs(cen[0] - want["xc"]).max() <= TOL * ext[0]
    assert np.abs(cen[1] - want["yc"]).max() <= TOL * ext[1]
    _compare(got, want)
    # the oracle's centre given as input: strips decided from the same centre
    c = torch.from_numpy(np.stack([want["xc"], want["yc"]])).cuda()
    got2 = ctx.nh_ri_velocity(qd, nstrips=37, rmax=0.8 * rmax, center=c)
    want2 = RI.ri_velocity(orc, q, nstrips=37, rmax=0.8 * rmax, center=(want["xc"], want["yc"]))
    _compare(got2, want2)
    assert torch.equal(got2["center"], c)


def test_ri_integer_lattice_edges(oracle_mod):
    """Order-2 elements of width 2 put the nodes on integers; centre on a
    node, eps = 1: squared radii equal to squared strip edges (perfect
    squares) and the centre are in no strip, identically on both sides."""
    import torch
    from paper_2504_08157_amd import nhsem
    n = 8
    mesh = W.MeshSpec((n, n, 1), 2, W.uniform_edges(0, 2 * n, n), W.uniform_edges(0, 2 * n, n),
                      W.uniform_edges(0, 2, 1), (False, False))
    ctx, orc = nhsem.Context(mesh, W.Physics()), oracle_mod.Oracle(mesh, W.Physics())
    x, y, z = orc.lattice_coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    q = np.zeros((5,) + orc.shape)
    q[1], q[2], q[3] = -2.5 * (Y - 6.0) + 0.1 * X, 2.5 * (X - 7.0), 0.3
    assert np.array_equal(x, np.arange(2 * n + 1.0))
    c = (np.full(orc.nz, 7.0), np.full(orc.nz, 6.0))
    for ns, rmax in ((6, 6.0), (1, 3.0), (9, 4.5)):
        want = RI.ri_velocity(orc, q, nstrips=ns, rmax=rmax, center=c)
        got = ctx.nh_ri_velocity(torch.from_numpy(q).cuda(), nstrips=ns, rmax=rmax,
                                 center=torch.from_numpy(np.stack(c)).cuda())
        _compare(got, want)


def test_ri_empty_rest_and_no_strip(oracle_mod):
    """r_max beyond the domain (empty outer strips), a state at rest (centre
    = domain midpoint, u_RI = 0), strips too narrow to hold a node."""
    import torch
    ctx, orc = _mesh(oracle_mod, (3, 3, 1), 4, (30e3, 30e3, 1e3), (True, True), False)
    q = _vortex_state(orc, 15e3, 15e3, rm=4e3, seed=2)
    qd = torch.from_numpy(q).cuda()
    _compare(ctx.nh_ri_velocity(qd, nstrips=20, rmax=60e3), RI.ri_velocity(orc, q, nstrips=20, rmax=60e3))
    rest = ctx.nh_ri_velocity(0 * qd, nstrips=20)
    wrest = RI.ri_velocity(orc, 0 * q, nstrips=20)
    assert np.array_equal(rest["center"].cpu().numpy(), np.stack([wrest["xc"], wrest["yc"]]))
    _compare(rest, wrest)
    c = np.full((2, orc.nz), 15e3)
    none = ctx.nh_ri_velocity(qd, nstrips=4, rmax=1e3, center=torch.from_numpy(c).cuda())
    assert (none["count"].cpu().numpy() == 0).all()
    assert none["result"].cpu().numpy()[:3].tolist() == [0.0, -1.0, -1.0]


def test_ri_argument_errors(oracle_mod):
    import torch
    from paper_2504_08157_amd import nhsem
    ctx, orc = _mesh(oracle_mod, (2, 2, 1), 2, (10e3, 10e3, 1e3), (True, True), False)
    q = torch.zeros((5,) + tuple(orc.shape), dtype=torch.float64, device="cuda")
    for ns, rmax in ((0, 1e3), (4097, 1e3), (10, 0.0), (10, float("nan"))):
        with pytest.raises(nhsem.NHError) as e:
            ctx.nh_ri_velocity(q, nstrips=ns, rmax=rmax)
        assert e.value.code == nhsem.NH_EINVAL


def test_ri_full_size_tc_share(oracle_mod):
    """The 128 x 128 x 20 element (N = 4) per-GPU share with its balanced
    vortex, in the launch configuration the benchmark times: every level
    and strip against the oracle."""
    import torch
    w = W.cfg_tc_large()
    from paper_2504_08157_amd import nhsem
    ctx = nhsem.Context(w.mesh, w.phys)
    orc = oracle_mod.Oracle(w.mesh, w.phys)
    x, y, z = orc.lattice_coords()
    q = W.initial_state(w, x, y, z)
    want = RI.ri_velocity(orc, q, nstrips=50)
    got = ctx.nh_ri_velocity(torch.from_numpy(q).cuda(), nstrips=50)
    ext = float(w.mesh.xe[-1] - w.mesh.xe[0])
    cen = got["center"].cpu().numpy()
    assert np.abs(cen[0] - want["xc"]).max() <= TOL * ext and np.abs(cen[1] - want["yc"]).max() <= TOL * ext
    _compare(got, want)
    assert want["u_ri"] > 5.0
