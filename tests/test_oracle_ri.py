"""Pins of the RI-velocity oracle (section on the RI velocity: u_RI as the
maximum of the azimuthally averaged tangential velocity, the speed-weighted
centroid per level, the strip approximation of the azimuthal mean) against
closed forms, symmetry and brute force on small lattices."""
import math

import numpy as np
import pytest

from oracle import ri_velocity as RI
from paper_2504_08157_amd import workloads as W


def _orc(oracle_mod, nel, N, xe, ye, ze, per):
    return oracle_mod.Oracle(W.MeshSpec(nel, N, xe, ye, ze, per), W.Physics())


def _state(orc, u, v, w):
    q = np.zeros((5,) + orc.shape)
    q[1], q[2], q[3] = u, v, w
    return q


def _grid(orc):
    x, y, z = orc.lattice_coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def test_centroid_linear_speed_closed_form(oracle_mod):
    """Speed a + b x (> 0) on walls [0, L]: the LGL quadrature integrates the
    degree-2 integrand exactly, so x_c = (a L^2/2 + b L^3/3) / (a L + b L^2/2)
    and y_c = the y midpoint, at every level."""
    L, Ly = 9e3, 7e3
    orc = _orc(oracle_mod, (3, 2, 2), 3, W.uniform_edges(0, L, 3), W.uniform_edges(0, Ly, 2),
               W.uniform_edges(0, 2e3, 2), (False, False))
    X, Y, Z = _grid(orc)
    a, b = 2.0, 3e-4
    s = a + b * X
    q = _state(orc, 0.6 * s, -0.8 * s, 0.0 * s)           # |u| = s
    xc, yc = RI.centroid(orc, q)
    want = (a * L ** 2 / 2 + b * L ** 3 / 3) / (a * L + b * L ** 2 / 2)
    np.testing.assert_allclose(xc, want, rtol=1e-13)
    np.testing.assert_allclose(yc, Ly / 2, rtol=1e-13)


def test_centroid_symmetric_vortex_and_rest_level(oracle_mod):
    """A vortex symmetric about the origin of a symmetric lattice (walls: both
    edges are nodes) has its centre at the origin; a level at rest takes the
    domain midpoint."""
    orc = _orc(oracle_mod, (4, 4, 2), 4, W.uniform_edges(-20e3, 20e3, 4), W.uniform_edges(-20e3, 20e3, 4),
               W.uniform_edges(0, 4e3, 2), (False, False))
    X, Y, Z = _grid(orc)
    r2 = X ** 2 + Y ** 2
    V = 10.0 * np.exp(-r2 / 8e3 ** 2)
    u, v = -V * Y / 5e3, V * X / 5e3
    u[-1] = 0.0
    v[-1] = 0.0
    xc, yc = RI.centroid(orc, _state(orc, u, v, 0 * u))
    assert np.abs(xc[:-1]).max() <= 1e-12 * 20e3 and np.abs(yc[:-1]).max() <= 1e-12 * 20e3
    assert xc[-1] == 0.0 and yc[-1] == 0.0


def test_tangential_speed_removes_radial_and_vertical(oracle_mod):
    """Solid rotation Omega (-dy, dx) plus radial alpha (dx, dy) plus any w:
    u_theta = |Omega| r at every point (r from hypot)."""
    rng = np.random.default_rng(1)
    dx, dy = rng.normal(size=(2, 200)) * 5e3
    om, al = -3e-4, 7e-5
    u = -om * dy + al * dx
    v = om * dx + al * dy
    w = rng.normal(size=200)
    ut = RI.tangential_speed(u, v, w, dx, dy)
    r = np.array([math.hypot(a, b) for a, b in zip(dx, dy)])
    np.testing.assert_allclose(ut, abs(om) * r, rtol=1e-12)


def test_strips_brute_force_integer_lattice(oracle_mod):
    """Order-1 elements of unit width put the nodes on integers; with the
    centre on a node and eps = 1 every squared radius and strip edge is an
    exact integer, so membership is j^2 < r^2 < (j+1)^2 in integer arithmetic
    (perfect squares, the centre and r >= r_max in no strip).  Strip means of
    solid rotation are |Omega| times the mean of hypot(dx, dy) over the
    members."""
    n = 15
    orc = _orc(oracle_mod, (n, n, 1), 1, W.uniform_edges(0, n, n), W.uniform_edges(0, n, n),
               W.uniform_edges(0, 1, 1), (False, False))
    X, Y, Z = _grid(orc)
    cx, cy = 7.0, 6.0
    om = 2.5
    q = _state(orc, -om * (Y - cy), om * (X - cx), 0.3 + 0 * X)
    ns = 6
    res = RI.ri_velocity(orc, q, nstrips=ns, rmax=6.0, center=(np.full(2, cx), np.full(2, cy)))
    x, y, _ = orc.lattice_coords()
    for k in range(2):
        cnt = [0] * ns
        acc = [0.0] * ns
        for iy in range(len(y)):
            for ix in range(len(x)):
                ddx, ddy = int(x[ix] - cx), int(y[iy] - cy)
                r2 = ddx * ddx + ddy * ddy
                for j in range(ns):
                    if j * j < r2 < (j + 1) * (j + 1):
                        cnt[j] += 1
                        acc[j] += om * math.hypot(ddx, ddy)
        assert res["count"][k].tolist() == cnt
        assert cnt[0] == 0 and min(cnt[1:]) > 0        # no integer point has 0 < r^2 < 1
        np.testing.assert_allclose(res["ubar"][k], [a / c if c else 0.0 for a, c in zip(acc, cnt)], rtol=1e-13)
    # u_RI is the outermost populated strip's mean (solid rotation grows with r)
    assert res["u_ri"] == res["ubar"][0, ns - 1] and res["r_ri"] == ns - 0.5


def test_empty_strips_and_maximum(oracle_mod):
    """r_max beyond the domain leaves outer strips empty (mean 0, count 0,
    not in the maximum); a state at rest has u_RI = 0 at the first populated
    strip; strips too narrow to hold a node leave u_RI = 0 with no location."""
    orc = _orc(oracle_mod, (3, 3, 1), 4, W.uniform_edges(0, 30e3, 3), W.uniform_edges(0, 30e3, 3),
               W.uniform_edges(0, 1e3, 1), (True, True))
    X, Y, Z = _grid(orc)
    dx, dy = X - 15e3, Y - 15e3
    V = -np.exp(-(dx ** 2 + dy ** 2) / 4e3 ** 2)     # negative rotation: u_theta >= 0 all the same
    q = _state(orc, -V * dy / 4e3, V * dx / 4e3, 0 * X)
    res = RI.ri_velocity(orc, q, nstrips=20, rmax=60e3)
    assert (res["count"][:, 11:] == 0).all() and (res["ubar"][:, 11:] == 0).all()
    assert res["u_ri"] == res["ubar"][res["count"] > 0].max() > 0
    rest = RI.ri_velocity(orc, 0 * q, nstrips=20)
    j0 = int(np.argmax(rest["count"][0] > 0))
    assert rest["u_ri"] == 0.0 and rest["r_ri"] == (j0 + 0.5) * rest["eps"] and rest["umax"] == 0.0
    # centre on a node, r_max below the nearest neighbour's distance (3.3 km)
    c = np.full(orc.nz, 15e3)
    none = RI.ri_velocity(orc, q, nstrips=4, rmax=1e3, center=(c, c))
    assert (none["count"] == 0).all() and none["u_ri"] == 0.0 and none["r_ri"] == -1.0 and none["z_ri"] == -1.0


def test_axisymmetric_vortex_u_ri(oracle_mod):
    """For an axisymmetric vortex V(r) = V_m (r / r_m) exp((1 - (r/r_m)^2) / 2)
    (peak V_m at r_m) on a resolved lattice, u_RI with 50 strips is V_m to the
    strip width's second order (|V''| eps^2 / 8 ~ 0.4 %), located in the
    strip that contains r_m; with a uniform w added it is unchanged (w is not
    tangential)."""
    L, n = 200e3, 40
    orc = _orc(oracle_mod, (n, n, 1), 4, W.uniform_edges(-L / 2, L / 2, n), W.uniform_edges(-L / 2, L / 2, n),
               W.uniform_edges(0, 1e3, 1), (True, True))
    X, Y, Z = _grid(orc)
    vm, rm = 20.0, 25e3
    r = np.sqrt(X ** 2 + Y ** 2)
    V = vm * (r / rm) * np.exp((1 - (r / rm) ** 2) / 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(r > 0, V / r, 0.0)
    q = _state(orc, -s * Y, s * X, 0 * X)
    res = RI.ri_velocity(orc, q, nstrips=50)
    eps = res["eps"]
    assert abs(res["u_ri"] - vm) <= 5e-3 * vm, res["u_ri"]
    assert abs(res["r_ri"] - rm) <= eps, (res["r_ri"], rm)
    q2 = _state(orc, q[1], q[2], 3.0 + 0 * X)
    res2 = RI.ri_velocity(orc, q2, nstrips=50, center=(res["xc"], res["yc"]))
    np.testing.assert_allclose(res2["ubar"], res["ubar"], rtol=1e-13, atol=1e-13 * vm)
    assert abs(res["umax"] - vm) <= 1e-2 * vm


@pytest.mark.parametrize("planted", ["swap_sign", "drop_radial"])
def test_planted_mistakes_fail(oracle_mod, planted):
    """A tangential speed with the radial part kept, or e_r with a wrong
    sign convention applied as rotation, breaks the solid-rotation pin."""
    rng = np.random.default_rng(3)
    dx, dy = rng.normal(size=(2, 50)) * 5e3
    om, al = 2e-4, 9e-5
    u = -om * dy + al * dx
    v = om * dx + al * dy
    r = np.hypot(dx, dy)
    if planted == "swap_sign":
        bad = np.abs(-u * dx + v * dy) / r
    else:
        bad = np.sqrt(u * u + v * v)
    assert not np.allclose(bad, abs(om) * r, rtol=1e-6)
    np.testing.assert_allclose(RI.tangential_speed(u, v, 0 * u, dx, dy), abs(om) * r, rtol=1e-12)
