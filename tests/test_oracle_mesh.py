"""Pins of the oracle's mesh, element->unique map and DSS'd mass
(Sec. 2.2, mass matrix; Algorithm 1 intma)."""
import os

import numpy as np
import pytest

from paper_2504_08157_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.txt")


def _mesh(nel, N, periodic, stretch=False):
    if stretch:
        e = [W.stretched_edges(0.0, L, n, seed=s) for n, L, s in zip(nel, (1000.0, 800.0, 500.0), (1, 2, 3))]
    else:
        e = [W.uniform_edges(0.0, L, n) for n, L in zip(nel, (1000.0, 800.0, 500.0))]
    return W.MeshSpec(tuple(nel), N, e[0], e[1], e[2], periodic)


@pytest.mark.parametrize("periodic", [(False, False), (True, True), (True, False)])
@pytest.mark.parametrize("stretch", [False, True])
def test_sizes_and_mass(oracle_mod, periodic, stretch):
    N = 3
    m = _mesh((3, 4, 2), N, periodic, stretch)
    o = oracle_mod.Oracle(m)
    nx = 3 * N + (0 if periodic[0] else 1)
    ny = 4 * N + (0 if periodic[1] else 1)
    nz = 2 * N + 1
    assert (o.nx, o.ny, o.nz) == (nx, ny, nz)
    assert o.U == nx * ny * nz and o.L == 24 * (N + 1) ** 3
    M = o.mass()
    # total mass = box volume
    assert abs(M.sum() - 1000.0 * 800.0 * 500.0) < 1e-15 * 4e8 * 10
    assert (M > 0).all()
    # separable product of independently assembled 1D masses
    xi, w, _ = oracle_mod.lgl(N)

    def m1(edges, per):
        n = (len(edges) - 1) * N + (0 if per else 1)
        out = np.zeros(n)
        for e in range(len(edges) - 1):
            h = edges[e + 1] - edges[e]
            for i in range(N + 1):
                out[(e * N + i) % n] += w[i] * h / 2
        return out
    Msep = (m1(m.ze, False)[:, None, None] * m1(m.ye, periodic[1])[None, :, None]
            * m1(m.xe, periodic[0])[None, None, :])
    np.testing.assert_allclose(M, Msep, rtol=1e-14)


def test_intma_periodic_identification(oracle_mod):
    N = 2
    m = _mesh((3, 2, 2), N, (True, True))
    o = oracle_mod.Oracle(m)
    im = o.intma().reshape(o.E, N + 1, N + 1, N + 1)  # [e][k][j][i]
    # every unique node is hit; counts follow the tensor structure
    cnt = np.bincount(im.ravel(), minlength=o.U)
    assert (cnt > 0).all()
    # last x-node of element ex = nel_x-1 is node 0 of element 0 (periodic)
    e_last = 2  # ex = 2, ey = 0, ez = 0
    assert im[e_last, 0, 0, N] == im[0, 0, 0, 0]
    # coordinates: shared nodes agree exactly; lattice is monotone
    x, y, z = o.lattice_coords()
    assert (np.diff(x) > 0).all() and (np.diff(z) > 0).all()
    assert x[0] == m.xe[0] and z[-1] == m.ze[-1]


def test_paper_dof_counts(oracle_mod):
    rows = []
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows.append((parts[0], tuple(int(v) for v in parts[1:4]), int(parts[4]), int(parts[5])))
    for name, nel, N, dof in rows:
        assert nel[0] * nel[1] * nel[2] * (N + 1) ** 3 * 5 == dof, name
    # the oracle's local-node count on the smallest printed grid
    name, nel, N, dof = [r for r in rows if r[0] == "weak_per_gpu"][0]
    m = W.MeshSpec(nel, N, W.uniform_edges(-400e3, 400e3, nel[0]), W.uniform_edges(-400e3, 400e3, nel[1]),
                   W.uniform_edges(0, 20e3, nel[2]), (True, True))
    o = oracle_mod.Oracle(m)
    assert o.L * 5 == dof
    # vertical spacing of Sec. 4.1: 20 km / (24 * 5) = 166.7 m, printed as 167 m
    assert abs(20000.0 / (24 * 5) - 167.0) < 0.5
