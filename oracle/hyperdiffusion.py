"""FP64 NumPy oracle of the tensor hyper-diffusion term (test infrastructure
only: used by the tests and nothing else).

Paper, section on tensor-based hyper-diffusion (equations hyperdiffusion,
tau_tensor, viscosity_scaled):

    H_q = (-1)^(alpha+1) (div tau grad)^alpha q,   alpha = 2 here,

with tau applied inside every application of the Laplacian, and

    tau = (J E) diag(nu_i lambda_i^-1) (J E)^T,

J = dx/dxi the Jacobian of the element map, G = J^-1 J^-T the metric tensor,
lambda_i^-1 its eigenvalues in ascending order and E its orthonormal
eigenvectors (columns), nu_i = c_i^(1/alpha) dx_i^2 / dt^(1/alpha).

Readings (the paper does not fix them):
  * dx_i is the element's extent along principal axis i, 2 / sqrt(lambda_i^-1)
    (for a box element: its edge length along that axis);
  * where G has repeated eigenvalues the principal axes are the coordinate
    axes, taken in the order x, y, z;
  * the Laplacian is the continuous-Galerkin weak form with the co-located
    LGL quadrature of the right-hand side: per element
    r_a = - sum_n w_n |J_n| grad psi_a(x_n) . tau_n grad q(x_n), then direct
    stiffness summation and the inverse of the assembled diagonal mass;
    no boundary term (natural condition on walls; periodic directions wrap);
  * H_q is applied to all five prognostic fields;
  * the no-flux walls are imposed strongly on the whole tendency, H_q
    included: after H_q is formed, the wall-normal velocity rows (u on the
    x walls, v on the y walls, w at the bottom and the top) are set to zero,
    as the right-hand side does after its DSS (hyperdiffusion_tendency).

Everything is evaluated element by element from the node coordinates; no
assumption on the element shape is made.
"""
from __future__ import annotations

from functools import cmp_to_key

import numpy as np


def principal_axes(G, tol=1e-10):
    """Eigenvalues (ascending) and eigenvectors (columns) of the symmetric
    3x3 metric tensor G.  A G that is diagonal to within tol (relative) keeps
    the coordinate axes, ordered by eigenvalue with values equal to within
    tol taken in x, y, z order (the Jacobian computed from node coordinates
    carries rounding noise of ~1e-13, which must not decide a tie)."""
    g = np.abs(G).max()
    off = G - np.diag(np.diag(G))
    if np.all(np.abs(off) <= tol * g):
        d = np.diag(G)

        def before(a, b):
            if d[a] < d[b] - tol * g:
                return -1
            if d[b] < d[a] - tol * g:
                return 1
            return -1 if a < b else 1

        order = sorted(range(3), key=cmp_to_key(before))
        return d[order], np.eye(3)[:, order]
    mu, E = np.linalg.eigh(G)
    return mu, E


def viscosity_tensor(J, c, dt, alpha=2):
    """tau at one node from the Jacobian J (3x3), the coefficients c (3) and
    the time step."""
    Jinv = np.linalg.inv(J)
    G = Jinv @ Jinv.T
    mu, E = principal_axes(G)                 # mu_i = lambda_i^-1, ascending
    dxi = 2.0 / np.sqrt(mu)                   # extent along principal axis i
    nu = np.asarray(c, dtype=np.float64) ** (1.0 / alpha) * dxi ** 2 / dt ** (1.0 / alpha)
    JE = J @ E
    return JE @ np.diag(nu * mu) @ JE.T


class ElementGeometry:
    """Node coordinates, Jacobians and quadrature weights of every element of
    an Oracle mesh: element e = ex + nel_x (ey + nel_y ez) spans
    [xe[ex], xe[ex+1]] x [ye[ey], ye[ey+1]] x [ze[ez], ze[ez+1]], its node
    (i, j, k) sits at the LGL points of that box (a periodic element keeps
    its own coordinates; the element-to-lattice map does the wrap)."""

    def __init__(self, orc):
        self.orc = orc
        xi, w, D = orc.basis()
        self.n1 = n1 = orc.N + 1
        self.D = D
        self.w3 = np.einsum("k,j,i->kji", w, w, w)
        self.im = orc.intma().reshape(-1, n1, n1, n1)   # [e][k][j][i] -> lattice index
        m = orc.mesh
        nel = [int(v) for v in m.nel]
        edges = [np.asarray(m.xe, dtype=np.float64), np.asarray(m.ye, dtype=np.float64),
                 np.asarray(m.ze, dtype=np.float64)]
        E = nel[0] * nel[1] * nel[2]
        X = np.zeros((E, n1, n1, n1, 3))
        for ez in range(nel[2]):
            for ey in range(nel[1]):
                for ex in range(nel[0]):
                    e = ex + nel[0] * (ey + nel[1] * ez)
                    cx = edges[0][ex] + (xi + 1.0) / 2.0 * (edges[0][ex + 1] - edges[0][ex])
                    cy = edges[1][ey] + (xi + 1.0) / 2.0 * (edges[1][ey + 1] - edges[1][ey])
                    cz = edges[2][ez] + (xi + 1.0) / 2.0 * (edges[2][ez + 1] - edges[2][ez])
                    X[e, :, :, :, 0] = cx[None, None, :]
                    X[e, :, :, :, 1] = cy[None, :, None]
                    X[e, :, :, :, 2] = cz[:, None, None]
        self.X = X
        # J[e,k,j,i][a, b] = d x_a / d xi_b (xi_0 along i, xi_1 along j, xi_2 along k)
        J = np.zeros(X.shape[:-1] + (3, 3))
        for a in range(3):
            J[..., a, 0] = np.einsum("im,ekjm->ekji", D, X[..., a])
            J[..., a, 1] = np.einsum("jm,ekmi->ekji", D, X[..., a])
            J[..., a, 2] = np.einsum("km,emji->ekji", D, X[..., a])
        self.J = J
        self.detJ = np.linalg.det(J)


def weak_laplacian(geo, q, c, dt, alpha=2):
    """(div tau grad) q on the lattice for every field of q [nf][U]."""
    orc, D, n1 = geo.orc, geo.D, geo.n1
    q = np.asarray(q, dtype=np.float64).reshape(-1, orc.U)
    E = geo.im.shape[0]
    tau = np.zeros(geo.J.shape)
    for e in range(E):
        for idx in np.ndindex(n1, n1, n1):
            tau[(e,) + idx] = viscosity_tensor(geo.J[(e,) + idx], c, dt, alpha)
    Jinv = np.linalg.inv(geo.J)
    # contravariant flux matrix per node: w |J| J^-1 tau J^-T
    K = np.einsum("ekji,ekjiab,ekjibc,ekjidc->ekjiad", geo.w3[None] * geo.detJ, Jinv, tau, Jinv)
    out = np.zeros_like(q)
    M = orc.mass().reshape(-1)
    for f in range(q.shape[0]):
        qe = q[f][geo.im]                                # [e][k][j][i]
        g = np.stack([np.einsum("im,ekjm->ekji", D, qe),
                      np.einsum("jm,ekmi->ekji", D, qe),
                      np.einsum("km,emji->ekji", D, qe)], axis=-1)
        F = np.einsum("ekjiab,ekjib->ekjia", K, g)
        r = -(np.einsum("mi,ekjm->ekji", D, F[..., 0]) +
              np.einsum("mj,ekmi->ekji", D, F[..., 1]) +
              np.einsum("mk,emji->ekji", D, F[..., 2]))
        acc = np.zeros(orc.U)
        np.add.at(acc, geo.im.reshape(-1), r.reshape(-1))
        out[f] = acc / M
    return out


def hyperdiffusion(geo, q, c, dt, alpha=2):
    """H_q = (-1)^(alpha+1) (div tau grad)^alpha q for every field of q."""
    r = np.asarray(q, dtype=np.float64).reshape(-1, geo.orc.U)
    for _ in range(alpha):
        r = weak_laplacian(geo, r, c, dt, alpha)
    return (-1) ** (alpha + 1) * r


def wall_mask(orc, F):
    """Zero the wall-normal velocity rows of a tendency F [5][U]: u where the
    lattice x index is 0 or n_x - 1 on a non-periodic x, v likewise in y, w
    at the bottom and top levels (the no-flux condition imposed strongly)."""
    F = np.array(F, dtype=np.float64).reshape((5,) + orc.shape)
    per = [bool(v) for v in orc.mesh.periodic]
    if not per[0]:
        F[1][:, :, 0] = 0.0
        F[1][:, :, -1] = 0.0
    if not per[1]:
        F[2][:, 0, :] = 0.0
        F[2][:, -1, :] = 0.0
    F[3][0] = 0.0
    F[3][-1] = 0.0
    return F.reshape(5, -1)


def hyperdiffusion_tendency(geo, q, c, dt, alpha=2):
    """The contribution of H_q to dq/dt: H_q of all five fields with the
    wall-normal velocity rows zeroed."""
    return wall_mask(geo.orc, hyperdiffusion(geo, q, c, dt, alpha))
