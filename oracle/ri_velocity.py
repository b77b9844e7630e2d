"""FP64 NumPy oracle of the RI-velocity diagnostic (test infrastructure only:
used by the tests and nothing else).

Paper, section on the RI velocity (equations u_RI, azimuthal average,
tangential velocity, centroid, and the strip approximation of the average):

    u_RI = max over (r, z) of  ubar_theta(r, z),
    ubar_theta(r, z) = azimuthal mean of u_theta at radius r and height z,
    u_theta = || (I - e_r e_r^T - e_z e_z^T) u ||,
    e_r = (x - x_c, y - y_c, 0) / || . ||,  e_z = (0, 0, 1),
    x_c(z) = int int ||u|| x dx dy / int int ||u|| dx dy   (per level),

with the azimuthal mean replaced by the arithmetic mean over the lattice
points of a narrow annulus (strip) at each radius and level, and 50 strips
of equal width in the paper's figures.

Readings (the paper does not fix them):
  * the x-y integrals at a level are the LGL quadrature on the lattice (the
    diagonal mass; its per-level factor cancels in the ratio), with the
    coordinates as they are (no periodic unwrapping: the vortex is assumed
    not to straddle a periodic boundary); a level where the speed vanishes
    everywhere takes the midpoint of the domain as its centre;
  * the strips cover 0 < r < r_max with width eps = r_max / n_strips; strip j
    is the open annulus j eps < r < (j + 1) eps, decided in FP64 on squared
    radii, r^2 = dx dx + dy dy against (j eps)(j eps) with no fused
    multiply-add; points on a strip edge, and the centre itself, belong to no
    strip;
  * an empty strip reports mean 0 and count 0 and takes no part in the
    maximum; ties in the maximum go to the first strip in (level, strip)
    order;
  * r_max is an input (the tests and benchmark use half the smaller
    horizontal extent of the domain);
  * alongside u_RI the maximum horizontal speed max sqrt(u^2 + v^2), the
    quantity the paper plots against it.
"""
from __future__ import annotations

import numpy as np


def centroid(orc, q):
    """Per-level centre (x_c[n_z], y_c[n_z]) of the speed field of state q."""
    x, y, _ = orc.lattice_coords()
    q = np.asarray(q, dtype=np.float64).reshape((5,) + orc.shape)
    speed = np.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2)
    W = orc.mass() * speed
    den = W.sum(axis=(1, 2))
    m = orc.mesh
    xm = 0.5 * (float(m.xe[0]) + float(m.xe[-1]))
    ym = 0.5 * (float(m.ye[0]) + float(m.ye[-1]))
    with np.errstate(invalid="ignore", divide="ignore"):
        xc = np.where(den > 0, (W * x[None, None, :]).sum(axis=(1, 2)) / den, xm)
        yc = np.where(den > 0, (W * y[None, :, None]).sum(axis=(1, 2)) / den, ym)
    return xc, yc


def tangential_speed(u, v, w, dx, dy):
    """u_theta = ||(I - e_r e_r^T - e_z e_z^T) u|| at points offset (dx, dy)
    from the centre (r > 0)."""
    r = np.sqrt(dx * dx + dy * dy)
    erx, ery = dx / r, dy / r
    ur = u * erx + v * ery                     # u . e_r
    px = u - ur * erx
    py = v - ur * ery
    pz = w - w                                 # (u . e_z) e_z removed
    return np.sqrt(px * px + py * py + pz * pz)


def strip_index(r2, eps, nstrips):
    """Strip of each squared radius (-1: in no strip)."""
    b = np.arange(nstrips + 1, dtype=np.float64) * eps
    b2 = b * b
    i = np.searchsorted(b2, r2, side="left")   # b2[i-1] < r2 <= b2[i]
    inside = (i >= 1) & (i <= nstrips)
    inside &= r2 < b2[np.minimum(i, nstrips)]
    return np.where(inside, i - 1, -1)


def ri_velocity(orc, q, nstrips=50, rmax=None, center=None):
    """The diagnostic of state q [5][U]: returns a dict with the centre
    (x_c, y_c per level), the strip means ubar [n_z][n_strips], the counts,
    u_RI with its strip radius and level height, and the maximum horizontal
    speed.  `center` (x_c, y_c arrays) replaces the computed centroid."""
    x, y, z = orc.lattice_coords()
    m = orc.mesh
    if rmax is None:
        rmax = 0.5 * min(float(m.xe[-1]) - float(m.xe[0]), float(m.ye[-1]) - float(m.ye[0]))
    eps = rmax / nstrips
    xc, yc = centroid(orc, q) if center is None else (np.asarray(center[0], float), np.asarray(center[1], float))
    q = np.asarray(q, dtype=np.float64).reshape((5,) + orc.shape)
    nz = orc.nz
    ubar = np.zeros((nz, nstrips))
    count = np.zeros((nz, nstrips), dtype=np.int64)
    X, Y = np.meshgrid(x, y)                   # [n_y][n_x]
    for k in range(nz):
        dx = X - xc[k]
        dy = Y - yc[k]
        r2 = dx * dx + dy * dy
        j = strip_index(r2.ravel(), eps, nstrips)
        sel = j >= 0
        ut = tangential_speed(q[1, k].ravel()[sel], q[2, k].ravel()[sel], q[3, k].ravel()[sel],
                              dx.ravel()[sel], dy.ravel()[sel])
        s = np.bincount(j[sel], weights=ut, minlength=nstrips)
        c = np.bincount(j[sel], minlength=nstrips)
        count[k] = c
        ubar[k] = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    flat = np.where(count.ravel() > 0, ubar.ravel(), -np.inf)
    if np.isfinite(flat).any():
        a = int(np.argmax(flat))
        kk, jj = divmod(a, nstrips)
        u_ri, r_ri, z_ri = float(ubar[kk, jj]), (jj + 0.5) * eps, float(z[kk])
    else:
        u_ri, r_ri, z_ri = 0.0, -1.0, -1.0
    umax = float(np.sqrt(q[1] ** 2 + q[2] ** 2).max())
    return {"xc": xc, "yc": yc, "ubar": ubar, "count": count, "u_ri": u_ri, "r_ri": r_ri, "z_ri": z_ri,
            "umax": umax, "eps": eps}
