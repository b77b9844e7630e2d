"""Seeded synthetic workloads shared by the GPU library and the CPU oracle.

This module holds only workload definitions: mesh edges, physical constants,
reference soundings, initial states and forcing fields evaluated at node
coordinates that the caller supplies.  It holds none of the method's
arithmetic (no basis, no derivatives, no assembly, no time stepping); each
side computes its own node coordinates and evaluates these functions there.

Every array is FP64 NumPy; the state layout is field-major ``[5][U]`` with
fields (rho', u, v, w, theta') and the unique node index
``I = ix + n_x (iy + n_y iz)`` (x fastest), i.e. a C-ordered array of shape
``(5, n_z, n_y, n_x)``.

The paper's tropical-cyclone case (Sec. 4.1) uses the Jordan (1958) sounding
and observed Guillermo (1997) heating, neither of which is available here.
The stand-ins keep the case's structure: a doubly periodic box, a warm-core
vortex of the form of Eq. (initial-velocity), convective heating bursts near
the radius of maximum wind, and a top sponge.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Physical constants of dry air (the paper does not print them; NUMA-literature
# values, passed explicitly to both sides).
G = 9.80616
CP = 1004.67
CV = 717.5
RD = CP - CV
PA = 1.0e5


@dataclass
class Physics:
    g: float = G
    R: float = RD
    cp: float = CP
    cv: float = CV
    p_a: float = PA
    f: float = 0.0           # f-plane Coriolis parameter [1/s]
    sponge_z0: float = 0.0   # sponge bottom [m]
    sponge_tau: float = 0.0  # sponge maximum rate [1/s]; 0 disables


@dataclass
class MeshSpec:
    nel: tuple
    order: int
    xe: np.ndarray
    ye: np.ndarray
    ze: np.ndarray
    periodic: tuple

    @property
    def lattice(self):
        N = self.order
        nx = self.nel[0] * N + (0 if self.periodic[0] else 1)
        ny = self.nel[1] * N + (0 if self.periodic[1] else 1)
        nz = self.nel[2] * N + 1
        return nx, ny, nz

    @property
    def U(self):
        nx, ny, nz = self.lattice
        return nx * ny * nz

    @property
    def E(self):
        return self.nel[0] * self.nel[1] * self.nel[2]

    @property
    def L(self):
        return self.E * (self.order + 1) ** 3


def uniform_edges(a, b, n):
    return np.linspace(a, b, n + 1)


def stretched_edges(a, b, n, ratio=1.5, seed=0):
    """Strictly increasing, non-uniform edges (for metric tests)."""
    rng = np.random.default_rng(seed)
    h = 1.0 + (ratio - 1.0) * rng.random(n)
    e = np.concatenate([[0.0], np.cumsum(h)])
    e = a + (b - a) * e / e[-1]
    e[-1] = b
    return e


# ---------------------------------------------------------------- references
def isentropic_reference(z, theta_s=300.0, phys: Physics | None = None):
    """Hydrostatic reference with constant theta0 (Exner pi0 = 1 - g z/(cp theta_s))."""
    p = phys or Physics()
    z = np.asarray(z, dtype=np.float64)
    pi0 = 1.0 - p.g * z / (p.cp * theta_s)
    theta0 = np.full_like(z, theta_s)
    rho0 = p.p_a * pi0 ** (p.cv / p.R) / (p.R * theta0)
    return rho0, theta0


def constant_n_reference(z, bv=0.01, theta_s=300.0, phys: Physics | None = None):
    """Hydrostatic reference with constant Brunt-Vaisala frequency bv."""
    p = phys or Physics()
    z = np.asarray(z, dtype=np.float64)
    theta0 = theta_s * np.exp(bv * bv * z / p.g)
    pi0 = 1.0 + p.g * p.g / (p.cp * bv * bv * theta_s) * (np.exp(-bv * bv * z / p.g) - 1.0)
    rho0 = p.p_a * pi0 ** (p.cv / p.R) / (p.R * theta0)
    return rho0, theta0


def exner_isentropic(z, theta_s=300.0, phys=None):
    p = phys or Physics()
    return 1.0 - p.g * np.asarray(z) / (p.cp * theta_s)


def exner_constant_n(z, bv=0.01, theta_s=300.0, phys=None):
    p = phys or Physics()
    z = np.asarray(z, dtype=np.float64)
    return 1.0 + p.g * p.g / (p.cp * bv * bv * theta_s) * (np.exp(-bv * bv * z / p.g) - 1.0)


# ---------------------------------------------------------------- states
def grid3(x, y, z):
    """3D coordinate arrays of shape (n_z, n_y, n_x) from lattice coordinates."""
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def rest_state(shape):
    return np.zeros((5,) + tuple(shape))


def bubble_state(x, y, z, rho0_z, theta0_z, center=(500.0, 500.0, 350.0),
                 theta_c=0.5, r_c=250.0):
    """Rising warm bubble: cosine-bell theta' of amplitude theta_c and radius r_c,
    at rest, with rho' chosen so that (rho0+rho')(theta0+theta') = rho0 theta0
    (zero pressure perturbation)."""
    X, Y, Z = grid3(x, y, z)
    r = np.sqrt((X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2)
    thp = np.where(r <= r_c, 0.5 * theta_c * (1.0 + np.cos(np.pi * r / r_c)), 0.0)
    th0 = theta0_z[:, None, None]
    r0 = rho0_z[:, None, None]
    rhop = r0 * (th0 / (th0 + thp) - 1.0)
    q = np.zeros((5,) + X.shape)
    q[0] = rhop
    q[4] = thp
    return q


def smooth_random_state(x, y, z, rho0_z, theta0_z, seed=0, amp=1.0, walls=(True, True)):
    """A non-degenerate smooth state for single-RHS parity: random low
    wavenumber velocity, density and temperature perturbations.  Normal
    velocities vanish on walls."""
    rng = np.random.default_rng(seed)
    X, Y, Z = grid3(x, y, z)
    Lx = x.max() - x.min() + (x[1] - x[0]) * (0 if walls[0] else 1)
    Ly = y.max() - y.min() + (y[1] - y[0]) * (0 if walls[1] else 1)
    H = z.max() - z.min()
    xs = (X - x.min()) / Lx
    ys = (Y - y.min()) / Ly
    zs = (Z - z.min()) / H

    def mode():
        a, b, c = rng.integers(1, 3, size=3)
        ph = rng.random(3) * 2 * np.pi
        return (np.sin(2 * np.pi * a * xs + ph[0]) * np.cos(2 * np.pi * b * ys + ph[1])
                * np.cos(np.pi * c * zs + ph[2]))

    q = np.zeros((5,) + X.shape)
    r0 = rho0_z[:, None, None]
    q[0] = 1e-3 * amp * r0 * mode()
    q[1] = amp * 3.0 * mode()
    q[2] = amp * 3.0 * mode()
    q[3] = amp * 1.0 * mode() * np.sin(np.pi * zs)
    q[4] = amp * 0.5 * mode()
    if walls[0]:
        q[1] *= np.sin(np.pi * xs)
    if walls[1]:
        q[2] *= np.sin(np.pi * ys)
    return q


# Vortex of Eq. (initial-velocity): V(r) from a Gaussian vorticity profile,
# vertical decay exp(-z^2/(2 D1^2)) (reading of the garbled exponent, sigma=2),
# lateral cut-off exp(-(r/D2)^6).
D1 = 5823.0
D2 = 200.0e3


def vortex_profile(r, vmax=20.0, rmax=50.0e3):
    L = rmax / 1.120906
    zeta0 = vmax / (0.319086 * L)
    r = np.asarray(r, dtype=np.float64)
    rs = np.where(r > 0, r, 1.0)
    V = np.where(r > 0, zeta0 * L * L * (1.0 - np.exp(-rs * rs / (L * L))) / (2.0 * rs), 0.0)
    return V * np.exp(-(r / D2) ** 6)


def vortex_state(x, y, z, rho0_z, theta0_z, exner0_z, dexner0_z, vmax=20.0, rmax=50.0e3,
                 f=5e-5, center=(0.0, 0.0), phys: Physics | None = None, r_inf=850.0e3):
    """Warm-core vortex in approximate gradient-wind and hydrostatic balance.

    pi'(r, z) = -(cp theta0)^-1 int_r^R (v^2/s + f v) ds; theta from
    cp theta d(pi)/dz = -g; rho and theta perturbations from the total Exner
    function.  The balance is approximate; both sides receive identical
    arrays, so it does not affect parity."""
    p = phys or Physics()
    # radial quantities on the horizontal plane, broadcast over levels
    dx = (np.asarray(x) - center[0])[None, None, :]
    dy = (np.asarray(y) - center[1])[None, :, None]
    r = np.sqrt(dx * dx + dy * dy)
    zz = np.asarray(z)
    Zf = np.exp(-zz * zz / (2 * D1 * D1))
    dZf = -zz / (D1 * D1) * Zf
    # radial integrals A(r) = int_r^R V^2/s ds, B(r) = int_r^R f V ds on a fine grid
    s = np.linspace(0.0, r_inf, 40001)
    Vs = vortex_profile(s, vmax, rmax)
    g1 = np.where(s > 0, Vs * Vs / np.where(s > 0, s, 1.0), 0.0)
    g2 = f * Vs
    ds = s[1] - s[0]
    cumA = np.concatenate([[0.0], np.cumsum(0.5 * (g1[1:] + g1[:-1]) * ds)])
    cumB = np.concatenate([[0.0], np.cumsum(0.5 * (g2[1:] + g2[:-1]) * ds)])
    A = cumA[-1] - np.interp(r, s, cumA)
    B = cumB[-1] - np.interp(r, s, cumB)
    Zc = Zf[:, None, None]
    dZc = dZf[:, None, None]
    th0 = theta0_z[:, None, None]
    dth0 = np.gradient(theta0_z, zz)[:, None, None]
    I = Zc * Zc * A + Zc * B
    dI = 2 * Zc * dZc * A + dZc * B
    pip = -I / (p.cp * th0)
    dpip = -dI / (p.cp * th0) + I * dth0 / (p.cp * th0 * th0)
    pi = exner0_z[:, None, None] + pip
    theta = -p.g / (p.cp * (dexner0_z[:, None, None] + dpip))
    rho = p.p_a * pi ** (p.cv / p.R) / (p.R * theta)
    vt = vortex_profile(r, vmax, rmax) * Zc
    rs = np.where(r > 0, r, 1.0)
    q = np.zeros((5, zz.size, dy.size, dx.size))
    q[0] = rho - rho0_z[:, None, None]
    q[1] = np.where(r > 0, -vt * dy / rs, 0.0)
    q[2] = np.where(r > 0, vt * dx / rs, 0.0)
    q[4] = theta - th0
    return q


@dataclass
class BurstSchedule:
    xc: np.ndarray
    yc: np.ndarray
    tb: np.ndarray
    amp: float = 10.0 / 3600.0   # K/s
    rb: float = 5.0e3
    taub: float = 1800.0
    ztop: float = 15.0e3


def burst_schedule(T=3600.0, seed=2, ring=40.0e3, per_hour=12, center=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    nb = max(1, int(round(per_hour * T / 3600.0)))
    taub = 1800.0
    phi = rng.random(nb) * 2 * np.pi
    tb = rng.random(nb) * max(T - taub, 0.0)
    return BurstSchedule(center[0] + ring * np.cos(phi), center[1] + ring * np.sin(phi), tb,
                         taub=taub)


def heating_field(x, y, z, t, sched: BurstSchedule):
    """Q(x, y, z, t) [K/s]: sum of Gaussian convective bursts with a
    sin(pi z / ztop) vertical profile below ztop and a sin^2 life cycle.
    Returned in (n_z, n_y, n_x) layout."""
    x = np.asarray(x); y = np.asarray(y); z = np.asarray(z)
    plane = np.zeros((y.size, x.size))
    for b in range(sched.xc.size):
        tt = (t - sched.tb[b]) / sched.taub
        if tt < 0.0 or tt > 1.0:
            continue
        life = math.sin(math.pi * tt) ** 2
        gx = np.exp(-((x - sched.xc[b]) / sched.rb) ** 2)
        gy = np.exp(-((y - sched.yc[b]) / sched.rb) ** 2)
        plane += sched.amp * life * np.outer(gy, gx)
    zp = np.where(z < sched.ztop, np.sin(np.pi * z / sched.ztop), 0.0)
    return zp[:, None, None] * plane[None, :, :]


def heating_snapshots(x, y, z, T, sched: BurstSchedule, nsnap=11):
    t = np.array([k * T / (nsnap - 1) for k in range(nsnap)])
    snaps = np.empty((nsnap, np.size(z), np.size(y), np.size(x)))
    for k, tk in enumerate(t):
        snaps[k] = heating_field(x, y, z, tk, sched)
    return t, snaps


# ---------------------------------------------------------------- configs
@dataclass
class Workload:
    name: str
    mesh: MeshSpec
    phys: Physics
    dt: float
    steps: int
    reference: str           # "isentropic" | "constant_n"
    ic: str                  # "bubble" | "vortex" | "rest" | "random"
    vmax: float = 20.0
    heating_T: float = 0.0   # window of the heating snapshots (0: no heating)
    heating_seed: int = 2
    extra: dict = field(default_factory=dict)


def cfg_bubble():
    """Rising warm bubble: 1 km cube, 4x4x4 elements, N=4, all walls, isentropic
    theta0 = 300 K, 0.5 K cosine bell of radius 250 m at z = 350 m, SSP-RK3,
    dt = 0.01 s, 20 steps."""
    n = 4
    mesh = MeshSpec((n, n, n), 4, uniform_edges(0, 1000.0, n), uniform_edges(0, 1000.0, n),
                    uniform_edges(0, 1000.0, n), (False, False))
    return Workload("bubble_4x4x4_N4", mesh, Physics(), 0.01, 20, "isentropic", "bubble")


def _tc_mesh(nx, ny, nz, N=4, half=600.0e3, H=20.0e3):
    return MeshSpec((nx, ny, nz), N, uniform_edges(-half, half, nx), uniform_edges(-half, half, ny),
                    uniform_edges(0.0, H, nz), (True, True))


def _tc_phys():
    return Physics(f=5e-5, sponge_z0=15.0e3, sponge_tau=0.02)


def cfg_tc_small():
    """Synthetic TC, 1200x1200x20 km f-plane box, 64x64x10 elements, N=4,
    dt = 0.5 s, 1 h (7200 steps)."""
    return Workload("tc_64x64x10_N4", _tc_mesh(64, 64, 10), _tc_phys(), 0.5, 7200,
                    "constant_n", "vortex", vmax=20.0, heating_T=3600.0)


def cfg_tc_large():
    """Per-GPU share: same physics at 128x128x20 elements, N=4, dt = 0.25 s,
    600 steps; heating from the 1 h burst schedule of the small case."""
    return Workload("tc_128x128x20_N4", _tc_mesh(128, 128, 20), _tc_phys(), 0.25, 600,
                    "constant_n", "vortex", vmax=20.0, heating_T=3600.0)


def cfg_hevi():
    """1D-IMEX (HEVI) case: 96x96x16 elements, N=4, dt = 2 s."""
    return Workload("tc_hevi_96x96x16_N4", _tc_mesh(96, 96, 16), _tc_phys(), 2.0, 50,
                    "constant_n", "vortex", vmax=20.0, heating_T=3600.0)


def cfg_ensemble_member(i):
    """Member i of the 48-instance uneven ensemble (rng(4000+i))."""
    rng = np.random.default_rng(4000 + i)
    nx = int(rng.integers(8, 41)); ny = int(rng.integers(8, 41)); nz = int(rng.integers(8, 17))
    N = int(rng.integers(3, 6)); vmax = float(rng.uniform(10.0, 30.0))
    if i == 0:
        nx, ny, nz = 8, 8, 8
    if i == 1:
        nx, ny, nz = 40, 40, 16
    return Workload(f"ens{i}_{nx}x{ny}x{nz}_N{N}", _tc_mesh(nx, ny, nz, N), _tc_phys(), 0.25, 100,
                    "constant_n", "vortex", vmax=vmax, heating_T=3600.0, heating_seed=5000 + i)


def reference_profiles(w: Workload, z):
    if w.reference == "isentropic":
        return isentropic_reference(z, phys=w.phys)
    return constant_n_reference(z, phys=w.phys)


def initial_state(w: Workload, x, y, z, seed=0):
    """Initial state of workload w on lattice coordinates (x, y, z)."""
    rho0, theta0 = reference_profiles(w, z)
    if w.ic == "bubble":
        return bubble_state(x, y, z, rho0, theta0)
    if w.ic == "rest":
        return rest_state((z.size, y.size, x.size))
    if w.ic == "random":
        return smooth_random_state(x, y, z, rho0, theta0, seed=seed,
                                   walls=(not w.mesh.periodic[0], not w.mesh.periodic[1]))
    if w.reference == "isentropic":
        ex = exner_isentropic(z, phys=w.phys)
        dex = np.full_like(z, -w.phys.g / (w.phys.cp * 300.0))
    else:
        bv, ths = 0.01, 300.0
        ex = exner_constant_n(z, bv, ths, w.phys)
        dex = -w.phys.g / (w.phys.cp * ths) * np.exp(-bv * bv * z / w.phys.g)
    return vortex_state(x, y, z, rho0, theta0, ex, dex, vmax=w.vmax, f=w.phys.f, phys=w.phys)


def heating(w: Workload, x, y, z, nsnap=11):
    """Heating snapshots (t[nsnap], Q[nsnap, n_z, n_y, n_x]) or None."""
    if w.heating_T <= 0:
        return None
    sched = burst_schedule(T=w.heating_T, seed=w.heating_seed)
    return heating_snapshots(x, y, z, w.heating_T, sched, nsnap)


def random_column_rhs(z, D, ncol, seed, modes=24):
    """Seeded right-hand sides for column solves, [5][n_z][ncol]: for each of
    (rho', w, theta') a random smooth profile (sum of sin(m pi zh / 2 + phase)
    with amplitudes ~ m^-p, p uniform in [0.5, 2.5]) plus white noise of
    log-uniform relative size, the field magnitude log-uniform over three
    decades, times the level factors D [3][n_z] (the reference density,
    sound speed and potential temperature); u = v = 0 and w = 0 on the bottom
    and top levels."""
    rng = np.random.default_rng(seed)
    z = np.asarray(z, dtype=np.float64)
    nz = z.size
    zh = (z - z[0]) / (z[-1] - z[0])
    q = np.zeros((5, nz, ncol))
    for f, fld in enumerate((0, 3, 4)):
        amp = 10.0 ** rng.uniform(-3.0, 0.0, size=ncol)
        decay = rng.uniform(0.5, 2.5, size=ncol)
        prof = np.zeros((nz, ncol))
        for m in range(1, modes + 1):
            a = rng.normal(size=ncol) * m ** (-decay)
            ph = rng.uniform(0.0, 2.0 * np.pi, size=ncol)
            prof += a * np.sin(m * np.pi * zh[:, None] / 2.0 + ph)
        prof += rng.normal(size=(nz, ncol)) * 10.0 ** rng.uniform(-3.0, 0.0, size=ncol)
        q[fld] = prof * amp * np.asarray(D[f])[:, None]
    q[3, 0] = 0.0
    q[3, -1] = 0.0
    return q
