"""Python side of the FP64 CPU oracle (test infrastructure only).

`Oracle` wraps the plain C implementation in ``nh_oracle.c`` (element
tendencies, DSS, SSP-RK3, the vertical HEVI operator).  The HEVI ARK2 step
with direct column solves (LAPACK through NumPy) lives here.

Nothing here is imported by the GPU library; nothing here imports it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)


def build(force=True):
    """Compile the oracle with gcc: plain FP64, no FMA contraction, OpenMP."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.or_lgl.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    lib.or_lgl.restype = ctypes.c_int
    lib.or_create.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp, _ip]
    lib.or_create.restype = ctypes.c_void_p
    lib.or_destroy.argtypes = [ctypes.c_void_p]
    lib.or_sizes.argtypes = [ctypes.c_void_p, _lp]
    lib.or_basis.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.or_lattice_coords.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.or_mass.argtypes = [ctypes.c_void_p, _dp]
    lib.or_intma.argtypes = [ctypes.c_void_p, _lp]
    lib.or_set_physics.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 8
    lib.or_set_reference.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.or_reference_pressure.argtypes = [ctypes.c_void_p, _dp]
    lib.or_set_forcing.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.or_set_forcing.restype = ctypes.c_int
    lib.or_element_tendency.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp]
    lib.or_rhs.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp]
    lib.or_rk3.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
    lib.or_dss.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.or_scatter.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    lib.or_lv_apply.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.or_l3_apply.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    lib.or_rhs_sample.restype = ctypes.c_int
    lib.or_rhs_sample.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, ctypes.c_int64, _lp, _dp]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lgl(N):
    """LGL nodes, weights and derivative matrix D[i, j] = h_j'(xi_i)."""
    lib = load()
    xi = np.zeros(N + 1); w = np.zeros(N + 1); D = np.zeros((N + 1, N + 1))
    if lib.or_lgl(N, _p(xi), _p(w), _p(D)) != 0:
        raise ValueError("unsupported order")
    return xi, w, D


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(load().or_num_threads())


def set_num_threads(n):
    """Threads of the oracle's later parallel loops."""
    load().or_set_num_threads(int(n))


class Oracle:
    """FP64 oracle on an axis-aligned hexahedral box (Sec. 4.1 domain shape)."""

    def __init__(self, mesh, phys=None):
        lib = load()
        self.lib = lib
        self.mesh = mesh
        nel = (ctypes.c_int * 3)(*[int(v) for v in mesh.nel])
        per = (ctypes.c_int * 2)(*[1 if v else 0 for v in mesh.periodic])
        self._xe, self._ye, self._ze = _c(mesh.xe), _c(mesh.ye), _c(mesh.ze)
        h = lib.or_create(int(mesh.order), nel, _p(self._xe), _p(self._ye), _p(self._ze), per)
        if not h:
            raise ValueError("invalid mesh")
        self.h = ctypes.c_void_p(h)
        s = np.zeros(6, dtype=np.int64)
        lib.or_sizes(self.h, s.ctypes.data_as(_lp))
        self.nx, self.ny, self.nz, self.U, self.L, self.E = [int(v) for v in s]
        self.N = int(mesh.order)
        if phys is not None:
            self.set_physics(phys)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.or_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- geometry
    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def basis(self):
        n1 = self.N + 1
        xi = np.zeros(n1); w = np.zeros(n1); D = np.zeros((n1, n1))
        self.lib.or_basis(self.h, _p(xi), _p(w), _p(D))
        return xi, w, D

    def lattice_coords(self):
        x = np.zeros(self.nx); y = np.zeros(self.ny); z = np.zeros(self.nz)
        self.lib.or_lattice_coords(self.h, _p(x), _p(y), _p(z))
        return x, y, z

    def mass(self):
        M = np.zeros(self.U)
        self.lib.or_mass(self.h, _p(M))
        return M.reshape(self.shape)

    def intma(self):
        im = np.zeros(self.L, dtype=np.int64)
        self.lib.or_intma(self.h, im.ctypes.data_as(_lp))
        return im

    # -- physics
    def set_physics(self, ph):
        self.phys = ph
        self.lib.or_set_physics(self.h, ph.g, ph.R, ph.cp, ph.cv, ph.p_a, ph.f,
                                ph.sponge_z0, ph.sponge_tau)

    def set_reference(self, rho0_z, theta0_z):
        self._rho0, self._theta0 = _c(rho0_z), _c(theta0_z)
        assert self._rho0.size == self.nz and self._theta0.size == self.nz
        self.lib.or_set_reference(self.h, _p(self._rho0), _p(self._theta0))

    def reference_pressure(self):
        p0 = np.zeros(self.nz)
        self.lib.or_reference_pressure(self.h, _p(p0))
        return p0

    def set_forcing(self, field, t, snaps):
        t = _c(np.atleast_1d(t))
        snaps = _c(snaps).reshape(t.size, self.U)
        if self.lib.or_set_forcing(self.h, int(field), int(t.size), _p(t), _p(snaps)) != 0:
            raise ValueError("bad forcing")

    def clear_forcing(self, field):
        self.lib.or_set_forcing(self.h, int(field), 0, None, None)

    # -- operators
    def element_tendency(self, t, q):
        q = _c(q).reshape(5, self.U)
        r = np.zeros((5, self.L))
        self.lib.or_element_tendency(self.h, float(t), _p(q), _p(r))
        return r

    def rhs(self, t, q):
        q = _c(q).reshape(5, self.U)
        out = np.zeros((5, self.U))
        self.lib.or_rhs(self.h, float(t), _p(q), _p(out))
        return out.reshape((5,) + self.shape)

    def rhs_sample(self, t, q, nodes):
        """Right-hand side [5][n] at unique nodes `nodes` only (same
        arithmetic as rhs)."""
        q = _c(q).reshape(5, self.U)
        uniq, inv = np.unique(np.asarray(nodes, dtype=np.int64), return_inverse=True)
        uniq = np.ascontiguousarray(uniq)
        out = np.zeros((5, uniq.size))
        rc = self.lib.or_rhs_sample(self.h, float(t), _p(q), int(uniq.size), uniq.ctypes.data_as(_lp), _p(out))
        if rc != 0:
            raise ValueError("or_rhs_sample: node index out of range or repeated")
        return out[:, inv.reshape(-1)]

    def rk3(self, t, dt, nsteps, q):
        q = _c(q).reshape(5, self.U).copy()
        self.lib.or_rk3(self.h, float(t), float(dt), int(nsteps), _p(q))
        return q.reshape((5,) + self.shape)

    def dss(self, E, mode=0):
        E = _c(E)
        nf = E.size // self.L
        out = np.zeros((nf, self.U))
        self.lib.or_dss(self.h, nf, int(mode), _p(E), _p(out))
        return out

    def scatter(self, Uv):
        Uv = _c(Uv)
        nf = Uv.size // self.U
        E = np.zeros((nf, self.L))
        self.lib.or_scatter(self.h, nf, _p(Uv), _p(E))
        return E

    def lv_apply(self, x):
        x = _c(x).reshape(5, self.U)
        y = np.zeros((5, self.U))
        self.lib.or_lv_apply(self.h, _p(x), _p(y))
        return y.reshape((5,) + self.shape)

    def l3_apply(self, x):
        """The 3D-IMEX linear operator (acoustic and gravity terms in all
        directions, implicit damping of w in the absorbing layer)."""
        x = _c(x).reshape(5, self.U)
        y = np.zeros((5, self.U))
        self.lib.or_l3_apply(self.h, _p(x), _p(y))
        return y.reshape((5,) + self.shape)


# ---------------------------------------------------------------- HEVI / ARK2
def hevi_coefficients():
    """ARK2 of Giraldo, Kelly & Constantinescu (2013), cited in Sec. 2.3 as
    ARK(2,3,2)b: explicit tableau A, implicit tableau At, weights b (= bt),
    abscissae c."""
    gam = 1.0 - 1.0 / math.sqrt(2.0)
    dlt = 1.0 / (2.0 * math.sqrt(2.0))
    alp = (3.0 + 2.0 * math.sqrt(2.0)) / 6.0
    A = np.array([[0, 0, 0], [2 * gam, 0, 0], [1 - alp, alp, 0]], dtype=np.float64)
    At = np.array([[0, 0, 0], [gam, gam, 0], [dlt, dlt, gam]], dtype=np.float64)
    b = np.array([dlt, dlt, gam])
    c = np.array([0.0, 2 * gam, 1.0])
    return A, At, b, c


def column_matrix(orc: Oracle):
    """Matrix of the oracle's own L_v restricted to one column, assembled by
    applying L_v to unit vectors of (rho', w, theta') at lattice column
    (0, 0).  Unknown ordering: field-major [rho'(z), w(z), theta'(z)].
    L_v couples only points of the same column and its coefficients depend
    on z alone, so one matrix serves every column."""
    nz = orc.nz
    fields = (0, 3, 4)
    n = 3 * nz
    Lm = np.zeros((n, n))
    for a, fa in enumerate(fields):
        for k in range(nz):
            x = np.zeros((5,) + orc.shape)
            x[fa, k, 0, 0] = 1.0
            y = orc.lv_apply(x)
            for b2, fb in enumerate(fields):
                Lm[b2 * nz:(b2 + 1) * nz, a * nz + k] = y[fb, :, 0, 0]
    return Lm


def _solve_columns(Lm, dt_a, rhs):
    """Solve (I - dt_a L_v) x = rhs for every column (LAPACK dgesv)."""
    nz = rhs.shape[1]
    n = 3 * nz
    A = np.eye(n) - dt_a * Lm
    B = np.concatenate([rhs[0].reshape(nz, -1), rhs[3].reshape(nz, -1), rhs[4].reshape(nz, -1)])
    X = np.linalg.solve(A, B)
    out = rhs.copy()
    out[0] = X[:nz].reshape(rhs[0].shape)
    out[3] = X[nz:2 * nz].reshape(rhs[0].shape)
    out[4] = X[2 * nz:].reshape(rhs[0].shape)
    return out


def ark2_generic(S, L, solve, t, dt, q):
    """One ARK2 step for dq/dt = [S(q) - L(q)] + L(q) (Sec. 2.3): stage i
    solves (I - dt At_ii L) Q_i = q + dt sum_{j<i} [A_ij (S - L)(Q_j) + At_ij L(Q_j)];
    q^{n+1} = q + dt sum_j b_j S(Q_j) (b = bt).  S(t, Q), L(Q) and
    solve(dt_a, rhs) are callables."""
    A, At, b, c = hevi_coefficients()
    Q = [q]
    Sv, Lv = [], []
    for i in range(3):
        if i > 0:
            rhs = q.copy()
            for j in range(i):
                rhs = rhs + dt * (A[i, j] * (Sv[j] - Lv[j]) + At[i, j] * Lv[j])
            Q.append(solve(dt * At[i, i], rhs))
        Sv.append(S(t + c[i] * dt, Q[i]))
        Lv.append(L(Q[i]))
    out = q.copy()
    for j in range(3):
        out = out + dt * b[j] * Sv[j]
    return out


def l3_matrix(orc: Oracle):
    """Dense matrix of the oracle's 3D linear operator over all 5U unknowns
    (field-major lattice order), by applying it to unit vectors: for small
    meshes, where the implicit systems of the 3D-IMEX step are then solved
    directly."""
    n = 5 * orc.U
    Lm = np.zeros((n, n))
    e = np.zeros(n)
    for a in range(n):
        e[a] = 1.0
        Lm[:, a] = orc.l3_apply(e).reshape(-1)
        e[a] = 0.0
    return Lm


def imex3d_step(orc: Oracle, Lm, t, dt, q):
    """One 3D-IMEX ARK2 step (Sec. 2.3): explicit part S - L, implicit L over
    the whole mesh, every stage system (I - dt At_ii L) Q = rhs solved
    directly with the dense matrix Lm of l3_matrix.  Returns q^{n+1}."""
    q = np.asarray(q, dtype=np.float64).reshape((5,) + orc.shape)
    n = Lm.shape[0]

    def solve(a, rhs):
        return np.linalg.solve(np.eye(n) - a * Lm, rhs.reshape(-1)).reshape(rhs.shape)

    return ark2_generic(orc.rhs, orc.l3_apply, solve, t, dt, q)


def ark2_step(orc: Oracle, Lm, t, dt, q):
    """One HEVI ARK2 step on the mesh: explicit part S - L_v, implicit L_v,
    every column solved directly.  Returns q^{n+1}."""
    q = np.asarray(q, dtype=np.float64).reshape((5,) + orc.shape)
    return ark2_generic(orc.rhs, orc.lv_apply, lambda a, r: _solve_columns(Lm, a, r), t, dt, q)
