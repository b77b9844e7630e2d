"""ctypes binding of libnhsem (include/nhsem.h): argument marshalling only.

Every function here forwards to the C ABI entry point of the same name;
device arrays are torch tensors on the GPU (their data pointers are passed),
streams are torch's current HIP stream.  All numerical work runs in the
gfx950 kernels of the library; nothing here computes on the CPU.  A missing
or unloadable library raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnhsem.so")

NH_OK = 0
NH_EINVAL = -1
NH_ESTATE = -2
NH_EHIP = -3
NH_ENOCONV = -4
NH_ENONFINITE = -5
NH_EUNSUPPORTED = -6
NH_ESPACE = -7
NH_FP64 = 0
NH_FP32_MIXED = 1
NH_DSS_SUM = 0
NH_DSS_MASS_AVG = 1

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class NHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nhsem error {code}: {msg}")
        self.code = code


class nh_mesh_desc(ctypes.Structure):
    _fields_ = [("nel", ctypes.c_int32 * 3), ("order", ctypes.c_int32),
                ("xe", _dp), ("ye", _dp), ("ze", _dp),
                ("periodic", ctypes.c_int32 * 2), ("precision", ctypes.c_int32)]


class nh_physics(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("g", "R", "cp", "cv", "p_a", "f", "sponge_z0", "sponge_tau")]


class nh_gmres_opts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_restarts", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("schur", ctypes.c_int32), ("precondition", ctypes.c_int32), ("guess_pick", ctypes.c_int32)]


class nh_solve_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("columns", "solves", "iters_total", "iters_max", "not_converged")]


# name -> (restype, argtypes); mirrors include/nhsem.h
_SIGS = {
    "nh_version": (ctypes.c_char_p, []),
    "nh_workspace_bytes": (ctypes.c_int32, [ctypes.POINTER(nh_mesh_desc), ctypes.POINTER(ctypes.c_size_t)]),
    "nh_init_mesh": (ctypes.c_int32, [ctypes.POINTER(nh_mesh_desc), ctypes.POINTER(nh_physics), _vp,
                                      ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "nh_set_stream": (ctypes.c_int32, [_vp, _vp]),
    "nh_set_precision": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "nh_set_tile": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "nh_tile_shape": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "nh_sizes": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int32)]),
    "nh_lattice_coords": (ctypes.c_int32, [_vp, _dp, _dp, _dp]),
    "nh_set_reference": (ctypes.c_int32, [_vp, _dp, _dp]),
    "nh_set_forcing": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, _dp, _vp]),
    "nh_set_state": (ctypes.c_int32, [_vp, _vp]),
    "nh_get_state": (ctypes.c_int32, [_vp, _vp]),
    "nh_state_ptr": (ctypes.c_int32, [_vp, ctypes.POINTER(_vp)]),
    "nh_rhs": (ctypes.c_int32, [_vp, ctypes.c_double, _vp, _vp]),
    "nh_rk_step": (ctypes.c_int32, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "nh_dss": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
    "nh_scatter": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp]),
    "nh_mass": (ctypes.c_int32, [_vp, _vp]),
    "nh_diagnostics": (ctypes.c_int32, [_vp, _dp]),
    "nh_check_finite": (ctypes.c_int32, [_vp]),
    "nh_hevi_workspace_bytes": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "nh_hevi_attach": (ctypes.c_int32, [_vp, _vp, ctypes.c_size_t]),
    "nh_lv_apply": (ctypes.c_int32, [_vp, _vp, _vp]),
    "nh_hevi_last_solves": (ctypes.c_int32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                             ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_double), _vp]),
    "nh_column_solve": (ctypes.c_int32, [_vp, ctypes.c_double, _vp, _vp, _vp, ctypes.POINTER(nh_gmres_opts),
                                         ctypes.POINTER(nh_solve_stats), _vp]),
    "nh_hevi_step": (ctypes.c_int32, [_vp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(nh_gmres_opts), _vp,
                                      ctypes.POINTER(nh_solve_stats)]),
    "nh_batch_workspace_bytes": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "nh_batch_create": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp,
                                         ctypes.POINTER(_vp)]),
    "nh_batch_step": (ctypes.c_int32, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "nh_batch_set_mode": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "nh_batch_last_error": (ctypes.c_int32, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "nh_batch_destroy": (ctypes.c_int32, [_vp]),
    "nh_mlp_workspace_bytes": (ctypes.c_int32, [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "nh_mlp_create": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_uint64, _vp, ctypes.c_size_t, _vp,
                                       ctypes.POINTER(_vp)]),
    "nh_mlp_forward": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp]),
    "nh_mlp_backward": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp]),
    "nh_mlp_train_step": (ctypes.c_int32, [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, ctypes.c_float, _vp]),
    "nh_mlp_adam_step": (ctypes.c_int32, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "nh_mlp_params": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "nh_mlp_set_params": (ctypes.c_int32, [_vp, _vp]),
    "nh_mlp_samples": (ctypes.c_int32, [_vp, _vp, ctypes.c_double, _vp, _vp, ctypes.c_int64, ctypes.c_int64,
                                        _vp, _vp, _vp, _vp, _vp]),
    "nh_mlp_guess": (ctypes.c_int32, [_vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
    "nh_mlp_set_passes": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "nh_mlp_set_decay": (ctypes.c_int32, [_vp, ctypes.c_float]),
    "nh_hyperdiffusion_workspace_bytes": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "nh_set_hyperdiffusion": (ctypes.c_int32, [_vp, _vp, ctypes.c_double, _vp, ctypes.c_size_t]),
    "nh_hyperdiffusion": (ctypes.c_int32, [_vp, _vp, _vp]),
    "nh_imex3d_workspace_bytes": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "nh_l3_apply": (ctypes.c_int32, [_vp, _vp, _vp]),
    "nh_global_solve": (ctypes.c_int32, [_vp, ctypes.c_double, _vp, _vp, _vp, ctypes.POINTER(nh_gmres_opts), _vp,
                                         ctypes.c_size_t, ctypes.POINTER(nh_solve_stats)]),
    "nh_imex3d_step": (ctypes.c_int32, [_vp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(nh_gmres_opts), _vp,
                                        ctypes.c_size_t, ctypes.POINTER(nh_solve_stats)]),
    "nh_ri_workspace_bytes": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "nh_ri_velocity": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp,
                                        _vp, _vp, ctypes.c_size_t]),
    "nh_ri_velocity_noalloc": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp,
                                                _vp, _vp, _vp]),
    "nh_mlp_last_error": (ctypes.c_int32, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "nh_mlp_destroy": (ctypes.c_int32, [_vp]),
    "nh_last_error": (ctypes.c_int32, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "nh_destroy": (ctypes.c_int32, [_vp]),
}

_lib = None


def load():
    """Load libnhsem.so (built in-tree).  torch is imported first so that the
    library binds to the same HIP runtime instance torch uses."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime shared with torch)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _err(ctx, code):
    buf = ctypes.create_string_buffer(512)
    load().nh_last_error(ctx, buf, 512)
    return NHError(code, buf.value.decode(errors="replace"))


def _check(ctx, code):
    if code != NH_OK:
        raise _err(ctx, code)


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _tptr(t):
    """Device address of a tensor (or a raw address given as int)."""
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_desc(mesh, precision=NH_FP64):
    xe = np.ascontiguousarray(mesh.xe, dtype=np.float64)
    ye = np.ascontiguousarray(mesh.ye, dtype=np.float64)
    ze = np.ascontiguousarray(mesh.ze, dtype=np.float64)
    d = nh_mesh_desc()
    d.nel[:] = [int(v) for v in mesh.nel]
    d.order = int(mesh.order)
    d.xe, d.ye, d.ze = _dptr(xe), _dptr(ye), _dptr(ze)
    d.periodic[:] = [1 if v else 0 for v in mesh.periodic]
    d.precision = int(precision)
    d._keep = (xe, ye, ze)
    return d


def make_physics(ph):
    p = nh_physics()
    for n in ("g", "R", "cp", "cv", "p_a", "f", "sponge_z0", "sponge_tau"):
        setattr(p, n, float(getattr(ph, n)))
    return p


# ------------------------------------------------------------- thin wrappers
def nh_version():
    return load().nh_version().decode()


def nh_workspace_bytes(desc):
    n = ctypes.c_size_t(0)
    _check(None, load().nh_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def nh_init_mesh(desc, phys, ws, stream=None):
    out = ctypes.c_void_p()
    code = load().nh_init_mesh(ctypes.byref(desc), ctypes.byref(phys), _tptr(ws), ws.numel(),
                               stream if stream is not None else _stream(), ctypes.byref(out))
    _check(None, code)
    return out


def nh_tile_shape(order, variant):
    tx = ctypes.c_int32(); ty = ctypes.c_int32()
    _check(None, load().nh_tile_shape(int(order), int(variant), ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


class Context:
    """Owns a workspace tensor and a library context for one mesh."""

    def __init__(self, mesh, phys, precision=NH_FP64, device="cuda"):
        import torch
        self.lib = load()
        self.mesh = mesh
        self.desc = make_desc(mesh, precision)
        self.phys_c = make_physics(phys)
        self.phys = phys
        nbytes = nh_workspace_bytes(self.desc)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.h = nh_init_mesh(self.desc, self.phys_c, self.ws)
        U = ctypes.c_int64(); L = ctypes.c_int64(); n = (ctypes.c_int32 * 3)()
        self._c(self.lib.nh_sizes(self.h, ctypes.byref(U), ctypes.byref(L), n))
        self.U, self.L = U.value, L.value
        self.nx, self.ny, self.nz = n[0], n[1], n[2]
        self._forcing = {}
        self.device = device

    def _c(self, code):
        _check(self.h, code)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def close(self):
        if getattr(self, "h", None):
            self.lib.nh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up
    def nh_set_stream(self, stream=None):
        self._c(self.lib.nh_set_stream(self.h, stream if stream is not None else _stream()))

    def nh_set_precision(self, precision):
        self._c(self.lib.nh_set_precision(self.h, int(precision)))

    def nh_set_tile(self, variant):
        self._c(self.lib.nh_set_tile(self.h, int(variant)))

    def nh_lattice_coords(self):
        x = np.zeros(self.nx); y = np.zeros(self.ny); z = np.zeros(self.nz)
        self._c(self.lib.nh_lattice_coords(self.h, _dptr(x), _dptr(y), _dptr(z)))
        return x, y, z

    def nh_set_reference(self, rho0_z, theta0_z):
        r = np.ascontiguousarray(rho0_z, dtype=np.float64)
        t = np.ascontiguousarray(theta0_z, dtype=np.float64)
        assert r.size == self.nz and t.size == self.nz
        self._c(self.lib.nh_set_reference(self.h, _dptr(r), _dptr(t)))

    def nh_set_forcing(self, field, t_snap, dev_snap):
        """dev_snap: device tensor [nsnap, U] (float64); kept alive here."""
        if dev_snap is None:
            self._c(self.lib.nh_set_forcing(self.h, int(field), 0, None, None))
            self._forcing.pop(field, None)
            return
        t = np.ascontiguousarray(np.atleast_1d(t_snap), dtype=np.float64)
        assert dev_snap.dtype.is_floating_point and dev_snap.numel() == t.size * self.U
        self._forcing[field] = (t, dev_snap)
        self._c(self.lib.nh_set_forcing(self.h, int(field), int(t.size), _dptr(t), _tptr(dev_snap)))

    def nh_set_state(self, q):
        assert q.is_contiguous() and q.numel() == 5 * self.U
        self._c(self.lib.nh_set_state(self.h, _tptr(q)))

    def nh_get_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty((5,) + self.shape, dtype=torch.float64, device=self.device)
        self._c(self.lib.nh_get_state(self.h, _tptr(out)))
        return out

    def nh_state_ptr(self):
        p = ctypes.c_void_p()
        self._c(self.lib.nh_state_ptr(self.h, ctypes.byref(p)))
        return p.value

    # -- hot path
    def nh_rhs(self, t, q, out=None):
        import torch
        if out is None:
            out = torch.empty_like(q)
        assert q.is_contiguous() and out.is_contiguous() and q.numel() == 5 * self.U
        self._c(self.lib.nh_rhs(self.h, float(t), _tptr(q), _tptr(out)))
        return out

    def nh_rk_step(self, t, dt, nsteps=1):
        self._c(self.lib.nh_rk_step(self.h, float(t), float(dt), int(nsteps)))

    def nh_dss(self, E, mode=NH_DSS_SUM, out=None):
        import torch
        nf = E.numel() // self.L
        if out is None:
            out = torch.empty((nf, self.U), dtype=torch.float64, device=E.device)
        self._c(self.lib.nh_dss(self.h, nf, int(mode), _tptr(E), _tptr(out)))
        return out

    def nh_scatter(self, Uv, out=None):
        import torch
        nf = Uv.numel() // self.U
        if out is None:
            out = torch.empty((nf, self.L), dtype=torch.float64, device=Uv.device)
        self._c(self.lib.nh_scatter(self.h, nf, _tptr(Uv), _tptr(out)))
        return out

    def nh_mass(self, out=None):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._c(self.lib.nh_mass(self.h, _tptr(out)))
        return out

    def nh_diagnostics(self):
        out = np.zeros(8)
        self._c(self.lib.nh_diagnostics(self.h, _dptr(out)))
        return out

    def nh_check_finite(self):
        return self.lib.nh_check_finite(self.h)

    # -- HEVI
    def nh_hevi_attach(self):
        import torch
        n = ctypes.c_size_t(0)
        self._c(self.lib.nh_hevi_workspace_bytes(self.h, ctypes.byref(n)))
        self.hws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._c(self.lib.nh_hevi_attach(self.h, _tptr(self.hws), n.value))

    def nh_set_hyperdiffusion(self, c, dt):
        """Enable the tensor hyper-diffusion term with coefficients c (3) and
        time step dt (c = None disables it)."""
        import torch
        if c is None:
            self._c(self.lib.nh_set_hyperdiffusion(self.h, None, 0.0, None, 0))
            return
        n = ctypes.c_size_t(0)
        self._c(self.lib.nh_hyperdiffusion_workspace_bytes(self.h, ctypes.byref(n)))
        self.hdws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        cc = (ctypes.c_double * 3)(*[float(v) for v in c])
        self._c(self.lib.nh_set_hyperdiffusion(self.h, cc, float(dt), _tptr(self.hdws), n.value))

    def nh_hyperdiffusion(self, q, out=None):
        import torch
        if out is None:
            out = torch.empty_like(q)
        self._c(self.lib.nh_hyperdiffusion(self.h, _tptr(q), _tptr(out)))
        return out

    def nh_ri_velocity(self, q, nstrips=50, rmax=None, center=None):
        """RI-velocity diagnostic of device state q: dict of device tensors
        center [2][n_z], ubar [n_z][nstrips], count [n_z][nstrips] and result
        [4] = (u_RI, its strip radius, its level height, max horizontal
        speed).  rmax defaults to half the smaller horizontal extent; center
        (a [2][n_z] device tensor) replaces the computed centroid."""
        import torch
        m = self.mesh
        if rmax is None:
            rmax = 0.5 * min(float(m.xe[-1]) - float(m.xe[0]), float(m.ye[-1]) - float(m.ye[0]))
        n = ctypes.c_size_t()
        self._c(self.lib.nh_ri_workspace_bytes(self.h, int(nstrips), ctypes.byref(n)))
        if getattr(self, "riws", None) is None or self.riws.numel() < n.value:
            self.riws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        nz = self.nz
        given = center is not None
        if given:
            if center.dtype != torch.float64 or not center.is_cuda or tuple(center.shape) != (2, nz):
                raise ValueError("center must be a float64 device tensor of shape (2, n_z)")
            cen = center.contiguous()
        else:
            cen = torch.empty((2, nz), dtype=torch.float64, device="cuda")
        ubar = torch.empty((nz, nstrips), dtype=torch.float64, device="cuda")
        count = torch.empty((nz, nstrips), dtype=torch.int32, device="cuda")
        res = torch.empty(4, dtype=torch.float64, device="cuda")
        self._c(self.lib.nh_ri_velocity(self.h, _tptr(q), int(nstrips), float(rmax), 1 if given else 0, _tptr(cen),
                                        _tptr(ubar), _tptr(count), _tptr(res), _tptr(self.riws), n.value))
        return {"center": cen, "ubar": ubar, "count": count, "result": res}

    def nh_ri_velocity_noalloc(self, q, nstrips=50, rmax=None, center=None, out=None):
        """nh_ri_velocity through the allocation-free entry point (partial sums
        in the library's fixed scratch).  out: optional dict of preallocated
        output tensors (center, ubar, count, result) as nh_ri_velocity returns."""
        import torch
        m = self.mesh
        if rmax is None:
            rmax = 0.5 * min(float(m.xe[-1]) - float(m.xe[0]), float(m.ye[-1]) - float(m.ye[0]))
        nz = self.nz
        given = center is not None
        if out is None:
            out = {"center": torch.empty((2, nz), dtype=torch.float64, device="cuda"),
                   "ubar": torch.empty((nz, nstrips), dtype=torch.float64, device="cuda"),
                   "count": torch.empty((nz, nstrips), dtype=torch.int32, device="cuda"),
                   "result": torch.empty(4, dtype=torch.float64, device="cuda")}
        if given:
            if center.dtype != torch.float64 or not center.is_cuda or tuple(center.shape) != (2, nz):
                raise ValueError("center must be a float64 device tensor of shape (2, n_z)")
            out["center"].copy_(center)
        self._c(self.lib.nh_ri_velocity_noalloc(self.h, _tptr(q), int(nstrips), float(rmax), 1 if given else 0,
                                                _tptr(out["center"]), _tptr(out["ubar"]), _tptr(out["count"]),
                                                _tptr(out["result"])))
        return out

    def nh_lv_apply(self, x, out=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        self._c(self.lib.nh_lv_apply(self.h, _tptr(x), _tptr(out)))
        return out

    def nh_column_solve(self, alpha, b, x0=None, out=None, restart=20, max_restarts=10, rtol=1e-10,
                        iters=None, check=True, schur=False, pick=False):
        import torch
        if out is None:
            out = torch.empty_like(b)
        opts = nh_gmres_opts(restart, max_restarts, rtol, int(bool(schur)), 0, int(bool(pick)))
        st = nh_solve_stats()
        code = self.lib.nh_column_solve(self.h, float(alpha), _tptr(b), _tptr(x0) if x0 is not None else None,
                                        _tptr(out), ctypes.byref(opts), ctypes.byref(st),
                                        _tptr(iters) if iters is not None else None)
        if check:
            self._c(code)
        return out, st

    def nh_hevi_step(self, t, dt, restart=20, max_restarts=10, rtol=1e-10, guess=None, check=True, schur=False,
                     pick=False):
        opts = nh_gmres_opts(restart, max_restarts, rtol, int(bool(schur)), 0, int(bool(pick)))
        st = nh_solve_stats()
        code = self.lib.nh_hevi_step(self.h, float(t), float(dt), ctypes.byref(opts),
                                     guess.h if guess is not None else None, ctypes.byref(st))
        if check:
            self._c(code)
        return st

    def _g3ws(self, restart):
        import torch
        n = ctypes.c_size_t()
        self._c(self.lib.nh_imex3d_workspace_bytes(self.h, int(restart), ctypes.byref(n)))
        if getattr(self, "g3ws", None) is None or self.g3ws.numel() < n.value:
            self.g3ws = None
            self.g3ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        return self.g3ws

    def nh_l3_apply(self, x, out=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        self._c(self.lib.nh_l3_apply(self.h, _tptr(x), _tptr(out)))
        return out

    def nh_global_solve(self, alpha, b, x0=None, out=None, restart=20, max_restarts=50, rtol=1e-10, check=True,
                        precondition=False):
        """(I - alpha L) x = b over the whole mesh (3D linear operator)."""
        import torch
        if out is None:
            out = torch.empty_like(b)
        ws = self._g3ws(restart)
        opts = nh_gmres_opts(restart, max_restarts, rtol, 0, int(bool(precondition)))
        st = nh_solve_stats()
        code = self.lib.nh_global_solve(self.h, float(alpha), _tptr(b), _tptr(x0) if x0 is not None else None,
                                        _tptr(out), ctypes.byref(opts), _tptr(ws), ws.numel(), ctypes.byref(st))
        if check:
            self._c(code)
        return out, st

    def nh_imex3d_step(self, t, dt, restart=20, max_restarts=50, rtol=1e-10, check=True, precondition=False):
        ws = self._g3ws(restart)
        opts = nh_gmres_opts(restart, max_restarts, rtol, 0, int(bool(precondition)))
        st = nh_solve_stats()
        code = self.lib.nh_imex3d_step(self.h, float(t), float(dt), ctypes.byref(opts), _tptr(ws), ws.numel(),
                                       ctypes.byref(st))
        if check:
            self._c(code)
        return st

    def nh_hevi_last_solves(self):
        """(alpha_per_dt, [(R2, X2), (R3, X3)]) as raw device addresses."""
        p = [ctypes.c_void_p() for _ in range(4)]
        a = ctypes.c_double()
        self._c(self.lib.nh_hevi_last_solves(self.h, *[ctypes.byref(v) for v in p], ctypes.byref(a), None))
        return a.value, [(p[0].value, p[1].value), (p[2].value, p[3].value)]

    def nh_last_error(self):
        buf = ctypes.create_string_buffer(512)
        self.lib.nh_last_error(self.h, buf, 512)
        return buf.value.decode(errors="replace")


MLP_IN, MLP_HID, MLP_OUT = 208, 256, 256


class ColumnMLP:
    """Owns a workspace tensor and a library MLP (FP16 MFMA forward, FP32
    backward, Adam)."""

    def __init__(self, max_batch=4096, seed=7, device="cuda"):
        import torch
        self.lib = load()
        n = ctypes.c_size_t(0)
        _check(None, self.lib.nh_mlp_workspace_bytes(int(max_batch), ctypes.byref(n)))
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(None, self.lib.nh_mlp_create(int(max_batch), int(seed), _tptr(self.ws), n.value, _stream(),
                                            ctypes.byref(h)))
        self.h = h
        self.max_batch = max_batch
        cnt = ctypes.c_int64()
        self._c(self.lib.nh_mlp_params(self.h, None, None, ctypes.byref(cnt)))
        self.nparam = cnt.value
        self.device = device

    def _c(self, code):
        if code != NH_OK:
            buf = ctypes.create_string_buffer(512)
            self.lib.nh_mlp_last_error(self.h, buf, 512)
            raise NHError(code, buf.value.decode(errors="replace"))

    def close(self):
        if getattr(self, "h", None):
            self.lib.nh_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nh_mlp_forward(self, x_f16, out=None):
        import torch
        B = x_f16.shape[0]
        if out is None:
            out = torch.empty((B, MLP_OUT), dtype=torch.float32, device=self.device)
        self._c(self.lib.nh_mlp_forward(self.h, B, _tptr(x_f16), _tptr(out)))
        return out

    def nh_mlp_backward(self, x_f16, dy):
        self._c(self.lib.nh_mlp_backward(self.h, x_f16.shape[0], _tptr(x_f16), _tptr(dy)))

    def nh_mlp_train_step(self, x_f16, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, loss=None):
        self._c(self.lib.nh_mlp_train_step(self.h, x_f16.shape[0], _tptr(x_f16), _tptr(t), lr, b1, b2, eps,
                                           _tptr(loss) if loss is not None else None))

    def nh_mlp_adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self._c(self.lib.nh_mlp_adam_step(self.h, lr, b1, b2, eps))

    def nh_mlp_params(self):
        import torch
        w = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        self._c(self.lib.nh_mlp_params(self.h, _tptr(w), _tptr(g), None))
        return w, g

    def nh_mlp_set_params(self, w):
        self._c(self.lib.nh_mlp_set_params(self.h, _tptr(w)))

    def nh_mlp_samples(self, ctx, alpha, b, x=None, col0=0, ncol=None, tmp=None, x0=None):
        """Features (FP16 [ncol][208]), scales and, with x, targets of columns:
        of the default start b, or of the start x0 ([3][U]) when given."""
        import torch
        ncol = ctx.nx * ctx.ny - col0 if ncol is None else ncol
        feat = torch.empty((ncol, MLP_IN), dtype=torch.float16, device=self.device)
        scale = torch.empty(ncol, dtype=torch.float64, device=self.device)
        tgt = torch.empty((ncol, MLP_OUT), dtype=torch.float32, device=self.device) if x is not None else None
        if tmp is None:
            tmp = torch.empty(5 * ctx.U, dtype=torch.float64, device=self.device)
        code = self.lib.nh_mlp_samples(self.h, ctx.h, float(alpha), _tptr(b), _tptr(x) if x is not None else None,
                                       int(col0), int(ncol), _tptr(feat), _tptr(scale),
                                       _tptr(tgt) if tgt is not None else None, _tptr(tmp),
                                       _tptr(x0) if x0 is not None else None)
        _check(ctx.h, code)
        return feat, scale, tgt

    def nh_mlp_set_decay(self, wd):
        self._c(self.lib.nh_mlp_set_decay(self.h, float(wd)))

    def nh_mlp_set_passes(self, passes):
        self._c(self.lib.nh_mlp_set_passes(self.h, int(passes)))

    def nh_mlp_guess(self, ctx, alpha, b, out=None, tmp=None):
        """Initial guess [3][U] (rho', w, theta') of the column solves for b [5][U]."""
        import torch
        if out is None:
            out = torch.empty(3 * ctx.U, dtype=torch.float64, device=self.device)
        if tmp is None:
            tmp = torch.empty(5 * ctx.U, dtype=torch.float64, device=self.device)
        _check(ctx.h, self.lib.nh_mlp_guess(self.h, ctx.h, float(alpha), _tptr(b), _tptr(tmp), _tptr(out)))
        return out


class Batch:
    """Batched SSP-RK3 over several Contexts, one graph per K steps."""

    def __init__(self, contexts, steps_per_graph=1, tile_variant=None, stream=None, persistent=False,
                 concurrent=False):
        import torch
        self.lib = load()
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c.h.value for c in self.contexts])
        self._arr = arr
        n = ctypes.c_size_t(0)
        _check(None, self.lib.nh_batch_workspace_bytes(arr, len(self.contexts), steps_per_graph, ctypes.byref(n)))
        self.ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        tv = None
        if tile_variant is not None:
            tv = (ctypes.c_int32 * 7)(*[int(tile_variant.get(k, 0)) for k in range(7)])
        h = ctypes.c_void_p()
        _check(None, self.lib.nh_batch_create(arr, len(self.contexts), steps_per_graph, tv, _tptr(self.ws),
                                              n.value, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.K = steps_per_graph
        if persistent or concurrent:
            self.nh_batch_set_mode(persistent, concurrent)

    def nh_batch_set_mode(self, persistent, concurrent):
        code = self.lib.nh_batch_set_mode(self.h, 1 if persistent else 0, 1 if concurrent else 0)
        if code != NH_OK:
            buf = ctypes.create_string_buffer(512)
            self.lib.nh_batch_last_error(self.h, buf, 512)
            raise NHError(code, buf.value.decode(errors="replace"))

    def nh_batch_step(self, t, dt, nsteps):
        code = self.lib.nh_batch_step(self.h, float(t), float(dt), int(nsteps))
        if code != NH_OK:
            buf = ctypes.create_string_buffer(512)
            self.lib.nh_batch_last_error(self.h, buf, 512)
            raise NHError(code, buf.value.decode(errors="replace"))

    def close(self):
        if getattr(self, "h", None):
            self.lib.nh_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
