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

    def nh_last_error(self):
        buf = ctypes.create_string_buffer(512)
        self.lib.nh_last_error(self.h, buf, 512)
        return buf.value.decode(errors="replace")
