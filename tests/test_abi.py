"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/nhsem.h, and rejects invalid descriptors before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2504_08157_amd import nhsem
from paper_2504_08157_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nhsem.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:nh_status|const char \*)\s*(nh_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol():
    lib = nhsem.load()
    decl = _declared()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(nhsem.exported_symbols()) == decl
    assert "gfx950" in nhsem.nh_version()


def _desc(**kw):
    m = W.cfg_bubble().mesh
    d = nhsem.make_desc(m)
    for k, v in kw.items():
        if k == "nel":
            d.nel[:] = v
        else:
            setattr(d, k, v)
    return d


def test_workspace_bytes_and_validation():
    d = _desc()
    n = nhsem.nh_workspace_bytes(d)
    U = 17 ** 3
    assert n >= 3 * 5 * U * 8
    for bad in (dict(order=1), dict(order=9), dict(nel=[0, 4, 4]), dict(precision=7)):
        with pytest.raises(nhsem.NHError) as e:
            nhsem.nh_workspace_bytes(_desc(**bad))
        assert e.value.code == nhsem.NH_EINVAL
    # non-increasing edges
    m = W.cfg_bubble().mesh
    m.xe = m.xe.copy(); m.xe[2] = m.xe[1]
    with pytest.raises(nhsem.NHError) as e:
        nhsem.nh_workspace_bytes(nhsem.make_desc(m))
    assert e.value.code == nhsem.NH_EINVAL


def test_init_rejects_before_device_work():
    lib = nhsem.load()
    d = _desc()
    ph = nhsem.make_physics(W.Physics())
    out = ctypes.c_void_p()
    # null workspace, misaligned workspace, too-small workspace: no device call is made
    assert lib.nh_init_mesh(ctypes.byref(d), ctypes.byref(ph), None, 1 << 30, None, ctypes.byref(out)) == nhsem.NH_EINVAL
    assert lib.nh_init_mesh(ctypes.byref(d), ctypes.byref(ph), ctypes.c_void_p(0x1001), 1 << 30, None,
                            ctypes.byref(out)) == nhsem.NH_EINVAL
    assert lib.nh_init_mesh(ctypes.byref(d), ctypes.byref(ph), ctypes.c_void_p(0x100000), 16, None,
                            ctypes.byref(out)) == nhsem.NH_ESPACE
    bad = nhsem.make_physics(W.Physics(cv=-1.0))
    assert lib.nh_init_mesh(ctypes.byref(d), ctypes.byref(bad), ctypes.c_void_p(0x100000), 1 << 40, None,
                            ctypes.byref(out)) == nhsem.NH_EINVAL
    assert out.value is None
    buf = ctypes.create_string_buffer(256)
    assert lib.nh_last_error(None, buf, 256) == 0 and b"physical" in buf.value
    # null context
    assert lib.nh_rk_step(None, 0.0, 1.0, 1) == nhsem.NH_EINVAL
