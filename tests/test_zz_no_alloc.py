"""The allocation-free RI entry point (partial sums in the library's fixed
per-GPU scratch) against the workspace form, called through the C ABI:
two calls in a row, the second on a smaller lattice with fewer strips, and a
request beyond the scratch refused before anything is launched."""
import numpy as np
import pytest

from paper_2504_08157_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(nel, N, ext):
    from paper_2504_08157_amd import nhsem
    mesh = W.MeshSpec(nel, N, W.uniform_edges(0, ext[0], nel[0]), W.uniform_edges(0, ext[1], nel[1]),
                      W.uniform_edges(0, ext[2], nel[2]), (True, True))
    return nhsem.Context(mesh, W.Physics())


def _state(ctx, seed):
    import torch
    x, y, z = ctx.nh_lattice_coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    xc, yc = 0.45 * x[-1], 0.55 * y[-1]
    dx, dy = X - xc - 1e3 * Z / z[-1], Y - yc
    r = np.sqrt(dx * dx + dy * dy) + 1e-9
    rm = 0.1 * x[-1]
    V = 20.0 * (r / rm) * np.exp((1 - (r / rm) ** 2) / 2)
    rng = np.random.default_rng(seed)
    q = np.zeros((5,) + ctx.shape)
    q[1] = -V * dy / r + 0.3 * rng.normal(size=ctx.shape)
    q[2] = V * dx / r + 0.3 * rng.normal(size=ctx.shape)
    q[3] = 0.2 * rng.normal(size=ctx.shape)
    return torch.from_numpy(q).cuda()


def _same(a, b):
    assert np.array_equal(a["count"].cpu().numpy(), b["count"].cpu().numpy())
    for k in ("center", "ubar", "result"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.abs(x - y).max() <= 1e-12 * max(np.abs(y).max(), 1e-300), k


def test_noalloc_matches_workspace_form():
    import torch
    from paper_2504_08157_amd import nhsem
    big = _ctx((64, 64, 3), 4, (640e3, 640e3, 6e3))      # 256 x 256 x 13 lattice, 16 chunks per level
    small = _ctx((6, 5, 3), 4, (60e3, 50e3, 6e3))        # 24 x 20 x 13 lattice, one chunk
    qb, qs = _state(big, 1), _state(small, 2)
    got_b = big.nh_ri_velocity_noalloc(qb, nstrips=50)
    want_b = big.nh_ri_velocity(qb, nstrips=50)
    got_s = small.nh_ri_velocity_noalloc(qs, nstrips=20)
    want_s = small.nh_ri_velocity(qs, nstrips=20)
    torch.cuda.synchronize()
    _same(got_b, want_b)
    _same(got_s, want_s)
    assert int(got_b["count"].sum().item()) > 0 and int(got_s["count"].sum().item()) > 0
    # a given centre is used as given
    cen = want_s["center"].clone() + 100.0
    _same(small.nh_ri_velocity_noalloc(qs, nstrips=20, center=cen), small.nh_ri_velocity(qs, nstrips=20, center=cen))
    # beyond the scratch: refused, outputs untouched
    keep = {k: v.clone() for k, v in got_b.items()}
    out = {"center": got_b["center"], "ubar": torch.zeros((big.nz, 4096), dtype=torch.float64, device="cuda"),
           "count": torch.zeros((big.nz, 4096), dtype=torch.int32, device="cuda"), "result": got_b["result"]}
    with pytest.raises(nhsem.NHError) as e:
        big.nh_ri_velocity_noalloc(qb, nstrips=4096, out=out)
    assert e.value.code == nhsem.NH_ESPACE
    torch.cuda.synchronize()
    assert torch.equal(out["center"], keep["center"]) and torch.equal(out["result"], keep["result"])
    assert int(out["count"].abs().sum().item()) == 0
