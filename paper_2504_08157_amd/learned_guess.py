"""Learned initial guess for the HEVI column solves: data collection from
the method's own solves, on-device training with the library's MLP kernels,
and the with/without comparison on held-out steps.

Python only sequences library calls here; every arithmetic step (HEVI
stages, GMRES, features, forward, backward, Adam) runs in the gfx950
kernels of libnhsem.
"""
from __future__ import annotations

import time

import numpy as np

from . import nhsem
from . import workloads as W


def hevi_context(w, device="cuda"):
    import torch
    ctx = nhsem.Context(w.mesh, w.phys)
    x, y, z = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.reference_profiles(w, z))
    ctx.nh_hevi_attach()
    heat = W.heating(w, x, y, z)
    if heat is not None:
        t, Q = heat
        ctx._heat = torch.from_numpy(Q.reshape(len(t), -1)).to(device)
        ctx.nh_set_forcing(4, t, ctx._heat)
    ctx.nh_set_state(torch.from_numpy(W.initial_state(w, x, y, z)).to(device))
    return ctx


def collect(mlp, w, steps, dt, t0=0.0, rtol=1e-10, max_per_step=None, seed=8):
    """Run `steps` HEVI steps of workload w; after each, turn both implicit
    solves into (features, targets).  Returns FP16 features and FP32 targets
    (device tensors)."""
    import torch
    ctx = hevi_context(w)
    feats, tgts = [], []
    ncol = ctx.nx * ctx.ny
    rng = np.random.default_rng(seed)
    for s in range(steps):
        ctx.nh_hevi_step(t0 + s * dt, dt, rtol=rtol, max_restarts=30)
        a_dt, solves = ctx.nh_hevi_last_solves()
        for (R, X) in solves:
            f, _, t = mlp.nh_mlp_samples(ctx, a_dt * dt, R, X)
            if max_per_step and ncol > max_per_step:
                idx = torch.from_numpy(rng.choice(ncol, max_per_step, replace=False)).cuda()
                f, t = f[idx], t[idx]
            feats.append(f)
            tgts.append(t)
    torch.cuda.synchronize()
    ctx.close()
    return torch.cat(feats), torch.cat(tgts)


def train(mlp, feats, tgts, epochs=4, batch=4096, lr=1e-3, seed=8, log=None):
    """Adam over shuffled minibatches; returns the loss history (host)."""
    import torch
    n = feats.shape[0] // 64 * 64
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=feats.device)
    hist = []
    t0 = time.perf_counter()
    nseen = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(feats.shape[0])).to(feats.device)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            mlp.nh_mlp_train_step(feats[idx].contiguous(), tgts[idx].contiguous(), lr=lr, loss=loss)
            nseen += batch
        hist.append(loss.item())
        if log:
            log(f"epoch {ep} loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return hist, nseen / (time.perf_counter() - t0)


def compare(mlp, w, warm, held, dt, rtol=1e-10):
    """From the state after `warm` default steps, run `held` steps twice --
    default guess and MLP guess -- and report GMRES iterations, step times
    and the difference of the final states."""
    import torch
    ctx = hevi_context(w)
    for s in range(warm):
        ctx.nh_hevi_step(s * dt, dt, rtol=rtol, max_restarts=30)
    q0 = ctx.nh_get_state().clone()
    out = {}
    finals = {}
    for name, g in (("default", None), ("mlp", mlp)):
        ctx.nh_set_state(q0)
        torch.cuda.synchronize()
        it, ms = 0, 0.0
        mx = 0
        for s in range(held):
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st = ctx.nh_hevi_step((warm + s) * dt, dt, rtol=rtol, max_restarts=30, guess=g)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            it += st.iters_total
            mx = max(mx, st.iters_max)
        solves = held * 2 * ctx.nx * ctx.ny
        out[name] = {"iters_per_solve": it / solves, "iters_max": mx, "ms_per_step": ms / held}
        finals[name] = ctx.nh_get_state().cpu().numpy()
    d = finals["mlp"] - finals["default"]
    out["state_rel_diff"] = [float(np.linalg.norm(d[f]) / max(np.linalg.norm(finals["default"][f]), 1e-300))
                             for f in range(5)]
    out["columns"] = ctx.nx * ctx.ny
    ctx.close()
    return out
