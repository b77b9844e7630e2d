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


def collect(mlp, w, steps, dt, t0=0.0, rtol=1e-10, max_per_step=None, seed=8, refine=False):
    """Run `steps` HEVI steps of workload w; after each, turn both implicit
    solves into (features, targets).  Returns FP16 features, FP32 targets
    (device tensors) and the implicit coefficient per dt of the solves.
    refine: samples of a refinement pass instead -- the start is the
    network's own first-pass guess, the features its residual and the
    targets the correction that remains."""
    import torch
    ctx = hevi_context(w)
    feats, tgts = [], []
    ncol = ctx.nx * ctx.ny
    rng = np.random.default_rng(seed)
    a_dt = None
    for s in range(steps):
        # the Schur form: the same solutions to the tolerance, in half the steps
        ctx.nh_hevi_step(t0 + s * dt, dt, rtol=rtol, max_restarts=30, restart=10, schur=True)
        a_dt, solves = ctx.nh_hevi_last_solves()
        for (R, X) in solves:
            x0 = mlp.nh_mlp_guess(ctx, a_dt * dt, R) if refine else None
            f, _, t = mlp.nh_mlp_samples(ctx, a_dt * dt, R, X, x0=x0)
            if max_per_step and ncol > max_per_step:
                idx = torch.from_numpy(rng.choice(ncol, max_per_step, replace=False)).cuda()
                f, t = f[idx], t[idx]
            feats.append(f)
            tgts.append(t)
    torch.cuda.synchronize()
    ctx.close()
    return torch.cat(feats), torch.cat(tgts), a_dt


def collect_random(mlp, w, batches, alpha, seed=11, rtol=1e-12, refine=False):
    """Solves of seeded random column right-hand sides on the column grid of
    workload w (the library's own batched GMRES, to rtol), turned into
    (features, targets): they span every direction of the column space,
    which the few structures of one simulation do not.  refine: samples of
    a refinement pass (see collect)."""
    import torch
    ctx = nhsem.Context(w.mesh, w.phys)
    x, y, z = ctx.nh_lattice_coords()
    rho0, th0 = W.reference_profiles(w, z)
    ctx.nh_set_reference(rho0, th0)
    ctx.nh_hevi_attach()
    # magnitudes of the random fields: reference density, a nominal sound
    # speed, reference potential temperature
    D = np.stack([rho0, np.full_like(rho0, 340.0), th0])
    ncol = ctx.nx * ctx.ny
    feats, tgts = [], []
    for k in range(batches):
        q = W.random_column_rhs(z, D, ncol, seed + k).reshape(5, -1)
        b = torch.from_numpy(np.ascontiguousarray(q)).cuda()
        xs, st = ctx.nh_column_solve(alpha, b, rtol=rtol, max_restarts=60, restart=10, schur=True)
        x0 = mlp.nh_mlp_guess(ctx, alpha, b) if refine else None
        f, _, t = mlp.nh_mlp_samples(ctx, alpha, b, xs, x0=x0)
        feats.append(f)
        tgts.append(t)
    torch.cuda.synchronize()
    ctx.close()
    return torch.cat(feats), torch.cat(tgts)


def train(mlp, feats, tgts, epochs=4, batch=4096, lr=1e-3, lr_final=None, seed=8, log=None, decay=0.0):
    """Adam over shuffled minibatches with a cosine learning-rate decay from
    lr to lr_final (default lr / 20), with decoupled weight decay `decay` on
    the hidden path (none on the bypass); returns the per-epoch loss history
    of the last minibatch (host) and the training rate in samples/s."""
    import math
    import torch
    n = feats.shape[0] // 64 * 64
    batch = min(batch, n)
    lr_final = lr / 20.0 if lr_final is None else lr_final
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=feats.device)
    hist = []
    per_epoch = max(1, (n - batch) // batch + 1)
    total = epochs * per_epoch
    t0 = time.perf_counter()
    nseen = 0
    step = 0
    mlp.nh_mlp_set_decay(decay)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(feats.shape[0])).to(feats.device)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / total))
            mlp.nh_mlp_train_step(feats[idx].contiguous(), tgts[idx].contiguous(), lr=a, loss=loss)
            nseen += batch
            step += 1
        hist.append(loss.item())
        if log:
            log(f"epoch {ep} loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    mlp.nh_mlp_set_decay(0.0)
    return hist, nseen / (time.perf_counter() - t0)


def initial_loss(feats, tgts):
    """Loss of the untrained network (zero output): mean of the targets squared."""
    return float((tgts.double() ** 2).mean().item())


def fit(mlp, w_eval, dt, warm, sources, epochs, batch=1024, lr=1e-3, max_per_step=None, random_grid=None,
        random_batches=0, finetune_epochs=0, finetune_batch=8192, finetune_lr=3e-4, finetune_lr_final=3e-6,
        finetune_decay=0.0, refine_random_batches=0, log=None):
    """Training set: the solves of `sources` (list of (workload, steps, dt))
    and of the first `warm` (>= 1) steps of w_eval, all generated by the
    method itself with the default guess, plus `random_batches` batches of
    random column solves on the column grid of `random_grid` (a workload with
    w_eval's vertical grid; default w_eval); then train on all of it, and
    for `finetune_epochs` more on the samples of w_eval's column grid alone
    (its own solves and the random ones) in large batches with a small
    learning rate and decoupled weight decay `finetune_decay` on the hidden
    path: the bypass can represent one grid's correction map exactly, and
    the other grids' samples pull it away from that map.  With
    refine_random_batches > 0 the fine-tune set also holds samples of a
    refinement pass (the network's own first-pass guess as the start) from
    the evaluated run's first steps and that many random batches, drawn
    after the first training phase.  log: a callable that receives progress
    lines.  Returns a summary dict."""
    import torch
    t0 = time.perf_counter()
    F, T = [], []
    for (ws, steps, dts) in sources:
        f, t, _ = collect(mlp, ws, steps=steps, dt=dts, max_per_step=max_per_step)
        F.append(f); T.append(t)
    f, t, a_dt = collect(mlp, w_eval, steps=max(warm, 1), dt=dt, max_per_step=max_per_step)
    F.append(f); T.append(t)
    n_sim = sum(int(x.shape[0]) for x in F)
    n_grid = len(F) - 1          # F[n_grid:] are samples of w_eval's column grid
    if random_batches > 0:
        f, t = collect_random(mlp, random_grid or w_eval, random_batches, a_dt * dt)
        F.append(f); T.append(t)
    feats, tgts = torch.cat(F), torch.cat(T)
    t_collect = time.perf_counter() - t0
    if log:
        log(f"collected {int(feats.shape[0])} samples in {t_collect:.1f} s")
    l0 = initial_loss(feats, tgts)
    hist, rate = train(mlp, feats, tgts, epochs=epochs, batch=batch, lr=lr, log=log)
    out = {"samples": int(feats.shape[0]), "samples_from_runs": n_sim, "loss_untrained": l0,
           "loss_last": hist[-1], "samples_per_s": rate, "collect_s": t_collect, "epochs": epochs,
           "batch": batch}
    del feats, tgts
    if finetune_epochs > 0:
        if refine_random_batches > 0:
            mlp.nh_mlp_set_passes(1)
            f, t, _ = collect(mlp, w_eval, steps=max(warm, 1), dt=dt, max_per_step=max_per_step, refine=True)
            F.append(f); T.append(t)
            f, t = collect_random(mlp, random_grid or w_eval, refine_random_batches, a_dt * dt, seed=911,
                                  refine=True)
            F.append(f); T.append(t)
            if log:
                log("collected the refinement-pass samples")
        fg, tg = torch.cat(F[n_grid:]), torch.cat(T[n_grid:])
        h2, rate2 = train(mlp, fg, tg, epochs=finetune_epochs, batch=finetune_batch, lr=finetune_lr,
                          lr_final=finetune_lr_final, decay=finetune_decay, log=log)
        out.update({"finetune_samples": int(fg.shape[0]), "finetune_epochs": finetune_epochs,
                    "finetune_decay": finetune_decay, "refine_random_batches": refine_random_batches,
                    "finetune_batch": finetune_batch, "finetune_loss_last": h2[-1],
                    "finetune_samples_per_s": rate2})
    return out


def compare(mlp, w, warm, held, dt, rtol=1e-10, restart=20, schur=False, refine_passes=2):
    """From the state after `warm` default steps, run `held` steps four
    times -- default guess, MLP guess, the MLP guess with the per-column
    choice against the default start (the smaller initial residual), and
    the MLP guess refined by further passes of the network on its own
    residual (refine_passes in all; reported as mlp_refined) -- and report
    GMRES iterations, step times and the difference of the final states
    (schur: solve the Schur complement in w)."""
    import torch
    ctx = hevi_context(w)
    for s in range(warm):
        ctx.nh_hevi_step(s * dt, dt, rtol=rtol, max_restarts=30, restart=restart, schur=schur)
    q0 = ctx.nh_get_state().clone()
    out = {}
    finals = {}
    for name, g, pick, passes in (("default", None, False, 1), ("mlp", mlp, False, 1), ("mlp_pick", mlp, True, 1),
                                  ("mlp_refined", mlp, False, refine_passes)):
        mlp.nh_mlp_set_passes(passes)
        ctx.nh_set_state(q0)
        torch.cuda.synchronize()
        it, ms = 0, 0.0
        mx = 0
        for s in range(held):
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st = ctx.nh_hevi_step((warm + s) * dt, dt, rtol=rtol, max_restarts=60, restart=restart, guess=g,
                                  schur=schur, pick=pick)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            it += st.iters_total
            mx = max(mx, st.iters_max)
        solves = held * 2 * ctx.nx * ctx.ny
        out[name] = {"iters_per_solve": it / solves, "iters_max": mx, "ms_per_step": ms / held}
        finals[name] = ctx.nh_get_state().cpu().numpy()
    mlp.nh_mlp_set_passes(1)
    dp = finals["mlp_pick"] - finals["default"]
    d2 = finals["mlp_refined"] - finals["default"]
    out["state_rel_diff_stacked_refined"] = float(np.linalg.norm(d2) / np.linalg.norm(finals["default"]))
    out["state_rel_diff_stacked_pick"] = float(np.linalg.norm(dp) / np.linalg.norm(finals["default"]))
    d = finals["mlp"] - finals["default"]
    out["state_rel_diff"] = [float(np.linalg.norm(d[f]) / max(np.linalg.norm(finals["default"][f]), 1e-300))
                             for f in range(5)]
    # in the norm the solver's tolerance is stated in (all fields stacked)
    out["state_rel_diff_stacked"] = float(np.linalg.norm(d) / np.linalg.norm(finals["default"]))
    out["columns"] = ctx.nx * ctx.ny
    out["final_default"] = finals["default"]   # for comparisons between solver forms
    ctx.close()
    return out
