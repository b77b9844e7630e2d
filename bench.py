"""Throughput of the SSP-RK3 step on one MI355X, printed as one JSON line.

Workload: the per-GPU tropical-cyclone share, 128 x 128 x 20 elements of
order 4 (E = 327,680; U = 21,233,664 unique nodes), doubly periodic
1200 x 1200 x 20 km f-plane box, balanced warm-core vortex, heating bursts,
Rayleigh sponge, dt = 0.25 s.  A step is one SSP-RK3 step: three launches of
the fused RHS/DSS/RK stage kernel over the whole lattice, inputs resident in
HBM.  value = unique DOF-stage updates per second (5 U x 3 stages per step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per unique node and stage: read q^s (40 B), q^n (40 B in
# stages 2 and 3), both heating snapshots (16 B), write q^{s+1} (40 B)
BYTES_STAGE = {1: 40 + 16 + 40, 2: 40 + 40 + 16 + 40, 3: 40 + 40 + 16 + 40}


COUNTERS = os.path.join(ROOT, "profiles", "stage_kernel_tc_128x128x20_N4_fp64_counters.txt")
COUNTERS_FP32 = os.path.join(ROOT, "profiles", "stage_kernel_tc_128x128x20_N4_fp32_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2504_08157_amd", "csrc", "nh_kernels.hip")


HD_COUNTERS = os.path.join(ROOT, "profiles", "hd_laplace_tc_128x128x20_N4_hbm_counters.txt")
BAT_COUNTERS = os.path.join(ROOT, "profiles", "stage_kernel_batched_ensemble48_hbm_counters.txt")
HD_SRC = os.path.join(ROOT, "paper_2504_08157_amd", "csrc", "nh_hyper.hip")


RI_COUNTERS = os.path.join(ROOT, "profiles", "ri_velocity_tc_128x128x20_N4_hbm_counters.txt")
RI_SRC = os.path.join(ROOT, "paper_2504_08157_amd", "csrc", "nh_ri.hip")
L3_COUNTERS = os.path.join(ROOT, "profiles", "l3_apply_tc_hevi_96x96x16_N4_hbm_counters.txt")
L3_SRC = os.path.join(ROOT, "paper_2504_08157_amd", "csrc", "nh_imex3d.hip")


def measured_traffic(tile, counters=COUNTERS, src=KERNEL_SRC, key="traffic_bytes_per_launch"):
    """HBM bytes per launch (or call) from a committed FETCH_SIZE / WRITE_SIZE
    summary (copy-calibrated), or None when the kernel source (the sources
    hashed in order, for a tuple) or the stage tile differs from the profiled
    one."""
    import hashlib
    try:
        kv = {}
        for line in open(counters):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.split()[0]
        h = hashlib.sha256()
        for path in (src if isinstance(src, tuple) else (src,)):
            h.update(open(path, "rb").read())
        if kv.get("source_sha256") != h.hexdigest() or (tile is not None and int(kv.get("tile_variant", -1)) != tile):
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


GMRES_COUNTERS = os.path.join(ROOT, "profiles", "gmres_column_hevi_96x96x16_N4_counters.txt")
GMRES_SRC = os.path.join(ROOT, "paper_2504_08157_amd", "csrc", "nh_hevi.hip")
# MI355X vector FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz; a
# wave64 VALU instruction occupies its SIMD for 4 cycles
FP64_VALU_PEAK_TFLOPS = 78.6
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def gmres_counters(form):
    """Per column and Arnoldi step of the column GMRES kernel of `form`
    ("full" or "schur"): VALU wave instructions and executed FP64 flops from
    the committed SQ counter summary, or None when nh_hevi.hip differs from
    the profiled source."""
    import hashlib
    try:
        kv = {}
        for line in open(GMRES_COUNTERS):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.split()[0]
        if kv.get("source_sha256") != hashlib.sha256(open(GMRES_SRC, "rb").read()).hexdigest():
            return None
        return float(kv[f"{form}_valu_insts_per_column_step"]), float(kv[f"{form}_fp64_flops_per_column_step"])
    except (OSError, KeyError, ValueError):
        return None


def time_column_solves(ctx, w, reps, rtol=1e-10):
    """The two implicit solves of the last HEVI step of ctx, solved again by
    nh_column_solve in the full and the Schur form (default guess, GMRES(10),
    rtol): live time per solve (HIP events on the library's stream), Arnoldi
    steps, and the kernel's place under the FP64 VALU roof from the counter
    summary."""
    import torch
    a_dt, solves = ctx.nh_hevi_last_solves()
    out = {}
    xs = torch.empty(5 * ctx.U, dtype=torch.float64, device="cuda")
    for form, schur in (("full", False), ("schur", True)):
        ms, steps, n = 0.0, 0, 0
        for (R, _) in solves:
            ctx.nh_column_solve(a_dt * w.dt, R, out=xs, restart=10, max_restarts=30, rtol=rtol, schur=schur)
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                _, st = ctx.nh_column_solve(a_dt * w.dt, R, out=xs, restart=10, max_restarts=30, rtol=rtol,
                                            schur=schur)
                e1.record()
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
                steps += st.iters_total
                n += 1
        ncol = ctx.nx * ctx.ny
        rate = steps / (ms / 1e3)   # column Arnoldi steps per second
        r = {"ms_per_solve": ms / n, "arnoldi_steps_per_column": steps / n / ncol, "column_steps_per_s": rate,
             "column_steps_per_solve": steps / n}
        c = gmres_counters(form)
        if c is not None:
            insts, flops = c
            r["roofline"] = {"bound": "alu", "achieved": flops * rate / 1e12, "peak": FP64_VALU_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": flops * rate / 1e12 / FP64_VALU_PEAK_TFLOPS,
                             "valu_issue_frac": insts * rate / VALU_ISSUE_PEAK,
                             "valu_insts_per_column_step": insts, "fp64_flops_per_column_step": flops,
                             "note": "executed FP64 flops and VALU instructions per column step from the "
                                     "committed SQ counter summary; time and steps live"}
        else:
            r["roofline"] = None
        out[form] = r
    return out


def bench_gmres(args):
    """Column GMRES alone on the 96 x 96 x 16, N = 4 HEVI case: `warmup`
    default HEVI steps, then the two implicit solves of the last one solved
    again `steps` times each, in the full and the Schur form."""
    from paper_2504_08157_amd import learned_guess as LG
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_hevi()
    ctx = LG.hevi_context(w)
    for s in range(max(args.warmup, 1)):
        ctx.nh_hevi_step(s * w.dt, w.dt, rtol=1e-10, max_restarts=30, restart=10, schur=True)
    res = time_column_solves(ctx, w, max(args.steps, 1))
    ncol = ctx.nx * ctx.ny
    U = ctx.U
    ctx.close()
    f = res["schur"]
    line = {
        "metric": "column Arnoldi steps/s (column GMRES, FP64)", "value": f["column_steps_per_s"],
        "unit": "column Arnoldi steps/s", "n_gpus": 1, "steps": args.steps, "warmup": max(args.warmup, 1),
        "ms_per_step": f["ms_per_solve"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "mode": "gmres", "columns": ncol, "U": U,
                   "gmres": "GMRES(10), rtol 1e-10, default guess, the last HEVI step's two solves"},
        "roofline": f["roofline"], "gmres": res}
    print(json.dumps(line), flush=True)


# GEMM flops per sample of the column MLP (208 -> 256 -> 256 -> 256 with the
# 208 -> 256 bypass): forward W1, W2, W3, S; backward dH2, dH1 and the four
# weight gradients
MLP_FWD_FLOPS = 2 * (208 * 256 + 256 * 256 + 256 * 256 + 208 * 256)
MLP_BWD_FLOPS = 2 * (256 * 256 * 2 + 208 * 256 * 2 + 256 * 256 * 2)
MFMA_F16_PEAK_TFLOPS = 2500.0
MFMA_F32_PEAK_TFLOPS = 157.3


def bench_mlp(args):
    """The column MLP's training kernels alone on seeded synthetic features
    and targets (batch 1024 and 4096): forward GEMMs (FP16 MFMA), backward
    (FP32 MFMA GEMMs, bias sums, SiLU derivative) and whole training steps
    (forward, MSE gradient, backward, Adam), timed with HIP events."""
    import numpy as np
    import torch
    from paper_2504_08157_amd import nhsem
    rng = np.random.default_rng(17)
    res = {}
    for B in (1024, 4096):
        m = nhsem.ColumnMLP(max_batch=B, seed=7)
        x = torch.from_numpy(rng.normal(size=(B, nhsem.MLP_IN)).astype(np.float16)).cuda()
        t = torch.from_numpy(rng.normal(scale=0.1, size=(B, nhsem.MLP_OUT)).astype(np.float32)).cuda()
        dy = torch.from_numpy(rng.normal(scale=1e-4, size=(B, nhsem.MLP_OUT)).astype(np.float32)).cuda()
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")

        def timed(fn, n):
            for _ in range(max(args.warmup, 1)):
                fn()
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n

        n = max(args.steps, 10)
        fwd = timed(lambda: m.nh_mlp_forward(x), n)
        bwd = timed(lambda: m.nh_mlp_backward(x, dy), n)
        stp = timed(lambda: m.nh_mlp_train_step(x, t, lr=1e-4, loss=loss), n)
        af = MLP_FWD_FLOPS * B / (fwd / 1e3) / 1e12
        ab = MLP_BWD_FLOPS * B / (bwd / 1e3) / 1e12
        res[str(B)] = {"forward_ms": fwd, "backward_ms": bwd, "train_step_ms": stp,
                       "samples_per_s": B / (stp / 1e3),
                       "forward_tflops": af, "forward_frac_of_f16_mfma_peak": af / MFMA_F16_PEAK_TFLOPS,
                       "backward_tflops": ab, "backward_frac_of_f32_mfma_peak": ab / MFMA_F32_PEAK_TFLOPS}
        del m
    r = res["4096"]
    line = {"metric": "MLP training samples/s (column guess network)", "value": r["samples_per_s"],
            "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["train_step_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f16+f32", "data": "synthetic",
            "config": {"workload": "column MLP 208-256-256-256 with bypass", "mode": "mlp", "batch": 4096},
            "roofline": {"bound": "mfma", "achieved": r["backward_tflops"], "peak": MFMA_F32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": r["backward_frac_of_f32_mfma_peak"],
                         "kernel": "backward (FP32 MFMA GEMMs with their bias sums and SiLU derivative)",
                         "flops_per_sample": MLP_BWD_FLOPS},
            "mlp": res}
    print(json.dumps(line), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--workload", default="tc_large", choices=["tc_large", "tc_small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-nel", type=int, default=128, help="horizontal elements of the oracle sample box")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="minimum oracle time of the CPU baseline")
    ap.add_argument("--tile", type=int, default=-1, help="stage-kernel tile variant; -1 = tune by timing")
    ap.add_argument("--copy-mib", type=int, default=1024, help="buffer size of the copy calibration")
    ap.add_argument("--err-steps", type=int, default=600, help="steps of the FP32-vs-FP64 comparison (precision mode)")
    ap.add_argument("--mode", choices=["rk", "hevi", "batched", "copy", "precision", "hyper", "ri", "imex3d",
                                       "gmres", "mlp"],
                    default="rk",
                    help="rk: SSP-RK3 on the per-GPU TC share (headline); hevi: HEVI ARK2 step with and "
                         "without the learned GMRES guess; batched: 48 uneven instances in graph launches; "
                         "copy: a plain device-to-device copy of known size, the calibration run for the "
                         "HBM byte counters; precision: FP32-mixed vs FP64 after --err-steps steps; "
                         "hyper: the tensor hyper-diffusion term alone and the SSP-RK3 step with it; "
                         "ri: the RI-velocity diagnostic (centroids, 50-strip azimuthal means, u_RI); "
                         "imex3d: 3D-IMEX ARK2 steps (global GMRES) against HEVI and explicit RK3; "
                         "gmres: the column GMRES alone (full and Schur form) with its FP64 VALU roofline; "
                         "mlp: the column MLP's forward, backward and training step alone")
    ap.add_argument("--members", type=int, default=48)
    ap.add_argument("--imex-time", type=float, default=8.0, help="simulated seconds of the imex3d comparison")
    ap.add_argument("--mlp-epochs", type=int, default=100, help="training epochs of the column MLP (hevi mode)")
    ap.add_argument("--mlp-random-batches", type=int, default=96,
                    help="batches of random column right-hand sides in the MLP training data (hevi mode)")
    ap.add_argument("--mlp-finetune-epochs", type=int, default=120,
                    help="further epochs on the evaluated column grid's samples alone, batch 8192 (hevi mode)")
    ap.add_argument("--mlp-finetune-decay", type=float, default=3.0,
                    help="decoupled weight decay of the hidden path during the fine-tune epochs (hevi mode)")
    ap.add_argument("--mlp-refine-batches", type=int, default=32,
                    help="random batches of refinement-pass samples in the fine-tune set (hevi mode)")
    ap.add_argument("--mlp-passes", type=int, default=3,
                    help="network passes of the refined learned guess (hevi mode)")
    ap.add_argument("--gmres-restart", type=int, default=10, help="Krylov vectors per GMRES cycle (hevi mode)")
    return ap.parse_args()


def cpu_baseline(w, nel, min_seconds):
    """The FP64 oracle, untuned, on a bounded sample of the same workload:
    whole SSP-RK3 steps of a nel x nel x 20 element box with the same element
    size, physics and order (nel = 128: the workload itself), repeated until
    at least min_seconds of oracle time have passed."""
    import numpy as np
    import oracle
    from paper_2504_08157_amd import workloads as W
    oracle.build(force=False)
    half = 600.0e3 * nel / w.mesh.nel[0]
    mesh = W._tc_mesh(nel, nel, w.mesh.nel[2], w.mesh.order, half=half)
    sub = W.Workload(w.name, mesh, w.phys, w.dt, 1, w.reference, w.ic, vmax=w.vmax, heating_T=w.heating_T)
    orc = oracle.Oracle(mesh, w.phys)
    x, y, z = orc.lattice_coords()
    orc.set_reference(*W.reference_profiles(sub, z))
    t, Q = W.heating(sub, x, y, z)
    orc.set_forcing(4, t, Q)
    q = W.initial_state(sub, x, y, z)
    steps, sec = 0, 0.0
    while sec < min_seconds and steps < 1000:
        t0 = time.perf_counter()
        q = orc.rk3(steps * w.dt, w.dt, 1, q)
        sec += time.perf_counter() - t0
        steps += 1
    out = {"value": 5 * orc.U * 3 * steps / sec, "unit": "DOF-stage updates/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{steps} SSP-RK3 steps (3 RHS each) of a {nel}x{nel}x{mesh.nel[2]} element N={mesh.order} "
                     f"box of the same workload (U={orc.U}), {sec:.2f} s",
           "cpu_model": cpu_model()}
    del orc, q, Q
    # the same oracle on one host thread, on a smaller box of the same
    # workload (a whole step of the full box takes about half a minute there)
    n1 = max(8, nel // 4)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        mesh1 = W._tc_mesh(n1, n1, w.mesh.nel[2], w.mesh.order, half=600.0e3 * n1 / w.mesh.nel[0])
        sub1 = W.Workload(w.name, mesh1, w.phys, w.dt, 1, w.reference, w.ic, vmax=w.vmax, heating_T=w.heating_T)
        orc = oracle.Oracle(mesh1, w.phys)
        x, y, z = orc.lattice_coords()
        orc.set_reference(*W.reference_profiles(sub1, z))
        t, Q = W.heating(sub1, x, y, z)
        orc.set_forcing(4, t, Q)
        q = W.initial_state(sub1, x, y, z)
        steps1, sec1 = 0, 0.0
        while sec1 < min_seconds / 2 and steps1 < 1000:
            t0 = time.perf_counter()
            q = orc.rk3(steps1 * w.dt, w.dt, 1, q)
            sec1 += time.perf_counter() - t0
            steps1 += 1
    finally:
        oracle.set_num_threads(threads)
    out["value_1thread"] = 5 * orc.U * 3 * steps1 / sec1
    out["sample_1thread"] = (f"{steps1} SSP-RK3 steps of a {n1}x{n1}x{mesh1.nel[2]} element N={mesh1.order} box "
                             f"(U={orc.U}) on 1 thread, {sec1:.2f} s")
    return out


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def bench_hevi(args):
    """HEVI ARK2 steps on the 96 x 96 x 16, N = 4 case with the default GMRES
    guess and with the column MLP, both to rtol 1e-10.  The MLP is trained on
    solves the method generates: the small TC mesh and the bubble mesh, the
    `warmup` default steps of this case (the held-out steps that are timed
    come after them), and random column right-hand sides solved by the
    library's column GMRES on this vertical grid."""
    import numpy as np
    import torch
    from paper_2504_08157_amd import learned_guess as LG
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_hevi()
    mlp = nhsem.ColumnMLP(max_batch=32768, seed=7)
    warm = max(args.warmup, 1)
    wr = W.cfg_hevi()
    wr.mesh = W._tc_mesh(32, 32, w.mesh.nel[2])   # same column grid, 16384 columns per random batch
    tr = LG.fit(mlp, w, w.dt, warm, [(W.cfg_tc_small(), 2, w.dt), (W.cfg_bubble(), 2, 0.5)],
                epochs=args.mlp_epochs, batch=1024, lr=1e-3, max_per_step=24576, random_grid=wr,
                random_batches=args.mlp_random_batches, finetune_epochs=args.mlp_finetune_epochs,
                finetune_decay=args.mlp_finetune_decay, refine_random_batches=args.mlp_refine_batches,
                log=lambda m: print(m, file=sys.stderr, flush=True))
    res = LG.compare(mlp, w, warm=warm, held=args.steps, dt=w.dt, restart=args.gmres_restart,
                     refine_passes=args.mlp_passes)
    print("compared the full form", file=sys.stderr, flush=True)
    # the same steps with the column systems solved through their Schur
    # complement in w (restart 10 only)
    res_s = None
    if args.gmres_restart == 10:
        res_s = LG.compare(mlp, w, warm=warm, held=args.steps, dt=w.dt, restart=10, schur=True,
                           refine_passes=args.mlp_passes)
        print("compared the Schur form", file=sys.stderr, flush=True)
    ctx = LG.hevi_context(w)
    for s in range(warm):
        ctx.nh_hevi_step(s * w.dt, w.dt, rtol=1e-10, max_restarts=30, restart=10, schur=True)
    gm = time_column_solves(ctx, w, 3)
    U = ctx.U
    ctx.close()
    d, m, m2 = res["default"], res["mlp"], res["mlp_refined"]
    out = {
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        # the learned guess refined by further network passes (the form the speed-up is quoted for)
        "value": 5 * U * 3 / (m2["ms_per_step"] / 1e3), "unit": "DOF-stage updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": warm, "ms_per_step": m2["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f16", "data": "synthetic",
        "config": {"workload": w.name, "mode": "hevi", "dt": w.dt,
                   "gmres": f"GMRES({args.gmres_restart}), rtol 1e-10",
                   "columns": res["columns"]},
        "hevi": {"default": d, "mlp": m, "speedup_step": d["ms_per_step"] / m["ms_per_step"],
                 "iteration_ratio": m["iters_per_solve"] / d["iters_per_solve"],
                 "mlp_pick": res["mlp_pick"], "speedup_step_pick": d["ms_per_step"] / res["mlp_pick"]["ms_per_step"],
                 "iteration_ratio_pick": res["mlp_pick"]["iters_per_solve"] / d["iters_per_solve"],
                 "state_rel_diff_stacked_pick": res["state_rel_diff_stacked_pick"],
                 "refine_passes": args.mlp_passes,
                 "mlp_refined": res["mlp_refined"],
                 "speedup_step_refined": d["ms_per_step"] / res["mlp_refined"]["ms_per_step"],
                 "iteration_ratio_refined": res["mlp_refined"]["iters_per_solve"] / d["iters_per_solve"],
                 "state_rel_diff_stacked_refined": res["state_rel_diff_stacked_refined"],
                 "state_rel_diff_mlp_vs_default": res["state_rel_diff"],
                 "state_rel_diff_stacked": res["state_rel_diff_stacked"],
                 "training": tr},
        # the dominant kernel of the timed steps: the full-form column GMRES
        "roofline": gm["full"]["roofline"],
        "gmres": gm,
    }
    if res_s is not None:
        ds, ms = res_s["default"], res_s["mlp"]
        out["hevi"]["schur_form"] = {
            "default": ds, "mlp": ms, "speedup_step": ds["ms_per_step"] / ms["ms_per_step"],
            "iteration_ratio": ms["iters_per_solve"] / ds["iters_per_solve"],
            "mlp_pick": res_s["mlp_pick"], "speedup_step_pick": ds["ms_per_step"] / res_s["mlp_pick"]["ms_per_step"],
            "iteration_ratio_pick": res_s["mlp_pick"]["iters_per_solve"] / ds["iters_per_solve"],
            "mlp_refined": res_s["mlp_refined"],
            "speedup_step_refined": ds["ms_per_step"] / res_s["mlp_refined"]["ms_per_step"],
            "iteration_ratio_refined": res_s["mlp_refined"]["iters_per_solve"] / ds["iters_per_solve"],
            "state_rel_diff_stacked_refined": res_s["state_rel_diff_stacked_refined"],
            "state_rel_diff_stacked": res_s["state_rel_diff_stacked"],
            "speedup_vs_full_form_default": d["ms_per_step"] / ds["ms_per_step"],
            "state_rel_diff_vs_full_form": float(
                np.linalg.norm(res_s["final_default"] - res["final_default"]) / np.linalg.norm(res["final_default"])),
        }
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """48 uneven ensemble members (8x8x8 .. 40x40x16 elements, N in 3..5),
    SSP-RK3 dt = 0.25 s: the members stepped one by one, then batched graph
    launches.  Tile tuner: for each order, the members of that order alone
    are batched with each of the three tile variants and the fastest is kept
    (per order and precision).  Launch forms timed with the tuned table: one
    workgroup per item or persistent, order groups in step or concurrent."""
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    prec = nhsem.NH_FP64 if args.precision == "fp64" else nhsem.NH_FP32_MIXED
    ctxs, q0s = [], []
    for i in range(args.members):
        w = W.cfg_ensemble_member(i)
        c = nhsem.Context(w.mesh, w.phys, precision=prec)
        x, y, z = c.nh_lattice_coords()
        c.nh_set_reference(*W.reference_profiles(w, z))
        t, Q = W.heating(w, x, y, z)
        c._heat = torch.from_numpy(Q.reshape(len(t), -1)).cuda()
        c.nh_set_forcing(4, t, c._heat)
        q0 = torch.from_numpy(W.initial_state(w, x, y, z)).cuda()
        c.nh_set_state(q0)
        ctxs.append(c); q0s.append(q0)
    dt, K = 0.25, 5
    Utot = sum(c.U for c in ctxs)
    torch.cuda.synchronize()

    def reset():
        for c, q0 in zip(ctxs, q0s):
            c.nh_set_state(q0)
        torch.cuda.synchronize()

    # one by one
    for c in ctxs:
        c.nh_rk_step(0.0, dt, 2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for c in ctxs:
        c.nh_rk_step(0.0, dt, args.steps)
    e1.record(); torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / args.steps
    reset()
    s = torch.cuda.Stream()

    def time_batch(members, table, persistent, concurrent, nsteps):
        with torch.cuda.stream(s):
            b = nhsem.Batch(members, steps_per_graph=K, tile_variant=table, stream=s, persistent=persistent,
                            concurrent=concurrent)
            b.nh_batch_step(0.0, dt, K)
            a0 = torch.cuda.Event(enable_timing=True); a1 = torch.cuda.Event(enable_timing=True)
            a0.record(s); b.nh_batch_step(K * dt, dt, nsteps); a1.record(s)
        torch.cuda.synchronize()
        b.close()
        return a0.elapsed_time(a1) / nsteps

    # tile tuner per order (and this precision)
    orders = sorted({c.mesh.order for c in ctxs})
    tune, table = {}, {}
    for N in orders:
        members = [c for c in ctxs if c.mesh.order == N]
        tune[N] = {}
        for v in (0, 1, 2):
            tune[N][v] = time_batch(members, {N: v}, True, False, 2 * K)
            reset()
        table[N] = min(tune[N], key=tune[N].get)
    steps = (args.steps + K - 1) // K * K
    forms = {}
    for name, pers, conc in (("graph", False, False), ("persistent", True, False), ("concurrent", False, True),
                             ("persistent_concurrent", True, True)):
        forms[name] = time_batch(ctxs, table, pers, conc, steps)
        reset()
    best = min(forms, key=forms.get)
    ms_batch = forms[best]
    # the line's run: the fastest form once more, states checked afterwards
    ms_batch = time_batch(ctxs, table, best in ("persistent", "persistent_concurrent"),
                          best in ("concurrent", "persistent_concurrent"), steps)
    ok = all(c.nh_check_finite() == 0 for c in ctxs)
    # algorithmic bytes per step: q^s read and q^{s+1} written each stage (40 +
    # 40 B per node), q^n read in stages 2 and 3 (40 B), both heating
    # snapshots each stage (16 B): 96 + 136 + 136 = 368 B per node and step
    alg = 368.0 * Utot
    gbs = alg / (ms_batch * 1e-3) / 1e9
    # HBM bytes per step from the committed counter summary, when this run's
    # kernel source, precision, ensemble, tile table and (persistent) launch
    # form are the profiled ones
    traffic = None
    if prec == nhsem.NH_FP64 and len(ctxs) == 48 and best.startswith("persistent"):
        try:
            with open(BAT_COUNTERS) as fh:
                line = [l for l in fh if l.startswith("tile_table:")][0]
            prof = {int(a): int(b) for a, b in (kv.split("=") for kv in line.split(":", 1)[1].strip().split(","))}
            if prof == {int(k): int(v) for k, v in table.items()}:
                traffic = measured_traffic(None, BAT_COUNTERS, KERNEL_SRC, key="traffic_bytes_per_step")
        except (OSError, IndexError, ValueError):
            traffic = None
    out = {
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": 5 * Utot * 3 / (ms_batch / 1e3), "unit": "DOF-stage updates/s", "n_gpus": 1,
        "steps": steps, "warmup": K, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == 0 else "f32+f64", "data": "synthetic",
        "config": {"workload": "ensemble48_uneven", "mode": "batched", "members": len(ctxs), "unique_nodes": Utot,
                   "steps_per_graph": K, "tile_table": {str(k): v for k, v in table.items()},
                   "tile_ms_per_step_by_order": {str(N): {str(v): t for v, t in tune[N].items()} for N in orders},
                   "form": best, "ms_per_step_by_form": forms},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per step (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_step": alg,
                     "kernel": "all stage launches of one batched SSP-RK3 step (3 stages x order groups)"},
        "batched": {"ms_per_step_one_by_one": ms_single, "speedup_vs_one_by_one": ms_single / ms_batch,
                    "finite": ok},
    }
    print(json.dumps(out), flush=True)


def _tc_context(w, prec):
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    ctx = nhsem.Context(w.mesh, w.phys, precision=prec)
    x, y, z = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.reference_profiles(w, z))
    t_snap, Q = W.heating(w, x, y, z)
    ctx._heat = torch.from_numpy(Q.reshape(len(t_snap), -1)).cuda()
    del Q
    ctx.nh_set_forcing(4, t_snap, ctx._heat)
    q0 = torch.from_numpy(W.initial_state(w, x, y, z)).cuda()
    ctx.nh_set_state(q0)
    return ctx, q0


def bench_precision(args):
    """FP32-mixed (FP32 contractions and fluxes; FP64 EOS, reference
    subtraction, DSS, RK) against the FP64 path on the per-GPU TC share:
    per-field relative L2 difference after --err-steps SSP-RK3 steps from
    the same initial state, and the time per step of each."""
    import numpy as np
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_tc_large() if args.workload == "tc_large" else W.cfg_tc_small()
    out = {}
    states = {}
    for name, prec in (("fp64", nhsem.NH_FP64), ("fp32", nhsem.NH_FP32_MIXED)):
        ctx, q0 = _tc_context(w, prec)
        tune = {}
        if args.tile < 0:
            # tile tuner for this precision: a few steps per variant
            for v in (0, 1, 2):
                ctx.nh_set_tile(v)
                ctx.nh_rk_step(0.0, w.dt, 2)
                a0 = torch.cuda.Event(enable_timing=True); a1 = torch.cuda.Event(enable_timing=True)
                a0.record(); ctx.nh_rk_step(0.0, w.dt, 10); a1.record()
                torch.cuda.synchronize()
                tune[v] = a0.elapsed_time(a1) / 10
            ctx.nh_set_state(q0)
        tile = min(tune, key=tune.get) if tune else args.tile
        ctx.nh_set_tile(tile)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.nh_rk_step(0.0, w.dt, args.err_steps)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": e0.elapsed_time(e1) / args.err_steps, "tile_variant": tile,
                     "tile_ms_per_step": {str(k): v for k, v in tune.items()}}
        states[name] = ctx.nh_get_state().cpu().numpy()
        ctx.close()
        del ctx, q0
        torch.cuda.empty_cache()
    a, b = states["fp32"], states["fp64"]
    rel = [float(np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), 1e-300)) for f in range(5)]
    U = a[0].size
    ms = out["fp32"]["ms_per_step"]
    print(json.dumps({
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": 5 * U * 3 / (ms / 1e3), "unit": "DOF-stage updates/s", "n_gpus": 1,
        "steps": args.err_steps, "warmup": 0, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "mode": "precision", "dt": w.dt},
        "precision": {"fields": ["rho'", "u", "v", "w", "theta'"], "rel_l2_fp32_vs_fp64": rel,
                      "ms_per_step": out, "speedup_fp32_over_fp64": out["fp64"]["ms_per_step"] / ms,
                      "simulated_s": args.err_steps * w.dt},
    }), flush=True)


def bench_hyper(args):
    """Tensor hyper-diffusion on the per-GPU TC share: H_q alone (two
    launches of the directional weak-Laplacian kernel) and the SSP-RK3 step
    with H_q in every stage's tendency (per stage: the stage kernel, then
    one plain and one accumulating Laplacian launch), against the step
    without it.  Coefficients c = (1e-6, 1e-6, 2e-6): explicit-stable at
    dt = 0.25 s on these elements."""
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_tc_large() if args.workload == "tc_large" else W.cfg_tc_small()
    ctx, q0 = _tc_context(w, nhsem.NH_FP64)
    ctx.nh_set_tile(0 if args.tile < 0 else args.tile)
    c = (1e-6, 1e-6, 2e-6)
    ctx.nh_set_hyperdiffusion(c, w.dt)
    U = ctx.U
    H = ctx.nh_hyperdiffusion(q0)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()

    def timed(fn, n):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(s)
        for _ in range(n):
            fn()
        b.record(s)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    ms_hq = timed(lambda: ctx.nh_hyperdiffusion(q0, out=H), args.steps)
    ctx.nh_set_state(q0)
    ms_with = timed(lambda: ctx.nh_rk_step(0.0, w.dt, 1), args.steps)
    if ctx.nh_check_finite() != 0:
        raise RuntimeError("non-finite state after the steps with hyper-diffusion")
    ctx.nh_set_hyperdiffusion(None, 0.0)
    ctx.nh_set_state(q0)
    ms_without = timed(lambda: ctx.nh_rk_step(0.0, w.dt, 1), args.steps)
    # H_q: per unique node, each launch reads 5 and writes 5 doubles
    bytes_hq = 2 * 2 * 5 * 8 * U
    achieved = bytes_hq / (ms_hq / 1e3) / 1e9
    print(json.dumps({
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": 5 * U * 3 / (ms_with / 1e3), "unit": "DOF-stage updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_with, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "mode": "hyper", "dt": w.dt, "coefficients": list(c)},
        "hyperdiffusion": {"ms_hq": ms_hq, "ms_step_with": ms_with, "ms_step_without": ms_without,
                           "step_cost_ratio": ms_with / ms_without},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(None, HD_COUNTERS, HD_SRC) if w.name == "tc_128x128x20_N4" else None,
                     "traffic_unit": "HBM bytes per plain launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": bytes_hq / 2,
                     "kernel": "hd_laplace_tile_kernel (plain form, two launches per H_q)",
                     "avg_launch_ms": ms_hq / 2},
    }), flush=True)


def bench_ri(args):
    """RI-velocity diagnostic on the per-GPU TC share (the balanced vortex
    after --warmup SSP-RK3 steps): per-level centroids, 50-strip azimuthal
    means of the tangential speed, u_RI.  Algorithmic bytes per node: u, v, w
    read by the centroid pass and u, v by the strip pass (40 B).  The oracle
    computes the same diagnostic on the host for the cpu_baseline figure."""
    import numpy as np
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_tc_large() if args.workload == "tc_large" else W.cfg_tc_small()
    ctx, q0 = _tc_context(w, nhsem.NH_FP64)
    ctx.nh_set_tile(0 if args.tile < 0 else args.tile)
    ctx.nh_rk_step(0.0, w.dt, args.warmup)
    q = ctx.nh_get_state()
    U = ctx.U
    out = ctx.nh_ri_velocity(q, nstrips=50)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(args.steps):
        out = ctx.nh_ri_velocity(q, nstrips=50)
    b.record(s)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    res = out["result"].cpu().numpy().tolist()
    bytes_call = 40 * U
    achieved = bytes_call / (ms / 1e3) / 1e9
    line = {
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": U / (ms / 1e3), "unit": "nodes/s (RI diagnostic)", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "mode": "ri", "nstrips": 50, "rk_steps_before": args.warmup},
        "ri": {"u_ri": res[0], "r_ri": res[1], "z_ri": res[2], "u_max": res[3]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(None, RI_COUNTERS, RI_SRC, "traffic_bytes_per_call")
                     if w.name == "tc_128x128x20_N4" else None,
                     "traffic_unit": "HBM bytes per call (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_call": bytes_call,
                     "kernel": "RI diagnostic (centroid and strip passes with their final reductions)"},
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import ri_velocity as RI
        oracle.build(force=False)
        orc = oracle.Oracle(w.mesh, w.phys)
        qh = q.cpu().numpy()
        t0 = time.perf_counter()
        want = RI.ri_velocity(orc, qh, nstrips=50)
        sec = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": U / sec, "unit": "nodes/s (RI diagnostic)", "cores": 1, "kind": "oracle",
                                "sample": "the full diagnostic of the same state, NumPy on one host thread",
                                "u_ri_oracle": want["u_ri"]}
    print(json.dumps(line), flush=True)


def bench_imex3d(args):
    """3D-IMEX ARK2 (global GMRES(20) to rtol 1e-8 per stage, plain and
    right-preconditioned by the column solves) on the 96 x 96 x 16, N = 4
    HEVI case against HEVI ARK2 (column GMRES(10), Schur form, rtol 1e-10)
    and explicit SSP-RK3, each from the same state over the
    same --imex-time simulated seconds: ms per step, ms per simulated second,
    Krylov steps per solve, and the state error against an RK3 reference at
    dt = 0.125 s."""
    import numpy as np
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W
    w = W.cfg_hevi()
    ctx, q0 = _tc_context(w, nhsem.NH_FP64)
    ctx.nh_set_tile(0 if args.tile < 0 else args.tile)
    T = args.imex_time
    U = ctx.U
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def run(kind, dt):
        ctx.nh_set_state(q0)
        n = max(1, int(round(T / dt)))
        its = solves = missed = 0
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for k in range(n):
            if kind == "rk3":
                ctx.nh_rk_step(k * dt, dt, 1)
            elif kind == "hevi":
                st = ctx.nh_hevi_step(k * dt, dt, restart=10, max_restarts=20, rtol=1e-10, schur=True)
                its += st.iters_total; solves += st.solves * st.columns   # column solves
            else:
                st = ctx.nh_imex3d_step(k * dt, dt, restart=20, max_restarts=40, rtol=1e-8, check=False,
                                        precondition=kind == "imex3d_pc")
                its += st.iters_total; solves += st.solves; missed += st.not_converged
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        out = {"dt": dt, "steps": n, "ms_per_step": ms / n, "ms_per_simulated_s": ms / (n * dt)}
        if solves:
            out["krylov_steps_per_solve"] = its / solves
            out["solves_missing_rtol"] = missed
        return out, ctx.nh_get_state().cpu().numpy().reshape(5, -1)

    ctx.nh_hevi_attach()
    ref_info, ref = run("rk3", 0.125)
    res = {}
    runs = [("rk3", 0.25), ("hevi", 2.0)] + [(k, d) for k in ("imex3d", "imex3d_pc") for d in (2.0, 4.0, 8.0)
                                            if d <= T + 1e-9]
    for kind, dt in runs:
        info, qf = run(kind, dt)
        info["state_rel_err_vs_reference"] = [float(np.linalg.norm(qf[f] - ref[f]) / np.linalg.norm(ref[f]))
                                              for f in range(5)]
        res[f"{kind}_dt{dt:g}"] = info
    best = res[f"imex3d_pc_dt{runs[-1][1]:g}"]
    # roofline of one application of the 3D operator (one walk for the
    # horizontal and the vertical part): per node 5 fields read and 5 written
    # (80 B)
    xq = ctx.nh_get_state()
    yq = torch.empty_like(xq)
    for _ in range(3):
        ctx.nh_l3_apply(xq, yq)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for _ in range(20):
        ctx.nh_l3_apply(xq, yq)
    b.record()
    torch.cuda.synchronize()
    l3_ms = a.elapsed_time(b) / 20
    l3_bytes = 80 * U
    l3_gbs = l3_bytes / (l3_ms / 1e3) / 1e9
    print(json.dumps({
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": 5 * U * 3 / (best["ms_per_step"] / 1e3), "unit": "DOF-stage updates/s", "n_gpus": 1,
        "steps": best["steps"], "warmup": 0, "ms_per_step": best["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "mode": "imex3d", "simulated_s": T,
                   "gmres": "global GMRES(20), rtol 1e-8 per stage (imex3d_pc: flexible, column solves as right "
                            "preconditioner); HEVI: column GMRES(10) Schur form, rtol 1e-10"},
        "imex3d": res, "reference": {"kind": "rk3", **ref_info},
        "roofline": {"bound": "hbm", "achieved": l3_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": l3_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(None, L3_COUNTERS, L3_SRC, "traffic_bytes_per_call"),
                     "traffic_unit": "HBM bytes per call (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_call": l3_bytes,
                     "kernel": "application of the 3D operator (l3_tile_kernel: horizontal and vertical parts)",
                     "avg_call_ms": l3_ms},
    }), flush=True)


def bench_copy(args):
    """A plain device copy of args.copy_mib MiB, timed; under the FETCH_SIZE /
    WRITE_SIZE counters it gives the counter-to-byte factor of this GPU."""
    import torch
    n = args.copy_mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    nbytes = 2 * n * 8
    print(json.dumps({"metric": "copy_bandwidth", "value": nbytes / ms / 1e6, "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
                      "read_bytes": n * 8, "write_bytes": n * 8}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              f"a design, not built", file=sys.stderr)
        sys.exit(2)
    if args.mode == "hevi":
        return bench_hevi(args)
    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "copy":
        return bench_copy(args)
    if args.mode == "precision":
        return bench_precision(args)
    if args.mode == "hyper":
        return bench_hyper(args)
    if args.mode == "ri":
        return bench_ri(args)
    if args.mode == "imex3d":
        return bench_imex3d(args)
    if args.mode == "gmres":
        return bench_gmres(args)
    if args.mode == "mlp":
        return bench_mlp(args)
    import numpy as np
    import torch
    from paper_2504_08157_amd import nhsem
    from paper_2504_08157_amd import workloads as W

    w = W.cfg_tc_large() if args.workload == "tc_large" else W.cfg_tc_small()
    prec = nhsem.NH_FP64 if args.precision == "fp64" else nhsem.NH_FP32_MIXED
    ctx = nhsem.Context(w.mesh, w.phys, precision=prec)
    x, y, z = ctx.nh_lattice_coords()
    ctx.nh_set_reference(*W.reference_profiles(w, z))
    t_snap, Q = W.heating(w, x, y, z)
    Qd = torch.from_numpy(Q.reshape(len(t_snap), -1)).cuda()
    del Q
    ctx.nh_set_forcing(4, t_snap, Qd)
    q0 = torch.from_numpy(W.initial_state(w, x, y, z)).cuda()
    ctx.nh_set_state(q0)
    torch.cuda.synchronize()

    dt = w.dt
    tile = args.tile
    tune = {}
    if tile < 0:
        # tile autotuning: time each variant over a few steps, keep the fastest
        for v in (0, 1, 2):
            ctx.nh_set_tile(v)
            ctx.nh_rk_step(0.0, dt, 2)
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(); ctx.nh_rk_step(0.0, dt, 5); e1.record()
            torch.cuda.synchronize()
            tune[v] = e0.elapsed_time(e1) / 5
        tile = min(tune, key=tune.get)
        ctx.nh_set_state(q0)
    ctx.nh_set_tile(tile)
    ctx.nh_rk_step(0.0, dt, args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    ctx.nh_rk_step(args.warmup * dt, dt, args.steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(stop)
    if ctx.nh_check_finite() != 0:
        raise RuntimeError("non-finite state after the timed steps")

    U = ctx.U
    launches = 3 * args.steps
    ms_step = ms / args.steps
    value = 5 * U * 3 * args.steps / (ms / 1e3)
    bytes_step = U * sum(BYTES_STAGE.values())
    achieved = bytes_step * args.steps / (ms / 1e3) / 1e9
    traffic = (measured_traffic(tile, COUNTERS if prec == nhsem.NH_FP64 else COUNTERS_FP32)
               if w.name == "tc_128x128x20_N4" else None)
    res = {
        "metric": "DOF-stage updates/s (FP32/batched vs FP64 plain) at stated L2 error; % HBM peak",
        "value": value,
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == nhsem.NH_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "elements": list(w.mesh.nel), "order": w.mesh.order,
            "unique_nodes": U, "local_nodes": ctx.L,
            "dof_convention": "unique nodes x 5 fields; paper convention (E (N+1)^3 x 5) = "
                              f"{value * ctx.L / U:.4e}",
            "dt": dt, "precision": args.precision,
            "tile_variant": tile, "tile_columns": list(nhsem.nh_tile_shape(w.mesh.order, tile)),
            "tile_ms_per_step": {str(k): v for k, v in tune.items()},
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per stage launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": bytes_step / 3,
            "kernel": "stage_kernel (fused RHS + DSS + SSP-RK stage)",
            "avg_launch_ms": ms / launches,
        },
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_nel, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
