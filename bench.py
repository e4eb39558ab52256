"""Throughput of the APM nested-grid gravity solve on one MI355X.

A step is one forward solve of the whole hot path over the workload: owner grids,
TSC deposit of every level (tile binning + LDS-tiled deposit with FP64
accumulation), the FFT convolution of every grid with Fourier-space differencing,
level composition, TSC interpolation to every particle and the FP64 totals (mass,
energy, net force).
Workload (the hierarchy the metric is quoted on): root 128^3 plus two centred
nested 64^3 levels, 2^20 equal-mass Plummer particles (scale 0.05), no gas,
synthetic and seeded.

Prints one JSON line:  value = particles/s of the FP32 step (inputs resident in
HBM), with cells/s, the FP64 step, errors against the FP64 oracle, the roofline of
the dominant kernel (HIP events on the library stream, in a second pass of the
same steps) and the oracle timed on the host as the CPU baseline.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(plan, npart_level, esize):
    """Algorithmic HBM bytes per step of each kernel name (what the method must
    move at least once; c = complex bytes = 2 esize)."""
    c = 2 * esize
    b = {k: 0.0 for k in ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv",
                          "deposit_tiles", "deposit_finalize", "compose", "interp", "bin_count",
                          "bin_scatter")}
    for g in plan.grids:
        gx, gy, gz = g["gmf_n"]
        fx, fy, fz = g["fld_n"]
        Mx, My, Mz = g["fft_n"]
        W = Mx // 2 + 1
        oct_ = (Mx // 2 + 1) * (My // 2 + 1) * (Mz // 2 + 1)
        b["fft_x_fwd"] += gx * gy * gz * esize + gy * gz * W * c
        b["fft_y_fwd"] += gz * gy * W * c + gz * My * W * c
        b["fft_z_conv"] += gz * My * W * c + oct_ * c + 3 * fz * My * W * c
        b["fft_y_inv"] += 3 * fz * My * W * c + 4 * fz * fy * W * c
        b["fft_x_inv"] += 4 * fz * fy * W * c + fx * fy * fz * 4 * esize
        b["deposit_finalize"] += gx * gy * gz * (8 + esize)     # FP64 mass in, GMF out
        if g["level"] > 0:      # own field read and rewritten in place, parent at 1/8 density
            b["compose"] += fx * fy * fz * 4 * esize * (2 + 1 / 8)
    for n in npart_level:
        b["deposit_tiles"] += n * 4 * esize            # sorted (s_x, s_y, s_z, m) records
    n = npart_level[0]
    nl = len(plan.levels)
    b["bin_count"] = n * 3 * esize + nl * n * 8       # positions in once, key + rank per level
    b["bin_scatter"] = nl * n * (4 * esize + 8) + sum(npart_level) * (4 * esize + 4)
    b["interp"] = n * (3 * esize + 4 + 4 * esize)     # positions + owner in, a + Phi out
    return b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB a few times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": src.numel() * 4,
                          "launches": 5}))
        return

    import apm_workloads as W
    from paper_1410_0010_amd import Context, Plan

    w = W.workload_plummer_nested()
    plan = Plan(w.root_n, w.grids)
    ctx = Context(plan, 0)
    active = w.active_cells()
    log(f"workload {w.name}: {w.npart} particles, {len(w.grids)} grids, {active} active cells")

    def tens(dtype):
        return [torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to(dev)
                for a in (w.x, w.y, w.z, w.m)]

    tuned = {}

    def run(dtype, steps, warmup, profile=False):
        x, y, z, m = tens(dtype)
        n = w.npart
        out = [torch.empty(n, dtype=x.dtype, device=dev) for _ in range(4)]
        tot = None
        ctx.solve(x, y, z, m, None, *out)
        torch.cuda.synchronize()
        if x.dtype not in tuned:
            tuned[x.dtype] = ctx.autotune(x.dtype, reps=5)
        for _ in range(warmup):
            ctx.solve(x, y, z, m, None, *out)
            tot = ctx.solve_totals(m, *out)
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s0.record()
        for _ in range(steps):
            ctx.solve(x, y, z, m, None, *out)
            tot = ctx.solve_totals(m, *out)
        s1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = s0.elapsed_time(s1) / steps
        prof = None
        if profile:
            ctx.profile(False)
            prof = ctx.profile_read()
        acc = np.stack([o.cpu().numpy().astype(np.float64) for o in out[:3]], 1)
        return dict(ms=ms, wall_ms=1000 * wall / steps, totals=tot, acc=acc,
                    pot=out[3].cpu().numpy().astype(np.float64), prof=prof)

    log(f"FP32: warmup {args.warmup}, {args.steps} timed steps")
    r32 = run(np.float32, args.steps, args.warmup)
    log(f"FP32: {r32['ms']:.3f} ms/step")
    log("FP32: profiled pass (HIP events around every kernel)")
    p32 = run(np.float32, args.steps, 1, profile=True)
    r64 = None
    if not args.no_fp64:
        r64 = run(np.float64, args.steps, args.warmup)
        log(f"FP64: {r64['ms']:.3f} ms/step")

    # dominant kernel of the FP32 step and its roofline
    npl = []
    for l in range(plan.nlevels):
        # particles binned on level l: those whose cell lies in the level's binning box
        lo = np.array([min(g["gmf_lo"][a] for g in plan.level_grids(l)) - 1 for a in range(3)])
        hi = np.array([max(g["gmf_lo"][a] + g["gmf_n"][a] for g in plan.level_grids(l)) + 1
                       for a in range(3)])
        inv = 1.0 / plan.levels[l]["dx"]
        cx = np.floor(np.stack([w.x, w.y, w.z], 1) * inv)
        npl.append(int(np.all((cx >= lo) & (cx < hi), axis=1).sum()))
    kb = kernel_bytes(plan, npl, 4)
    steps = args.steps
    per_kernel = {k: dict(ms_per_step=v[0] / steps, launches_per_step=v[1] / steps)
                  for k, v in p32["prof"].items()}
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])
    dom_ms = per_kernel[dom]["ms_per_step"]
    dom_launch_ms = dom_ms / per_kernel[dom]["launches_per_step"]
    achieved = kb.get(dom, 0.0) / (dom_ms * 1e-3) / 1e9
    for k in per_kernel:
        if kb.get(k):
            per_kernel[k]["gbs"] = kb[k] / (per_kernel[k]["ms_per_step"] * 1e-3) / 1e9
    log("per-kernel (FP32): " + ", ".join(
        f"{k} {v['ms_per_step'] * 1e3:.1f}us" + (f" {v['gbs']:.0f}GB/s" if 'gbs' in v else "")
        for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]['ms_per_step'])))

    # errors against the FP64 oracle and the oracle's own time (CPU baseline)
    cpu = None
    err = {}
    if not args.no_cpu_baseline:
        from oracle import apm_oracle as O
        log("oracle: Green's functions (cached, as on the GPU), then one timed forward solve")
        op = O.OraclePlan(w.root_n, w.grids)
        cache = {g.index: O.greens(op, g) for g in op.grids}
        x32 = [a.astype(np.float32).astype(np.float64) for a in (w.x, w.y, w.z, w.m)]
        t0 = time.perf_counter()
        ref32 = O.solve(op, *x32, cache=cache)
        t_or = time.perf_counter() - t0
        log(f"oracle solve {t_or:.1f} s")
        own = ref32["owner"] >= 0
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        err["fp32_acc_rel_l2"] = rel(r32["acc"][own], ref32["acc"][own])
        err["fp32_pot_rel_l2"] = rel(r32["pot"][own], ref32["pot"][own])
        if r64 is not None:
            ref64 = O.solve(op, w.x, w.y, w.z, w.m, cache=cache)
            err["fp64_acc_rel_l2"] = rel(r64["acc"][own], ref64["acc"][own])
            err["fp64_pot_rel_l2"] = rel(r64["pot"][own], ref64["pot"][own])
        cpu = {"value": w.npart / t_or, "unit": "particles/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload, one forward solve (numpy FP64, single thread), "
                         "Green's functions precomputed as on the GPU",
               "seconds": t_or}

    value = w.npart / (r32["ms"] * 1e-3)
    line = {
        "metric": "particles/s per APM forward solve (+ cells/s, fp32 vs fp64, % HBM peak)",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer_nested: root 128^3 + 2 nested 64^3 levels, "
                               "2^20 Plummer particles (b=0.05), no gas",
                   "particles": w.npart, "active_cells": active, "grids": len(w.grids),
                   "fft": "256^3 root (doubled, isolated), 128^3 subgrids",
                   "gradient": "spectral"},
        "cells_per_s": active / (r32["ms"] * 1e-3),
        "fp64": None if r64 is None else {
            "particles_per_s": w.npart / (r64["ms"] * 1e-3),
            "cells_per_s": active / (r64["ms"] * 1e-3), "ms_per_step": r64["ms"]},
        "error_vs_fp64_oracle": err,
        "totals_fp32": {"mass_per_level": list(r32["totals"][:plan.nlevels]),
                        "energy": r32["totals"][plan.nlevels],
                        "net_force": list(r32["totals"][plan.nlevels + 1:])},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_ms": dom_launch_ms,
                     "algorithmic_bytes_per_step": kb.get(dom, 0.0),
                     "profiled_ms_per_step": p32["ms"]},
        "kernels_fp32": per_kernel,
        "launch": {"graph": "apm_solve captured once, replayed per step",
                   "autotuned_lines_per_block": {k: v["lines"] for d in tuned.values()
                                                 for k, v in d.items()}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
