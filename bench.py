"""Throughput of the APM nested-grid gravity solve on one MI355X.

A step is one pass of the whole hot path over the workload:
  forward  owner grids, TSC deposit of every level (tile binning + LDS-tiled
           deposit with FP64 accumulation), the FFT convolution of every grid with
           Fourier-space differencing, level composition, TSC interpolation to every
           particle, and the FP64 totals (mass per level, energy, net force);
  adjoint  the reverse sweep for the gradient of the potential energy W with respect
           to positions and masses (and gas), after the forward solve.
Workloads (synthetic and seeded, shaped like the paper's tests):
  plummer_nested  root 128^3 + 2 nested 64^3 levels, 2^20 Plummer particles
                  (b = 0.05), no gas -- the default and the headline line;
  root32_gas      single isolated root 32^3, 4096 particles + Gaussian gas blob;
  clumps          root 64^3 + 256 non-cubic level-1 grids (sides 8..48) on 256
                  Plummer clumps, 2^21 particles, lognormal masses;
  plummer_gas     root 256^3 + 2 nested 128^3 levels, 2^22 Plummer particles plus a
                  lognormal k^-2 random gas field (forward + adjoint);
  large_nested    root 512^3 + 3 nested 256^3 levels, 2^24 Plummer particles plus two
                  orbiting point masses; also 100 leapfrog steps and the energy drift;
  plummer_periodic  the plummer_nested geometry with a periodic root (root FFT 128^3,
                  not 256^3), 2^20 Plummer particles reaching the box edges;
  sine_wave       the sine wave test: periodic root 64^3 + levels over
                  [0.34375, 0.65625)^3 and [0.421875, 0.578125)^3, gas 2 + sin(2 pi x),
                  4096 massless tracer particles.

Prints one JSON line: value = particles/s of the FP32 forward step (inputs resident in
HBM), with cells/s, the forward+adjoint step, the FP64 steps, errors against the FP64
oracle, the roofline of the dominant kernel (HIP events on the library stream) and the
oracle timed on the host as the CPU baseline.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload plummer_nested]
                    [--no-cpu-baseline] [--no-fp64] [--no-adjoint]
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


def kernel_bytes(plan, npart, npart_level, esize, root_gas=False):
    """Algorithmic HBM bytes per step of each kernel name: what the method must move
    at least once (c = complex bytes = 2 esize)."""
    c = 2 * esize
    names = ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "deposit_tiles",
             "deposit_finalize", "compose", "interp", "unpack", "bin_count", "bin_scatter",
             "adj_fft_x",
             "adj_fft_y", "adj_fft_z", "adj_fft_y_inv", "adj_fft_x_inv", "adj_interp",
             "adj_deposit_grid", "adj_deposit_particles", "adj_restrict")
    b = {k: 0.0 for k in names}
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
        # the transposed passes move the same arrays in the other direction; their
        # field-box input is the FP64 cotangent
        b["adj_fft_x"] += fx * fy * fz * 4 * 8 + 4 * fz * fy * W * c
        b["adj_fft_y"] += 4 * fz * fy * W * c + 3 * fz * My * W * c
        b["adj_fft_z"] += 3 * fz * My * W * c + oct_ * c + gz * My * W * c
        b["adj_fft_y_inv"] += gz * My * W * c + gz * gy * W * c
        b["adj_fft_x_inv"] += gy * gz * W * c + gx * gy * gz * esize
        b["deposit_finalize"] += gx * gy * gz * (8 + esize)     # FP64 mass in, GMF out
        b["adj_deposit_grid"] += gx * gy * gz * (esize + 8)     # GMF cotangent in, FP64 out
        if g["level"] > 0:      # own field read and rewritten in place, parent at 1/8 density
            b["compose"] += fx * fy * fz * 4 * esize * (2 + 1 / 8)
            b["adj_restrict"] += fx * fy * fz * 4 * 8 * (1 + 2 / 8)
    binned = sum(npart_level)
    for nb in npart_level:
        b["deposit_tiles"] += nb * 4 * esize           # sorted (x/dx, y/dx, z/dx, m) records
        b["adj_deposit_particles"] += nb * (4 * esize + 8 + 4 * 8)
    nl = len(plan.levels)
    b["bin_count"] = npart * 3 * esize + nl * npart * 8      # positions once, key + rank per level
    b["bin_scatter"] = nl * npart * (4 * esize + 8) + binned * (4 * esize + 8)
    b["interp"] = binned * (4 * esize + 8) + npart * 4 * esize   # sorted records in, a + Phi out
    b["unpack"] = npart * (4 * esize + 4 + 4 * esize)   # (a, Phi) records + owner in, 4 arrays out
    if plan.cfg.boundary == 1:                          # periodic: the average density
        N = plan.grids[0]["n"][0]
        b["mean_density"] = npart * 4 * esize + (N ** 3 * esize if root_gas else 0)
    b["adj_interp"] = binned * (4 * esize + 8) + npart * (esize + 3 * 8)
    b["owner"] = npart * (3 * esize + 4)                # positions in, owner out
    b["totals"] = (sum(L["gmf_elems"] for L in plan.levels) * esize
                   + npart * (5 * esize + 4))           # GMFs, m, a, Phi, owner
    b["bin_clear"] = b["bin_scan"] = 0.0
    for l in range(nl):                                 # per level: tile counters, mass grid
        gs = plan.level_grids(l)
        kn = [max(g["gmf_lo"][a] + g["gmf_n"][a] for g in gs) + 1 -
              (min(g["gmf_lo"][a] for g in gs) - 1) for a in range(3)]
        ntiles = int(np.prod([(k + 7) // 8 for k in kn]))
        rep = 1
        while rep < 16 and ntiles * rep * 2 <= 1 << 18:
            rep *= 2
        b["bin_clear"] += (ntiles * rep + 1) * 4 + int(np.prod(kn)) * 8
        b["bin_scan"] += 2 * ntiles * rep * 4 + ntiles * 8   # counters in and out, items
    return b


def sine_wave_accuracy(Context, Plan, dev):
    """The sine wave test's accuracy (Sec. 3): per level, the largest deviation over the
    active cells of a_x and Phi from the continuum solution -4 pi (P / 2 pi)^2
    sin(2 pi x / P), relative to its amplitude, for P = 1 and 0.2: FP32 and FP64 with
    the spectral gradient, and FP64 with the two-point one (Sec. 2.2 names both)."""
    import torch
    import apm_workloads as W
    out = {}
    for P, grad, dt in [(P, g, d) for P in (1.0, 0.2)
                        for g, d in (("spectral", torch.float32), ("spectral", torch.float64),
                                     ("fd2", torch.float64))]:
        w = W.workload_sine_wave(period=P)
        plan = Plan(w.root_n, w.grids, boundary="periodic", gradient=grad)
        ctx = Context(plan, 0)
        k = 2 * np.pi / P
        amp_a, amp_p = 4 * np.pi / k, 4 * np.pi / k ** 2
        x, y, z, m = (torch.from_numpy(np.asarray(a, np.float64)).to(dev).to(dt)
                      for a in (w.x, w.y, w.z, w.m))
        gas = [ctx.pack_gas(l, w.gas, dt) for l in range(plan.nlevels)]
        ctx.solve(x, y, z, m, gas)
        torch.cuda.synchronize()
        lv = []
        for l in range(plan.nlevels):
            F = ctx.solved_field(l, dt)
            g = plan.level_grids(l)[0]
            f = ctx.field_view(F, g["index"]).cpu().numpy().astype(np.float64)
            a0 = [g["lo"][i] - g["fld_lo"][i] for i in range(3)]
            f = f[a0[2]:a0[2] + g["n"][2], a0[1]:a0[1] + g["n"][1], a0[0]:a0[0] + g["n"][0]]
            xc = (g["lo"][0] + np.arange(g["n"][0]) + 0.5) * g["dx"]
            ea = float(np.abs(f[..., 0] - amp_a * np.cos(k * xc)).max() / amp_a)
            ep = float(np.abs(f[..., 3] + amp_p * np.sin(k * xc)).max() / amp_p)
            lv.append({"level": l, "max_rel_err_ax": ea, "max_rel_err_phi": ep})
        out[f"P={P:g}/{grad}/{'f32' if dt == torch.float32 else 'f64'}"] = lv
    return out


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` (FP32) from the committed counter summary
    profiles/<kernel>_<workload>_fp32_counters.md: FETCH_SIZE and WRITE_SIZE per
    dispatch (KiB), each scaled by the factor a plain copy of known size gives.  None
    when there is no summary or it was taken on other native sources."""
    from paper_1410_0010_amd import profstats
    rec = profstats.traffic_record(
        os.path.join(ROOT, "profiles", f"{kernel}_{workload}_fp32_counters.md"))
    if not rec or rec.get("kernel") != kernel or rec.get("sources_sha256") != profstats.sources_sha256():
        return None
    return 1024.0 * (float(rec["fetch_kib"]) * float(rec["fetch_scale"]) +
                     float(rec["write_kib"]) * float(rec["write_scale"]))


WORKLOADS = {
    "plummer_nested": ("plummer_nested: root 128^3 + 2 nested 64^3 levels, 2^20 Plummer "
                       "particles (b=0.05), no gas"),
    "root32_gas": ("root32_gas: single isolated root 32^3, 4096 particles uniform in the "
                   "central half-box + Gaussian gas blob (sigma 0.1, mass 1)"),
    "clumps": ("clumps: root 64^3 + 256 level-1 grids, sides uniform in [8,48] per axis "
               "(non-cubic, centred on clumps, may overlap), 2^21 particles in 256 Plummer "
               "clumps (b=0.01), lognormal masses"),
    "plummer_gas": ("plummer_gas: root 256^3 + 2 nested 128^3 levels, 2^22 Plummer particles "
                    "(b=0.05) + lognormal k^-2 random gas field"),
    "large_nested": ("large_nested: root 512^3 (1024^3 padded FFT) + 3 nested 256^3 levels, "
                     "2^24 Plummer particles (b=0.02) + 2 orbiting point masses m=0.1"),
    "plummer_periodic": ("plummer_periodic: periodic root 128^3 (128^3 FFT) + 2 nested 64^3 "
                         "levels, 2^20 Plummer particles (b=0.05) over the whole box, no gas"),
    "sine_wave": ("sine_wave: the sine wave test, periodic root 64^3 + levels over "
                  "[0.34375,0.65625)^3 and [0.421875,0.578125)^3 (40^3 each), gas "
                  "2 + sin(2 pi x), 4096 massless tracers"),
}


def make_workload(name):
    import apm_workloads as W
    if name == "plummer_nested":
        return W.workload_plummer_nested()
    if name == "root32_gas":
        return W.workload_root32_uniform_gas()
    if name == "clumps":
        return W.workload_clumps()
    if name == "plummer_gas":
        return W.workload_plummer_gas()
    if name == "large_nested":
        return W.workload_large_nested()
    if name == "plummer_periodic":
        return W.workload_plummer_periodic()
    if name == "sine_wave":
        return W.workload_sine_wave()
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer_nested", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--leapfrog-steps", type=int, default=100,
                    help="KDK steps timed for large_nested (energy drift)")
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

    from paper_1410_0010_amd import Context, Plan

    w = make_workload(args.workload)
    plan = Plan(w.root_n, w.grids, boundary=w.boundary)
    ctx = Context(plan, 0)
    active = w.active_cells()
    n = w.npart
    log(f"workload {w.name}: {n} particles, {len(w.grids)} grids, {active} active cells")
    fp64_ok = not args.no_fp64 and args.workload != "large_nested"
    do_adj = not args.no_adjoint

    def tens(dtype):
        return [torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype))).to(dev)
                for a in (w.x, w.y, w.z, w.m)]

    def gas_for(tdt):
        g = [ctx.pack_gas(l, w.gas, tdt) for l in range(plan.nlevels)]
        return g if any(v is not None for v in g) else None

    tuned = {}

    def run(dtype, steps, warmup, adjoint=False, profile=False):
        x, y, z, m = tens(dtype)
        gas = gas_for(x.dtype)
        out = [torch.empty(n, dtype=x.dtype, device=dev) for _ in range(4)]
        tot_dev = torch.zeros(plan.nlevels + 5, dtype=torch.float64, device=dev)
        grads = None
        ctx.solve(x, y, z, m, gas, *out)
        torch.cuda.synchronize()
        if x.dtype not in tuned:
            tuned[x.dtype] = ctx.autotune(x.dtype, reps=5)

        def step():
            ctx.solve(x, y, z, m, gas, *out)
            tot = ctx.solve_totals(m, *out, gas=gas, out=tot_dev)    # stays on the GPU
            g = ctx.solve_adjoint(x, y, z, m, gas, out[3], wbar=1.0) if adjoint else None
            return tot, g

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s0.record()
        for _ in range(steps):
            tot, grads = step()
        s1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = s0.elapsed_time(s1) / steps
        prof = None
        if profile:
            ctx.profile(False)
            prof = ctx.profile_read()
        res = dict(ms=ms, wall_ms=1000 * wall / steps, totals=tot.cpu().numpy(), prof=prof,
                   acc=np.stack([o.cpu().numpy().astype(np.float64) for o in out[:3]], 1),
                   pot=out[3].cpu().numpy().astype(np.float64))
        if grads is not None:
            res["gx"] = np.stack([t.cpu().numpy().astype(np.float64) for t in grads[:3]], 1)
            res["gm"] = grads[3].cpu().numpy().astype(np.float64)
        return res

    log(f"FP32 forward: warmup {args.warmup}, {args.steps} timed steps")
    r32 = run(np.float32, args.steps, args.warmup)
    log(f"FP32 forward: {r32['ms']:.3f} ms/step")
    a32 = a64 = r64 = None
    if do_adj:
        a32 = run(np.float32, args.steps, 1, adjoint=True)
        log(f"FP32 forward+adjoint: {a32['ms']:.3f} ms/step")
    log("FP32: profiled pass (HIP events around every kernel)")
    psteps = max(3, args.steps // 4)
    p32 = run(np.float32, psteps, 1, adjoint=do_adj, profile=True)
    if fp64_ok:
        r64 = run(np.float64, args.steps, args.warmup)
        log(f"FP64 forward: {r64['ms']:.3f} ms/step")
        if do_adj:
            a64 = run(np.float64, args.steps, 1, adjoint=True)
            log(f"FP64 forward+adjoint: {a64['ms']:.3f} ms/step")

    # per-kernel times of the FP32 step, the dominant forward kernel and its roofline
    npl = []
    pos = np.stack([w.x, w.y, w.z], 1)
    for l in range(plan.nlevels):
        lo = np.array([min(g["gmf_lo"][a] for g in plan.level_grids(l)) - 1 for a in range(3)])
        hi = np.array([max(g["gmf_lo"][a] + g["gmf_n"][a] for g in plan.level_grids(l)) + 1
                       for a in range(3)])
        cx = np.floor(pos * (1.0 / plan.levels[l]["dx"]))
        inside = np.all((cx >= lo) & (cx < hi), axis=1) & np.all((pos >= 0) & (pos < 1), axis=1)
        npl.append(int(inside.sum()))
    kb = kernel_bytes(plan, n, npl, 4, root_gas=w.gas[0] is not None)
    per_kernel = {k: dict(ms_per_step=v[0] / psteps, launches_per_step=v[1] / psteps)
                  for k, v in p32["prof"].items()}
    forward_names = [k for k in per_kernel if not k.startswith("adj")]
    dom = max(forward_names, key=lambda k: per_kernel[k]["ms_per_step"])
    dom_ms = per_kernel[dom]["ms_per_step"]
    dom_launches = per_kernel[dom]["launches_per_step"]
    dom_launch_ms = dom_ms / dom_launches
    achieved = kb.get(dom, 0.0) / (dom_ms * 1e-3) / 1e9
    for k in per_kernel:
        if kb.get(k):
            per_kernel[k]["gbs"] = kb[k] / (per_kernel[k]["ms_per_step"] * 1e-3) / 1e9
    log("per-kernel (FP32): " + ", ".join(
        f"{k} {v['ms_per_step'] * 1e3:.1f}us" + (f" {v['gbs']:.0f}GB/s" if 'gbs' in v else "")
        for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]['ms_per_step'])))

    # leapfrog (large nested run): KDK steps, energy drift.  The two point masses'
    # self-energy (1/2 m Phi_self, Phi_self from a solve of the mass alone) depends on
    # the softening of the level they sit on, which halves when they cross into a
    # finer level; the drift is reported with and without that term, measured at 11
    # checkpoints (the run is timed as 10 segments of steps / 10).
    lf = None
    if args.workload == "large_nested" and args.leapfrog_steps > 0:
        x, y, z, m = tens(np.float32)
        vx, vy, vz = (torch.from_numpy(np.asarray(v, np.float32)).to(dev)
                      for v in (w.vx, w.vy, w.vz))
        r, b = 0.036, 0.02
        v = np.sqrt(r * (0.1 / (2 * r) ** 2 + r ** 3 / (r * r + b * b) ** 1.5 / r ** 2))
        h = 2 * np.pi * r / v / 400
        nst = args.leapfrog_steps
        nseg = 10 if nst % 10 == 0 else 1
        pot = torch.empty_like(x)
        x0, y0, z0 = x.clone(), y.clone(), z.clone()
        vx0, vy0, vz0 = vx.clone(), vy.clone(), vz.clone()
        ctx.leapfrog(x, y, z, vx, vy, vz, m, h, 1, pot=pot)      # warm-up and graph capture
        for a, b_ in ((x, x0), (y, y0), (z, z0), (vx, vx0), (vy, vy0), (vz, vz0)):
            a.copy_(b_)
        ctx_self = Context(plan, 0)

        def self_energy():
            e = 0.0
            for j in (n - 2, n - 1):
                _, _, _, ps = ctx_self.solve(x[j:j + 1], y[j:j + 1], z[j:j + 1], m[j:j + 1])
                e += 0.5 * float(w.m[j]) * float(ps.cpu()[0])
            return e

        energies, selfs = [], []
        sec = 0.0
        for seg in range(nseg):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, _, e = ctx.leapfrog(x, y, z, vx, vy, vz, m, h, nst // nseg, pot=pot)
            torch.cuda.synchronize()
            sec += time.perf_counter() - t0
            if seg == 0:
                energies.append(float(e[0]))
                xs = [t.clone() for t in (x, y, z)]
                # self-energy at the initial positions
                x.copy_(x0); y.copy_(y0); z.copy_(z0)
                selfs.append(self_energy())
                x.copy_(xs[0]); y.copy_(xs[1]); z.copy_(xs[2])
            energies.append(float(e[-1]))
            selfs.append(self_energy())
        E = np.array(energies)
        Ec = E - np.array(selfs)
        dev_ = lambda a: float(np.max(np.abs(a - a[0])) / abs(a[0]))
        lf = {"steps": nst, "dt": h, "seconds": sec, "ms_per_step": 1000 * sec / nst,
              "particle_steps_per_s": n * nst / sec, "energy_checkpoints": E.tolist(),
              "point_mass_self_energy": selfs,
              "energy_drift": float(abs(E[-1] - E[0]) / abs(E[0])),
              "energy_max_rel_dev": dev_(E),
              "energy_drift_excl_point_mass_self": float(abs(Ec[-1] - Ec[0]) / abs(Ec[0])),
              "energy_max_rel_dev_excl_point_mass_self": dev_(Ec)}
        log(f"leapfrog: {nst} steps, {lf['ms_per_step']:.2f} ms/step, energy drift "
            f"{lf['energy_drift']:.3e} (max {lf['energy_max_rel_dev']:.3e}); without the point "
            f"masses' self-energy {lf['energy_drift_excl_point_mass_self']:.3e} "
            f"(max {lf['energy_max_rel_dev_excl_point_mass_self']:.3e})")

    # errors against the FP64 oracle and the oracle's own time (CPU baseline)
    cpu = None
    err = {}
    if not args.no_cpu_baseline and args.workload in ("plummer_nested", "root32_gas",
                                                      "plummer_periodic", "sine_wave"):
        from oracle import apm_oracle as O
        from oracle import apm_adjoint as A
        log("oracle: Green's functions (cached, as on the GPU), then one timed forward solve "
            "and one timed reverse sweep")
        op = O.OraclePlan(w.root_n, w.grids, boundary=w.boundary)
        cache = {g.index: O.greens(op, g) for g in op.grids}
        rd = lambda a: None if a is None else np.asarray(a, np.float32).astype(np.float64)
        x32 = [rd(a) for a in (w.x, w.y, w.z, w.m)]
        g32 = [rd(a) for a in w.gas]
        t0 = time.perf_counter()
        ref32 = O.solve(op, *x32, g32, cache=cache)
        t_fwd = time.perf_counter() - t0
        t_adj = None
        if do_adj:
            t0 = time.perf_counter()
            adj32 = A.energy_gradient(op, *x32, g32, cache=cache, fwd=ref32)
            t_adj = time.perf_counter() - t0
        log(f"oracle forward {t_fwd:.1f} s" + (f", reverse sweep {t_adj:.1f} s" if t_adj else ""))
        own = ref32["owner"] >= 0
        def rel(a, b):
            nb = float(np.linalg.norm(b))
            return float(np.linalg.norm(a - b)) / nb if nb > 0 else None   # e.g. massless tracers
        err["fp32_acc_rel_l2"] = rel(r32["acc"][own], ref32["acc"][own])
        err["fp32_pot_rel_l2"] = rel(r32["pot"][own], ref32["pot"][own])
        if a32 is not None:
            err["fp32_grad_x_rel_l2"] = rel(a32["gx"], adj32["x"])
            err["fp32_grad_m_rel_l2"] = rel(a32["gm"], adj32["m"])
        if r64 is not None:
            x64 = [np.asarray(a, np.float64) for a in (w.x, w.y, w.z, w.m)]
            g64 = [None if a is None else np.asarray(a, np.float64) for a in w.gas]
            ref64 = O.solve(op, *x64, g64, cache=cache)
            err["fp64_acc_rel_l2"] = rel(r64["acc"][own], ref64["acc"][own])
            err["fp64_pot_rel_l2"] = rel(r64["pot"][own], ref64["pot"][own])
            if a64 is not None:
                adj64 = A.energy_gradient(op, *x64, g64, cache=cache, fwd=ref64)
                err["fp64_grad_x_rel_l2"] = rel(a64["gx"], adj64["x"])
                err["fp64_grad_m_rel_l2"] = rel(a64["gm"], adj64["m"])
        cpu = {"value": n / t_fwd, "unit": "particles/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload, one forward solve (numpy FP64, single thread), "
                         "Green's functions precomputed as on the GPU",
               "seconds": t_fwd}
        if t_adj is not None:
            cpu["fwd_adjoint"] = {"value": n / (t_fwd + t_adj), "unit": "particles/s",
                                  "seconds": t_fwd + t_adj}

    sw_acc = None
    if args.workload == "sine_wave":
        sw_acc = sine_wave_accuracy(Context, Plan, dev)
        log("sine wave vs the continuum solution: " + "; ".join(
            f"{k}: " + ", ".join(f"L{v['level']} {v['max_rel_err_ax']:.2e}" for v in lv)
            for k, lv in sw_acc.items()))

    value = n / (r32["ms"] * 1e-3)
    step_info = lambda r: None if r is None else {
        "particles_per_s": n / (r["ms"] * 1e-3), "cells_per_s": active / (r["ms"] * 1e-3),
        "ms_per_step": r["ms"]}
    line = {
        "metric": "particles/s per APM forward solve (+ cells/s, fwd+adjoint, fp32 vs fp64, "
                  "% HBM peak)",
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
        "config": {"workload": WORKLOADS[args.workload],
                   "particles": n, "active_cells": active, "grids": len(w.grids),
                   "fft_dims_first_grids": [g["fft_n"] for g in plan.grids[:4]],
                   "gradient": "spectral", "boundary": w.boundary},
        "cells_per_s": active / (r32["ms"] * 1e-3),
        "fwd_adjoint_fp32": step_info(a32),
        "fp64": step_info(r64),
        "fwd_adjoint_fp64": step_info(a64),
        "error_vs_fp64_oracle": err,
        "totals_fp32": {"mass_per_level": list(r32["totals"][:plan.nlevels]),
                        "energy": r32["totals"][plan.nlevels],
                        "net_force": list(r32["totals"][plan.nlevels + 1:plan.nlevels + 4])},
        "leapfrog_fp32": lf,
        "sine_wave_vs_analytic": sw_acc,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, args.workload),
                     "avg_launch_ms": dom_launch_ms,
                     "algorithmic_bytes_per_launch": kb.get(dom, 0.0) / dom_launches,
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
