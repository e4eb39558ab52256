"""Throughput of the APM nested-grid gravity solve on one MI355X.

A step is one pass of the whole hot path over the workload:
  forward  owner grids, TSC deposit of every level (tile binning + LDS-tiled
           deposit with FP64 accumulation), the FFT convolution of every grid with
           Fourier-space differencing, level composition, TSC interpolation to every
           particle, and the FP64 totals (mass per level, energy, net force);
  adjoint  the reverse sweep for the gradient of the potential energy W with respect
           to positions and masses (and gas), after the forward solve.
Workloads (synthetic and seeded, shaped like the paper's tests):
  large_nested    root 512^3 (1024^3 padded FFT) + 3 nested 256^3 levels, 2^24 Plummer
                  particles (b = 0.02) plus two orbiting point masses -- the default:
                  the largest configuration, on one GPU; also 100 leapfrog steps and
                  the energy drift;
  plummer_nested  root 128^3 + 2 nested 64^3 levels, 2^20 Plummer particles
                  (b = 0.05), no gas;
  root32_gas      single isolated root 32^3, 4096 particles + Gaussian gas blob;
  clumps          root 64^3 + 256 non-cubic level-1 grids (sides 8..48) on 256
                  Plummer clumps, 2^21 particles, lognormal masses;
  plummer_gas     root 256^3 + 2 nested 128^3 levels, 2^22 Plummer particles plus a
                  lognormal k^-2 random gas field (forward + adjoint);
  plummer_periodic  the plummer_nested geometry with a periodic root (root FFT 128^3,
                  not 256^3), 2^20 Plummer particles reaching the box edges;
  sine_wave       the sine wave test: periodic root 64^3 + levels over
                  [0.34375, 0.65625)^3 and [0.421875, 0.578125)^3, gas 2 + sin(2 pi x),
                  4096 massless tracer particles.

Prints one JSON line: value = particles/s of the FP32 forward step (inputs resident in
HBM), with cells/s, the forward+adjoint step, the FP64 steps, the staged per-level FP64
path, errors against the FP64 oracle, the roofline of the dominant kernel (HIP events
on the library stream) and the oracle timed on the host as the CPU baseline.

The oracle leg runs first, before the GPU is touched, in a pool of worker processes
(the unchanged oracle functions over particle chunks and kz-plane ranges).  On the
large workload it is staged (a full oracle solve of the 1024^3 root takes many
minutes): the GMF of every grid at sampled cells and the level masses, and the own
field of the finest grid (deposit, Green's function, 512^3 convolution) at sampled
cells; --oracle-full runs the whole oracle solve instead (every grid, composition,
every particle), for a one-off check.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--workload large_nested]
                    [--no-cpu-baseline] [--oracle-full] [--no-fp64] [--no-adjoint]
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------------------
# algorithmic bytes
# --------------------------------------------------------------------------------------

def pass_b_floor(plan, esize):
    """Bytes per step of the z pass (pass B) in a three-pass convolution (x-y planes,
    z columns with the multiply, y-x planes): read and write the gz My (Mx/2+1)
    complex intermediate once and read the (M/2+1)^3 kernel octant (one real per
    entry), summed over the grids."""
    b = 0.0
    for g in plan.grids:
        gz = g["gmf_n"][2]
        Mx, My, Mz = g["fft_n"]
        W = Mx // 2 + 1
        b += 2 * gz * My * W * 2 * esize + (Mx // 2 + 1) * (My // 2 + 1) * (Mz // 2 + 1) * esize
    return b


def conv_arrays(plan):
    """(z-pass output arrays, y-pass output arrays, kernel-table values per octant
    entry) of the library's transform passes for this plan: with the spectral gradient
    one kernel serves force and potential (two z arrays, three y arrays, one value),
    with the two-point gradient the potential has its own (three, four, a pair)."""
    return (3, 4, 2) if plan.cfg.gradient == 1 else (2, 3, 1)


def kernel_bytes(plan, npart, npart_level, esize, root_gas=False, pot_only_adjoint=True):
    """Algorithmic HBM bytes per step of each kernel name: what the method must move
    at least once with the arrays each pass reads and writes (c = complex bytes =
    2 esize).  The reverse sweep benchmarked is the gradient of W, whose transposed
    convolution carries the potential's cotangent alone (one FP64 value per field
    cell, one complex array per pass until the z pass)."""
    c = 2 * esize
    fs = 1 if pot_only_adjoint else 4
    names = ("fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv", "deposit_tiles",
             "deposit_finalize", "compose", "interp", "unpack", "sort", "tile_ranges",
             "adj_fft_x", "adj_fft_y", "adj_fft_z", "adj_fft_y_inv", "adj_fft_x_inv",
             "adj_interp", "adj_deposit_grid", "adj_deposit_particles", "adj_restrict",
             "adj_finish")
    b = {k: 0.0 for k in names}
    nz, ny, tv = conv_arrays(plan)
    for g in plan.grids:
        gx, gy, gz = g["gmf_n"]
        fx, fy, fz = g["fld_n"]
        Mx, My, Mz = g["fft_n"]
        W = Mx // 2 + 1
        oct_ = (Mx // 2 + 1) * (My // 2 + 1) * (Mz // 2 + 1)
        b["fft_x_fwd"] += gx * gy * gz * esize + gy * gz * W * c
        b["fft_y_fwd"] += gz * gy * W * c + gz * My * W * c
        b["fft_z_conv"] += gz * My * W * c + oct_ * tv * esize + nz * fz * My * W * c
        b["fft_y_inv"] += nz * fz * My * W * c + ny * fz * fy * W * c
        b["fft_x_inv"] += ny * fz * fy * W * c + fx * fy * fz * 4 * esize
        # the transposed passes move the same arrays in the other direction; their
        # field-box input is the FP64 cotangent (fs values per cell)
        b["adj_fft_x"] += fx * fy * fz * fs * 8 + fs * fz * fy * W * c
        b["adj_fft_y"] += fs * fz * fy * W * c + min(fs, 3) * fz * My * W * c
        b["adj_fft_z"] += (min(fs, 3) * fz * My * W * c + oct_ * tv * esize
                           + gz * My * W * c)
        b["adj_fft_y_inv"] += gz * My * W * c + gz * gy * W * c
        b["adj_fft_x_inv"] += gy * gz * W * c + gx * gy * gz * esize
        b["deposit_finalize"] += gx * gy * gz * (8 + esize)     # FP64 mass in, GMF out
        b["adj_deposit_grid"] += gx * gy * gz * (esize + 8)     # GMF cotangent in, FP64 out
        if g["level"] > 0:      # own field read and rewritten in place, parent at 1/8 density
            b["compose"] += fx * fy * fz * 4 * esize * (2 + 1 / 8)
            b["adj_restrict"] += fx * fy * fz * fs * 8 * (1 + 2 / 8)
    binned = sum(npart_level)
    for nb in npart_level:
        b["deposit_tiles"] += nb * 4 * esize           # sorted (x/dx, y/dx, z/dx, m) records
        b["adj_deposit_particles"] += nb * (4 * esize + 8 + 4 * 8)
    nl = len(plan.levels)
    # the particle sort: Morton bits of the finest level's 8^3 tiles, 8 a pass, keys of
    # 4 bytes below 32 bits; keys + indices read and written each pass, the digit
    # counts read with the keys; records packed, then gathered in sorted order
    nbits = 3 * max(0, int(round(np.log2(plan.grids[0]["n"][0] << (nl - 1)))) - 3)
    ks = 8 if nbits >= 32 else 4
    passes = (nbits + 8) // 8
    b["sort"] = (npart * (4 * esize) + npart * (ks + 4 + 4 * esize + 4)    # keys, owners, pack
                 + passes * npart * (ks + 2 * (ks + 4))                   # digit counts, scatter
                 + npart * (4 + 4 * esize + 4) + npart * (4 * esize + 8))  # gather
    b["tile_ranges"] = npart * ks
    b["interp"] = binned * (4 * esize + 8) + npart * 4 * esize   # sorted records in, a + Phi out
    b["unpack"] = npart * (4 * esize + 4 + 4 * esize)   # (a, Phi) records + owner in, 4 arrays out
    if plan.cfg.boundary == 1:                          # periodic: the average density
        N = plan.grids[0]["n"][0]
        b["mean_density"] = npart * 4 * esize + (N ** 3 * esize if root_gas else 0)
    b["adj_interp"] = binned * (4 * esize + 8) + npart * (esize + 3 * 8)
    # sorted reference and record, each level's and the interpolation's terms, the
    # potential, the record out; then the records and owners in, four arrays out
    b["adj_finish"] = (npart * (8 + 4 * esize + 4 * esize + esize + 4 * esize) + binned * 4 * esize
                       + npart * (4 * esize + 4 + 4 * esize))
    b["owner"] = npart * (3 * esize + 4)                # positions in, owner out
    b["totals"] = (sum(L["gmf_elems"] for L in plan.levels) * esize
                   + npart * (5 * esize + 4))           # GMFs, m, a, Phi, owner
    b["bin_clear"] = b["bin_scan"] = 0.0
    for l in range(nl):                                 # per level: tile runs, mass grid
        gs = plan.level_grids(l)
        klo = [min(g["gmf_lo"][a] for g in gs) - 1 for a in range(3)]
        khi = [max(g["gmf_lo"][a] + g["gmf_n"][a] for g in gs) for a in range(3)]   # inclusive
        ntiles = int(np.prod([khi[a] // 8 - klo[a] // 8 + 1 for a in range(3)]))
        b["bin_clear"] += ntiles * 8 + int(np.prod([khi[a] - klo[a] + 1 for a in range(3)])) * 8
        b["bin_scan"] += ntiles * 8 * 2 + ntiles * 4        # runs in (twice), item starts out
    return b


def floor_bytes(kernel, plan, npart_level, esize):
    """Floor bytes per step of a kernel family (the roofline's
    `achieved`): pass B for the z pass, 4 esize per binned particle + esize per GMF
    cell for the deposit, else None (the kernel's own algorithmic bytes are used)."""
    if kernel == "fft_z_conv":
        return pass_b_floor(plan, esize)
    if kernel == "deposit_tiles":
        return sum(npart_level) * 4 * esize + sum(L["gmf_elems"] for L in plan.levels) * esize
    return None


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


# --------------------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------------------

WORKLOADS = {
    "large_nested": ("large_nested: root 512^3 (1024^3 padded FFT) + 3 nested 256^3 levels, "
                     "2^24 Plummer particles (b=0.02) + 2 orbiting point masses m=0.1"),
    "plummer_nested": ("plummer_nested: root 128^3 + 2 nested 64^3 levels, 2^20 Plummer "
                       "particles (b=0.05), no gas"),
    "root32_gas": ("root32_gas: single isolated root 32^3, 4096 particles uniform in the "
                   "central half-box + Gaussian gas blob (sigma 0.1, mass 1)"),
    "clumps": ("clumps: root 64^3 + 256 level-1 grids, sides uniform in [8,48] per axis "
               "(non-cubic, centred on clumps, may overlap), 2^21 particles in 256 Plummer "
               "clumps (b=0.01), lognormal masses"),
    "plummer_gas": ("plummer_gas: root 256^3 + 2 nested 128^3 levels, 2^22 Plummer particles "
                    "(b=0.05) + lognormal k^-2 random gas field"),
    "plummer_periodic": ("plummer_periodic: periodic root 128^3 (128^3 FFT) + 2 nested 64^3 "
                         "levels, 2^20 Plummer particles (b=0.05) over the whole box, no gas"),
    "sine_wave": ("sine_wave: the sine wave test, periodic root 64^3 + levels over "
                  "[0.34375,0.65625)^3 and [0.421875,0.578125)^3 (40^3 each), gas "
                  "2 + sin(2 pi x), 4096 massless tracers"),
}

# the oracle solves these whole (in seconds to a minute); the others are staged
FULL_ORACLE = ("plummer_nested", "root32_gas", "plummer_periodic", "sine_wave")


def make_workload(name):
    import apm_workloads as W
    return {"plummer_nested": W.workload_plummer_nested, "root32_gas": W.workload_root32_uniform_gas,
            "clumps": W.workload_clumps, "plummer_gas": W.workload_plummer_gas,
            "large_nested": W.workload_large_nested,
            "plummer_periodic": W.workload_plummer_periodic,
            "sine_wave": W.workload_sine_wave}[name]()


# --------------------------------------------------------------------------------------
# the staged oracle on the host cores (worker processes forked before any GPU use)
# --------------------------------------------------------------------------------------

_OW = {}          # what forked workers read: plan, particles, James planes, fields


def _w_deposit(args):
    """Oracle deposit of particles [lo, hi) onto grid gi: the whole GMF array, or only
    its values at `idx` (flat) plus its sum."""
    from oracle import apm_oracle as O
    gi, lo, hi, idx = args
    plan, (x, y, z, m) = _OW["plan"], _OW["p"]
    rho = O.deposit_particles(plan, plan.grids[gi], x[lo:hi], y[lo:hi], z[lo:hi], m[lo:hi])
    if idx is None:
        return gi, rho, float(rho.sum())
    return gi, rho.reshape(-1)[idx], float(rho.sum())


def _w_greens(args):
    from oracle import apm_oracle as O
    gi, p0, p1 = args
    plan = _OW["plan"]
    g = plan.grids[gi]
    if g.level == 0 and not plan.periodic:
        return gi, p0, O.greens_root(plan, planes=(p0, p1), james=_OW["james"][p0:p1])
    return gi, p0, O.greens(plan, g, planes=(p0, p1))


def _w_interp(args):
    from oracle import apm_oracle as O
    lo, hi = args
    plan, (x, y, z, m) = _OW["plan"], _OW["p"]
    return lo, O.interp(plan, _OW["fields"], _OW["owner"][lo:hi], x[lo:hi], y[lo:hi], z[lo:hi])


def _pool(workers):
    return mp.get_context("fork").Pool(workers)


def _chunks(n, k):
    e = np.linspace(0, n, k + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(e[:-1], e[1:]) if b > a]


def _deposit_grids(plan, npart, grids, workers, samples):
    """GMF of each grid in `grids` (the whole array where samples[gi] is None, else the
    values at samples[gi]) and its sum, from particle chunks deposited in parallel."""
    def nchunks(gi):                    # whole arrays of a 512^3 root: fewer, larger chunks
        big = samples.get(gi) is None and np.prod(plan.grids[gi].gmf_n) > (1 << 26)
        return max(4, workers // 4) if big else workers
    tasks = [(gi, lo, hi, samples.get(gi)) for gi in grids for lo, hi in _chunks(npart, nchunks(gi))]
    out, tot = {}, {gi: 0.0 for gi in grids}
    with _pool(workers) as pool:
        for gi, v, s in pool.imap_unordered(_w_deposit, tasks):
            out[gi] = v if gi not in out else out[gi] + v
            tot[gi] += s
    return out, tot


def _greens_parallel(plan, gi, workers):
    g = plan.grids[gi]
    Mz = int(g.M[2])
    tasks = [(gi, a, b) for a, b in _chunks(Mz, 4 * workers)]
    parts = {}
    with _pool(workers) as pool:
        for _, p0, k in pool.imap_unordered(_w_greens, tasks):
            parts[p0] = k
    keys = sorted(parts)
    gf = np.concatenate([parts[k][0] for k in keys], axis=0)
    same = all(parts[k][0] is parts[k][1] for k in keys)
    gp = gf if same else np.concatenate([parts[k][1] for k in keys], axis=0)
    return gf, gp


def staged_oracle(w, full, workers, seed=1410):
    """The FP64 oracle on the FP32-rounded inputs of the workload, on `workers` host
    processes.  Staged (full = False): every grid's GMF (particles and gas) at 4096
    sampled cells and its mass; the finest grid's deposit, Green's function and
    convolution, its own field at 64 sampled field cells.  Full: the whole solve (every grid's GMF, own and composed
    field, owner grids, every particle's acceleration and potential)."""
    from oracle import apm_oracle as O
    rd = lambda a: np.asarray(a, np.float32).astype(np.float64)
    x, y, z, m = (rd(a) for a in (w.x, w.y, w.z, w.m))
    gas = [None if a is None else rd(a) for a in w.gas]
    plan = O.OraclePlan(w.root_n, w.grids)
    _OW.clear()
    _OW.update(plan=plan, p=(x, y, z, m))
    rng = np.random.default_rng(seed)
    res = {"mode": "full" if full else "staged", "workers": workers}
    t_all = time.perf_counter()
    fin = len(plan.grids) - 1
    if not full:
        samples = {g.index: rng.choice(int(np.prod(g.gmf_n)), min(4096, int(np.prod(g.gmf_n))),
                                       replace=False) for g in plan.grids}
        t0 = time.perf_counter()
        gmf, tot = _deposit_grids(plan, w.npart, [fin], workers, {})
        t_dep_fin = time.perf_counter() - t0
        rest, tot2 = _deposit_grids(plan, w.npart, list(range(fin)), workers, samples)
        tot.update(tot2)
        if any(a is not None for a in gas):             # own gas, the parent's on ghosts
            for gq in plan.grids:
                gp = O.add_gas(plan, gq, np.zeros(tuple(int(v) for v in gq.gmf_n[::-1])), gas)
                tot[gq.index] += float(gp.sum())
                if gq.index == fin:
                    gmf[fin] = gmf[fin] + gp
                else:
                    rest[gq.index] = rest[gq.index] + gp.reshape(-1)[samples[gq.index]]
        g = plan.grids[fin]
        rho = gmf[fin]
        res["gmf_samples"] = {gi: (samples[gi], rest[gi]) for gi in range(fin)}
        res["gmf_samples"][fin] = (samples[fin], rho.reshape(-1)[samples[fin]])
        log(f"oracle: GMFs ({t_dep_fin:.1f} s for the finest grid's deposit)")
        t0 = time.perf_counter()
        kern = _greens_parallel(plan, fin, workers)
        log(f"oracle: finest grid's Green's function {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        short = O.convolve(plan, g, rho, kern)
        t_conv = time.perf_counter() - t0
        cells = rng.choice(int(np.prod(g.fld_n)), min(64, int(np.prod(g.fld_n))), replace=False)
        res["own_samples"] = {fin: (cells, short.reshape(-1, 4)[cells])}
        res["mass"] = {gi: tot[gi] * plan.grids[gi].dx ** 3 for gi in tot}
        res["sample_seconds"] = t_dep_fin + t_conv
        res["sample_desc"] = (f"the forward solve of the finest grid alone: TSC deposit of all "
                              f"{w.npart} particles onto its GMF ({workers} processes) and its "
                              f"{'x'.join(str(int(v)) for v in g.M)} convolution (one core), "
                              f"Green's function precomputed as on the GPU")
        res["sample_cells"] = int(np.prod(g.n))
        log(f"oracle: finest grid's convolution {t_conv:.1f} s")
    else:
        if not plan.periodic:
            t0 = time.perf_counter()
            _OW["james"] = O.greens_root_james(plan)
            log(f"oracle: James root kernel {time.perf_counter() - t0:.1f} s")
        kerns = {}
        t0 = time.perf_counter()
        for g in plan.grids:
            kerns[g.index] = _greens_parallel(plan, g.index, workers)
        _OW.pop("james", None)
        log(f"oracle: Green's functions {time.perf_counter() - t0:.1f} s")
        t_solve = time.perf_counter()
        gmf, tot = _deposit_grids(plan, w.npart, [g.index for g in plan.grids], workers, {})
        for gq in plan.grids:
            if any(a is not None for a in gas):
                gp = O.add_gas(plan, gq, np.zeros(tuple(int(v) for v in gq.gmf_n[::-1])), gas)
                gmf[gq.index] = gmf[gq.index] + gp
                tot[gq.index] += float(gp.sum())
        log(f"oracle: deposits {time.perf_counter() - t_solve:.1f} s")
        short, fld = {}, {}
        for g in plan.grids:
            t0 = time.perf_counter()
            short[g.index] = O.convolve(plan, g, gmf[g.index], kerns.pop(g.index))
            log(f"oracle: convolution of grid {g.index} {time.perf_counter() - t0:.1f} s")
        for lev in range(plan.nlevels):
            for g in plan.level_grids(lev):
                fld[g.index] = O.compose(plan, g, short[g.index],
                                         fld[g.parent] if g.parent >= 0 else None)
        own = O.owner_of(plan, x, y, z)
        _OW.update(fields=[fld[g.index] for g in plan.grids], owner=own)
        pa = np.zeros((w.npart, 4))
        with _pool(workers) as pool:
            for lo, v in pool.imap_unordered(_w_interp, _chunks(w.npart, 4 * workers)):
                pa[lo:lo + v.shape[0]] = v
        res["solve_seconds"] = time.perf_counter() - t_solve
        res.update(gmf=gmf, short=short, field=fld, owner=own, acc=pa[:, :3], pot=pa[:, 3],
                   mass={gi: tot[gi] * plan.grids[gi].dx ** 3 for gi in tot})
        res["sample_seconds"] = res["solve_seconds"]
        res["sample_desc"] = (f"the whole forward solve ({workers} processes for deposits, "
                              f"Green's functions and interpolation; convolutions on one core), "
                              f"Green's functions precomputed as on the GPU")
        res["sample_cells"] = w.active_cells()
    _OW.clear()
    res["oracle_seconds"] = time.perf_counter() - t_all
    return res


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else None


def staged_errors(ref, got, plan_grids):
    """Errors of GPU outputs against the staged oracle results (relative L2 over the
    compared values)."""
    e = {}
    for gi, (idx, vals) in ref.get("gmf_samples", {}).items():
        e[f"gmf_grid{gi}_sampled"] = rel(got["gmf"][gi].reshape(-1)[idx], vals)
    for gi, (cells, vals) in ref.get("own_samples", {}).items():
        f = got["own"][gi].reshape(-1, 4)[cells]
        e[f"own_acc_grid{gi}_sampled"] = rel(f[:, :3], vals[:, :3])
        e[f"own_pot_grid{gi}_sampled"] = rel(f[:, 3], vals[:, 3])
    if "field" in ref:
        for gi in ref["field"]:
            e[f"gmf_grid{gi}"] = rel(got["gmf"][gi], ref["gmf"][gi])
            e[f"own_acc_grid{gi}"] = rel(got["own"][gi][..., :3], ref["short"][gi][..., :3])
            e[f"own_pot_grid{gi}"] = rel(got["own"][gi][..., 3], ref["short"][gi][..., 3])
            e[f"field_acc_grid{gi}"] = rel(got["field"][gi][..., :3], ref["field"][gi][..., :3])
            e[f"field_pot_grid{gi}"] = rel(got["field"][gi][..., 3], ref["field"][gi][..., 3])
        own = ref["owner"] >= 0
        e["owner_mismatches"] = int(np.sum(got["owner"] != ref["owner"]))
        e["acc_rel_l2"] = rel(got["acc"][own], ref["acc"][own])
        e["pot_rel_l2"] = rel(got["pot"][own], ref["pot"][own])
    lev_mass = {}
    for gi, mref in ref["mass"].items():
        lev = plan_grids[gi]["level"]
        lev_mass[lev] = lev_mass.get(lev, 0.0) + mref
    for lev, mref in sorted(lev_mass.items()):
        e[f"mass_level{lev}_rel"] = abs(got["mass"][lev] - mref) / abs(mref)
    return e


# --------------------------------------------------------------------------------------
# main
# --------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_nested", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-full", action="store_true",
                    help="large workloads: run the whole oracle solve (many minutes) instead "
                         "of the staged one")
    ap.add_argument("--oracle-workers", type=int, default=0,
                    help="host processes of the oracle leg (0: the CPUs this process may use, "
                         "at most 16)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-compensated", action="store_true",
                    help="skip the solve with the compensated FP32 deposit")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the FP32 profiled pass (serial, no graph) and its roofline: "
                         "the run to take a kernel trace of")
    ap.add_argument("--no-staged", action="store_true",
                    help="skip the staged per-level FP64 timing")
    ap.add_argument("--leapfrog-steps", type=int, default=100,
                    help="KDK steps timed for large_nested (energy drift)")
    ap.add_argument("--leapfrog-dt-div", type=int, default=400,
                    help="large_nested: the leapfrog step is the point masses' period over this")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB a few times (the reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    w = None
    ref = None
    if not args.calibrate_copy:
        w = make_workload(args.workload)
        log(f"workload {w.name}: {w.npart} particles, {len(w.grids)} grids, "
            f"{w.active_cells()} active cells")
    if w is not None and not args.no_cpu_baseline and args.workload not in FULL_ORACLE:
        workers = args.oracle_workers or min(16, len(os.sched_getaffinity(0)))
        log(f"oracle leg ({'full' if args.oracle_full else 'staged'}) on {workers} processes")
        ref = staged_oracle(w, args.oracle_full, workers)
        log(f"oracle leg done in {ref['oracle_seconds']:.1f} s")

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

    plan = Plan(w.root_n, w.grids, boundary=w.boundary)
    ctx = ctx0 = Context(plan, 0)
    # the same solve with the compensated FP32 deposit (FP32 pairs, no FP64 accumulation)
    plan_c = Plan(w.root_n, w.grids, boundary=w.boundary, deposit_accum="f32_comp")
    ctx_c = Context(plan_c, 0)
    active = w.active_cells()
    n = w.npart
    fp64_ok = not args.no_fp64
    do_adj = not args.no_adjoint

    def tens(dtype, src=None):
        src = src or (w.x, w.y, w.z, w.m)
        return [torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype))).to(dev) for a in src]

    def gas_for(tdt):
        g = [ctx.pack_gas(l, w.gas, tdt) for l in range(plan.nlevels)]
        return g if any(v is not None for v in g) else None

    tuned = {}

    def run(dtype, steps, warmup, adjoint=False, profile=False, c=None, serial=False):
        ctx = c or ctx0
        if serial:                             # every solve on one stream, no graph
            ctx.profile(True)
        x, y, z, m = tens(dtype)
        gas = gas_for(x.dtype)
        out = [torch.empty(n, dtype=x.dtype, device=dev) for _ in range(4)]
        tot_dev = torch.zeros(plan.nlevels + 5, dtype=torch.float64, device=dev)
        grads = None
        ctx.solve(x, y, z, m, gas, *out)
        torch.cuda.synchronize()
        if (id(ctx), x.dtype) not in tuned:
            tuned[(id(ctx), x.dtype)] = ctx.autotune(x.dtype, reps=5)

        def step():
            ctx.solve(x, y, z, m, gas, *out)
            tot = ctx.solve_totals(m, *out, gas=gas, out=tot_dev)    # stays on the GPU
            g = ctx.solve_adjoint(x, y, z, m, gas, out[3], wbar=1.0) if adjoint else None
            return tot, g

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t_w = time.perf_counter()              # and at least 0.3 s of work: clocks up
        while warmup and time.perf_counter() - t_w < 0.3:
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
        res = dict(ms=ms, wall_ms=1000 * wall / steps, totals=tot.cpu().numpy(), prof=prof)
        if grads is not None:
            res["gx"] = np.stack([t.cpu().numpy().astype(np.float64) for t in grads[:3]], 1)
            res["gm"] = grads[3].cpu().numpy().astype(np.float64)
        res["acc"] = np.stack([o.cpu().numpy().astype(np.float64) for o in out[:3]], 1)
        res["pot"] = out[3].cpu().numpy().astype(np.float64)
        del x, y, z, m, out
        return res

    def staged_path(dtype, steps, src=None, outputs=False, c=None, gas_src=None):
        """The plain per-level path through the staged entry points (owner, deposit,
        solve_level, accel, interp per level, totals), eager: ms per step, and the
        outputs of the last step when asked."""
        ctx = c or ctx0
        x, y, z, m = tens(dtype, src)
        gas = [ctx.pack_gas(l, gas_src or w.gas, x.dtype) for l in range(plan.nlevels)]
        ax, ay, az, pot = (torch.zeros(n, dtype=x.dtype, device=dev) for _ in range(4))
        gmf = [ctx.empty_gmf(l, x.dtype) for l in range(plan.nlevels)]
        own = [ctx.empty_field(l, x.dtype) for l in range(plan.nlevels)]
        fld = [ctx.empty_field(l, x.dtype) for l in range(plan.nlevels)]
        owner = torch.empty(n, dtype=torch.int32, device=dev)

        def step():
            ctx.owner(x, y, z, out=owner)
            for l in range(plan.nlevels):
                ctx.deposit(l, x, y, z, m, gas[l], gas[l - 1] if l > 0 else None, out=gmf[l])
            for l in range(plan.nlevels):
                ctx.solve_level(l, gmf[l], out=own[l])
            for l in range(plan.nlevels):
                ctx.accel(l, own[l], fld[l - 1] if l > 0 else None, out=fld[l])
            for l in range(plan.nlevels):
                ctx.interp(l, fld[l], x, y, z, owner, ax, ay, az, pot)
            return ctx.totals(gmf, m, owner, ax, ay, az, pot)

        step()
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(steps):
            tot = step()
        s1.record()
        torch.cuda.synchronize()
        res = {"ms": s0.elapsed_time(s1) / steps}
        if outputs:
            # own fields: the staged solve_level outputs (the composed ones are fld)
            cpu = lambda t: t.cpu().numpy().astype(np.float64)
            res.update(
                gmf=[ctx.gmf_view(gmf[g["level"]], g["index"]).cpu().numpy().astype(np.float64)
                     for g in plan.grids],
                own=[cpu(ctx.field_view(own[g["level"]], g["index"])) for g in plan.grids],
                field=[cpu(ctx.field_view(fld[g["level"]], g["index"])) for g in plan.grids],
                owner=owner.cpu().numpy(), acc=np.stack([cpu(ax), cpu(ay), cpu(az)], 1),
                pot=cpu(pot), mass=list(tot[:plan.nlevels]))
        del x, y, z, m, gmf, own, fld
        return res

    a32 = a64 = r64 = s64 = rc = None
    comp = {}
    if args.profile_only:
        # only the profiled pass, every solve of the process serial (for a kernel trace
        # whose per-kernel averages are the figures this line reports)
        log(f"FP32: profiled pass only, {args.steps} steps, every solve on one stream")
        psteps = args.steps
        p32 = run(np.float32, psteps, args.warmup, adjoint=do_adj, profile=True, serial=True)
        r32 = p32
        fp64_ok = False
    else:
        log(f"FP32 forward: warmup {args.warmup}, {args.steps} timed steps")
        r32 = run(np.float32, args.steps, args.warmup)
        log(f"FP32 forward: {r32['ms']:.3f} ms/step")
        if do_adj:
            a32 = run(np.float32, args.steps, 1, adjoint=True)
            log(f"FP32 forward+adjoint: {a32['ms']:.3f} ms/step")
        log("FP32: profiled pass (HIP events around every kernel, one stream, no graph)")
        psteps = max(3, args.steps // 3)
        p32 = run(np.float32, psteps, 1, adjoint=do_adj, profile=True)
    if not args.profile_only and not args.no_compensated:
        rc = run(np.float32, args.steps, args.warmup, c=ctx_c)
        log(f"FP32 forward, compensated FP32 deposit: {rc['ms']:.3f} ms/step")
        pc = run(np.float32, psteps, 1, profile=True, c=ctx_c)
        comp = {"deposit_ms_per_step": {k: pc["prof"][k][0] / psteps for k in
                                        ("deposit_tiles", "deposit_finalize") if k in pc["prof"]},
                "deposit_ms_per_step_fp64_accum": {k: p32["prof"][k][0] / psteps for k in
                                                   ("deposit_tiles", "deposit_finalize")
                                                   if k in p32["prof"]}}
        log("deposit kernels, compensated FP32 vs FP64 accumulation (ms): "
            + ", ".join(f"{k} {v:.3f} vs {comp['deposit_ms_per_step_fp64_accum'].get(k, 0):.3f}"
                        for k, v in comp["deposit_ms_per_step"].items()))
    if fp64_ok:
        r64 = run(np.float64, args.steps, args.warmup)
        log(f"FP64 forward: {r64['ms']:.3f} ms/step")
        if do_adj:
            a64 = run(np.float64, max(3, args.steps // 2), 1, adjoint=True)
            log(f"FP64 forward+adjoint: {a64['ms']:.3f} ms/step")
        if not args.no_staged:
            s64 = staged_path(np.float64, max(3, args.steps // 2))
            log(f"FP64 staged per-level path: {s64['ms']:.3f} ms/step")

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
    del pos
    kb = kernel_bytes(plan, n, npl, 4, root_gas=w.gas[0] is not None)
    per_kernel = {k: dict(ms_per_step=v[0] / psteps, launches_per_step=v[1] / psteps)
                  for k, v in p32["prof"].items()}
    forward_names = [k for k in per_kernel if not k.startswith("adj")]
    dom = max(forward_names, key=lambda k: per_kernel[k]["ms_per_step"])
    dom_ms = per_kernel[dom]["ms_per_step"]
    dom_launches = per_kernel[dom]["launches_per_step"]
    dom_launch_ms = dom_ms / dom_launches
    floor_b = floor_bytes(dom, plan, npl, 4)
    ach_b = floor_b if floor_b is not None else kb.get(dom, 0.0)
    achieved = ach_b / (dom_ms * 1e-3) / 1e9
    for k in per_kernel:
        if kb.get(k):
            per_kernel[k]["gbs"] = kb[k] / (per_kernel[k]["ms_per_step"] * 1e-3) / 1e9
    log("per-kernel (FP32): " + ", ".join(
        f"{k} {v['ms_per_step'] * 1e3:.1f}us" + (f" {v['gbs']:.0f}GB/s" if 'gbs' in v else "")
        for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1]['ms_per_step'])))
    fwd_kernels_ms = sum(v["ms_per_step"] for k, v in per_kernel.items() if not k.startswith("adj"))

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
        h = 2 * np.pi * r / v / args.leapfrog_dt_div
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
                x.copy_(x0); y.copy_(y0); z.copy_(z0)
                selfs.append(self_energy())
                x.copy_(xs[0]); y.copy_(xs[1]); z.copy_(xs[2])
            energies.append(float(e[-1]))
            selfs.append(self_energy())
        E = np.array(energies)
        Ec = E - np.array(selfs)
        dev_ = lambda a: float(np.max(np.abs(a - a[0])) / abs(a[0]))
        lf = {"steps": nst, "dt": h, "dt_divisor": args.leapfrog_dt_div, "seconds": sec,
              "ms_per_step": 1000 * sec / nst,
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
        del x, y, z, m, vx, vy, vz, x0, y0, z0, vx0, vy0, vz0, pot, ctx_self

    # errors against the FP64 oracle, and the oracle's own time (CPU baseline)
    cpu = None
    err = {}
    if ref is not None:
        rd = [np.asarray(a, np.float32) for a in (w.x, w.y, w.z, w.m)]
        # the oracle's inputs: the FP32-rounded particles and gas
        rdg = [None if a is None else np.asarray(a, np.float32).astype(np.float64) for a in w.gas]
        for name, dt, c in (("fp32", np.float32, None), ("fp32comp", np.float32, ctx_c),
                            ("fp64", np.float64, None)):
            if (dt == np.float64 and not fp64_ok) or (c is ctx_c and args.no_compensated):
                continue
            got = staged_path(dt, 1, src=rd, outputs=True, c=c, gas_src=rdg)
            e = staged_errors(ref, got, plan.grids)
            err.update({f"{name}_{k}": v for k, v in e.items()})
            del got
        log("errors vs the oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()
                                                  if isinstance(v, float)))
        cpu = {"value": ref["sample_cells"] / ref["sample_seconds"], "unit": "cells/s",
               "cores": ref["workers"], "kind": "oracle", "sample": ref["sample_desc"],
               "seconds": ref["sample_seconds"], "oracle_leg_seconds": ref["oracle_seconds"],
               "mode": ref["mode"]}
        if ref["mode"] == "full":
            cpu["particles_per_s"] = n / ref["sample_seconds"]
    elif not args.no_cpu_baseline and args.workload in FULL_ORACLE:
        from oracle import apm_oracle as O
        from oracle import apm_adjoint as A
        log("oracle: Green's functions (cached, as on the GPU), then one timed forward solve "
            "and one timed reverse sweep")
        op = O.OraclePlan(w.root_n, w.grids, boundary=w.boundary)
        cache = {g.index: O.greens(op, g) for g in op.grids}
        rdn = lambda a: None if a is None else np.asarray(a, np.float32).astype(np.float64)
        x32 = [rdn(a) for a in (w.x, w.y, w.z, w.m)]
        g32 = [rdn(a) for a in w.gas]
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
        "fp32_compensated_deposit": (dict(step_info(rc), **comp) if rc is not None else None),
        "fp64": step_info(r64),
        "fwd_adjoint_fp64": step_info(a64),
        "staged_per_level_fp64": step_info(s64),
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
                     "bytes_basis": ("three-pass floor (pass B: the z pass)" if floor_b is not None
                                     else "kernel's algorithmic bytes"),
                     "algorithmic_bytes_per_launch": ach_b / dom_launches,
                     "algorithmic_bytes_per_step": ach_b,
                     "kernel_array_bytes_per_step": kb.get(dom, 0.0),
                     "profiled_ms_per_step": p32["ms"],
                     "forward_kernels_ms_per_step": fwd_kernels_ms},
        "kernels_fp32": per_kernel,
        "launch": {"graph": ("none: every solve serial (profile-only run)" if args.profile_only
                             else "apm_solve captured once, replayed per step"),
                   "autotuned_lines_per_block": {k: v["lines"] for d in tuned.values()
                                                 for k, v in d.items()}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


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


if __name__ == "__main__":
    main()
