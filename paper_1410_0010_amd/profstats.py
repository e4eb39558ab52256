"""Per-kernel statistics from rocprofv3 csv output: a kernel trace (``--kernel-trace``)
or, with ``--counters``, a counter collection (``--pmc ...``).

    python -m paper_1410_0010_amd.profstats <trace.csv | output dir> [--dtype float]
    python -m paper_1410_0010_amd.profstats --counters <counter_collection.csv | dir>

For each kernel it reports all dispatches and, separately, the dispatches of its most
frequent launch shape (grid, workgroup, LDS): a timed run launches every transform
pass with one tuned shape, while the autotuner's candidate launches use others.  The
family table merges the instantiations of one kernel (e.g. both FFT lengths of the z
pass) under the name the library's own per-kernel timer uses, so its per-launch
average is comparable with that timer's."""

import argparse
import collections
import csv
import glob
import hashlib
import os
import statistics
import sys

# kernel function -> family name of the library's per-kernel timer
FAMILY = {
    "k_fft_x_fwd": "fft_x_fwd", "k_fft_y_fwd": "fft_y_fwd", "k_fft_z_conv": "fft_z_conv",
    "k_fft_y_inv": "fft_y_inv", "k_fft_x_inv": "fft_x_inv",
    "k_adj_x": "adj_fft_x", "k_adjp_x": "adj_fft_x", "k_adj_y": "adj_fft_y", "k_adjp_y": "adj_fft_y",
    "k_adj_z": "adj_fft_z", "k_adjp_z": "adj_fft_z", "k_adj_y_inv": "adj_fft_y_inv",
    "k_adj_x_inv": "adj_fft_x_inv",
    "k_dep_clear": "bin_clear", "k_scan_tiles": "bin_scan",
    "k_sort_keys": "sort", "k_radix_hist": "sort", "k_hscan_reduce": "sort", "k_hscan_mid": "sort",
    "k_hscan_down": "sort", "k_radix_scatter": "sort", "k_sort_gather": "sort",
    "k_tile_ranges": "tile_ranges",
    "k_scan_blocks": "bin_scan", "k_scan_emit": "bin_scan",
    "k_adj_interp_grad": "adj_interp", "k_totals_parts": "totals", "k_particle_totals": "totals",
    "k_totals_finish": "totals",
    "k_deposit_tiles": "deposit_tiles",
    "k_deposit_finalize": "deposit_finalize", "k_owner": "owner", "k_compose": "compose",
    "k_interp_tiles": "interp", "k_interp": "interp", "k_unpack": "unpack",
    "k_adj_interp": "adj_interp", "k_adj_deposit_particles": "adj_deposit_particles",
    "k_adj_deposit_grid": "adj_deposit_grid", "k_adj_restrict": "adj_restrict",
    "k_adj_finish": "adj_finish", "k_adj_unpack": "adj_finish", "k_zero_ranges": "adj_clear",
}


def sources_sha256():
    """Fingerprint of the native sources (every file under csrc/ and the C header):
    counter figures taken on other sources do not describe the current kernels."""
    here = os.path.dirname(os.path.abspath(__file__))
    files = sorted(glob.glob(os.path.join(here, "csrc", "*")))
    files.append(os.path.join(os.path.dirname(here), "include", "apm.h"))
    h = hashlib.sha256()
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def traffic_record(path):
    """The key=value fields of the line starting with 'traffic-record:' in a counter
    summary (None if the file or the line is missing)."""
    if not os.path.isfile(path):
        return None
    with open(path) as f:
        for line in f:
            line = line.strip().strip("`")
            if line.startswith("traffic-record:"):
                return dict(kv.split("=", 1) for kv in line.split(":", 1)[1].split())
    return None


def short_name(full):
    s = full.replace("void ", "").replace("apm::", "").replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in s:                      # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def other_dtype(dtype):
    """The precision a family table leaves out (instantiations on index types stay)."""
    return "double" if dtype == "float" else "float"


def find(path, suffix):
    if os.path.isdir(path):
        hits = glob.glob(os.path.join(path, "**", "*" + suffix), recursive=True)
        if not hits:
            sys.exit(f"no *{suffix} under {path}")
        return hits[0]
    return path


def load_counters(path):
    """(kernel, launch shape, counter) -> values per dispatch."""
    path = find(path, "counter_collection.csv")
    out = collections.defaultdict(list)
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            shape = (int(r["Grid_Size"]), int(r["Workgroup_Size"]), int(r["LDS_Block_Size"]))
            out[(short_name(r["Kernel_Name"]), shape, r["Counter_Name"])].append(
                float(r["Counter_Value"]))
    return path, out


def counters_main(path, dtype):
    path, data = load_counters(path)
    per_kernel = collections.defaultdict(dict)
    for (name, shape, ctr), v in data.items():
        per_kernel[(name, ctr)][shape] = v
    print(f"counters: {os.path.basename(path)} (values per dispatch, as rocprofv3 reports them)\n")
    print("| kernel | counter | main-shape dispatches | avg per dispatch | all dispatches | avg |")
    print("|---|---|---:|---:|---:|---:|")
    fam = collections.defaultdict(list)
    rows = []
    for (name, ctr), shapes in per_kernel.items():
        top = max(shapes, key=lambda k: len(shapes[k]))
        sel = shapes[top]
        allv = [x for v in shapes.values() for x in v]
        rows.append((name, ctr, sel, allv))
        base = name.split("<")[0]
        if base in FAMILY and other_dtype(dtype) not in name[len(base):]:
            fam[(FAMILY[base], ctr)].extend(sel)
    for name, ctr, sel, allv in sorted(rows, key=lambda r: -sum(r[2]) / len(r[2])):
        print(f"| `{name}` | {ctr} | {len(sel)} | {sum(sel) / len(sel):.1f} | {len(allv)} | "
              f"{sum(allv) / len(allv):.1f} |")
    print(f"\nFamilies ({dtype}; main-shape dispatches of every instantiation):\n")
    print("| family | counter | dispatches | avg per dispatch |")
    print("|---|---|---:|---:|")
    for (f, ctr), v in sorted(fam.items(), key=lambda kv: -sum(kv[1]) / len(kv[1])):
        print(f"| {f} | {ctr} | {len(v)} | {sum(v) / len(v):.1f} |")


def load(path):
    path = find(path, "kernel_trace.csv")
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            shape = tuple(int(r[k]) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
                                              "Workgroup_Size_X", "Workgroup_Size_Y",
                                              "Workgroup_Size_Z", "LDS_Block_Size"))
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
            rows.append((short_name(r["Kernel_Name"]), shape, us))
    return path, rows


def stats(v):
    return dict(n=len(v), avg=sum(v) / len(v), med=statistics.median(v), min=min(v), max=max(v),
                tot=sum(v))


def timeline_main(path, first, last):
    """Launch timeline of repeated solves in a kernel trace: a solve runs from a
    dispatch of `first` to the next dispatch of `last`; per solve, its span, the time
    some kernel was running (union of the dispatch intervals, both streams), the sum
    of the dispatch times, and the idle gaps between dispatches."""
    path = find(path, "kernel_trace.csv")
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
                         short_name(r["Kernel_Name"])))
    rows.sort()
    starts = [i for i, r in enumerate(rows) if r[2].split("<")[0] == first]
    solves = []
    for a, b in zip(starts, starts[1:] + [len(rows)]):
        seg = rows[a:b]
        ends = [j for j, r in enumerate(seg) if r[2].split("<")[0] == last]
        if not ends:
            continue
        seg = seg[:ends[0] + 1]
        iv = sorted((r[0], r[1]) for r in seg)
        busy, gaps = 0, []
        cs, ce = iv[0]
        for s0, e0 in iv[1:]:
            if s0 > ce:
                busy += ce - cs
                gaps.append(s0 - ce)
                cs, ce = s0, e0
            else:
                ce = max(ce, e0)
        busy += ce - cs
        solves.append(dict(n=len(seg), span=(max(r[1] for r in seg) - seg[0][0]) / 1e3,
                           busy=busy / 1e3, ksum=sum(r[1] - r[0] for r in seg) / 1e3,
                           gaps=len(gaps), gapsum=sum(gaps) / 1e3,
                           maxgap=max(gaps) / 1e3 if gaps else 0.0))
    if not solves:
        sys.exit("no solve found between the given kernels")
    common = statistics.mode(s["n"] for s in solves)
    sel = [s for s in solves if s["n"] == common]
    print(f"timeline: {os.path.basename(path)}, {len(solves)} solves from `{first}` to "
          f"`{last}`; {len(sel)} of {common} dispatches (the common shape) summarised\n")
    print("| per solve | median | min | max |")
    print("|---|---:|---:|---:|")
    for k, label in (("span", "span, us"), ("busy", "some kernel running, us"),
                     ("ksum", "sum of dispatch times, us"), ("gapsum", "idle gaps, us"),
                     ("gaps", "idle gaps, count"), ("maxgap", "largest gap, us")):
        v = [s[k] for s in sel]
        print(f"| {label} | {statistics.median(v):.1f} | {min(v):.1f} | {max(v):.1f} |")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("trace", nargs="?")
    ap.add_argument("--dtype", default="float", help="precision for the family table")
    ap.add_argument("--counters", action="store_true", help="the input is a counter collection")
    ap.add_argument("--sha", action="store_true", help="print the native sources' fingerprint")
    ap.add_argument("--timeline", nargs=2, metavar=("FIRST", "LAST"),
                    help="launch timeline of the solves from kernel FIRST to kernel LAST")
    a = ap.parse_args(argv)
    if a.timeline:
        timeline_main(a.trace, *a.timeline)
        return
    if a.sha:
        print(sources_sha256())
        return
    if a.counters:
        counters_main(a.trace, a.dtype)
        return
    path, rows = load(a.trace)
    by = collections.defaultdict(list)
    for name, shape, us in rows:
        by[name].append((shape, us))
    table = []
    fam = collections.defaultdict(list)
    for name, d in by.items():
        shapes = collections.Counter(s for s, _ in d)
        top = shapes.most_common(1)[0][0]
        sel = [us for s, us in d if s == top]
        table.append((name, stats([us for _, us in d]), stats(sel), top))
        base = name.split("<")[0]
        targs = name[len(base):]
        if base in FAMILY and other_dtype(a.dtype) not in targs:
            fam[FAMILY[base]].extend(sel)
    table.sort(key=lambda t: -t[1]["tot"])
    total = sum(t[1]["tot"] for t in table)
    print(f"trace: {os.path.basename(path)}, {len(rows)} dispatches, {total / 1e3:.3f} ms of kernel time\n")
    print("| kernel | dispatches | avg us | total ms | % | main shape: dispatches | avg us | median us |"
          " min us | max us |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    for name, s_all, s_sel, _ in table:
        print(f"| `{name}` | {s_all['n']} | {s_all['avg']:.1f} | {s_all['tot'] / 1e3:.3f} | "
              f"{100 * s_all['tot'] / total:.1f} | {s_sel['n']} | {s_sel['avg']:.1f} | "
              f"{s_sel['med']:.1f} | {s_sel['min']:.1f} | {s_sel['max']:.1f} |")
    print(f"\nFamilies ({a.dtype}; main-shape dispatches of every instantiation, i.e. every FFT "
          "length):\n")
    print("| family | dispatches | avg us per launch | median us |")
    print("|---|---:|---:|---:|")
    for f, v in sorted(fam.items(), key=lambda kv: -sum(kv[1])):
        s = stats(v)
        print(f"| {f} | {s['n']} | {s['avg']:.1f} | {s['med']:.1f} |")


if __name__ == "__main__":
    main()
