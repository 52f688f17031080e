"""Summaries of rocprofv3 output for this library's kernels (measurement tooling, not part of
the method).

    python -m paper_1412_0781_amd.prof_summary trace DIR --command "..."
        per-kernel calls / total / average / min / max duration from a --kernel-trace --stats
        run, plus the full-pass dispatches of the forward kernels (largest grid of each)
    python -m paper_1412_0781_amd.prof_summary calib --fetch DIR --write DIR --gib G --command-fetch "..." --command-write "..."
        FETCH_SIZE / WRITE_SIZE of a plain device copy of G GiB: the factors that turn the
        counters into bytes
    python -m paper_1412_0781_amd.prof_summary hbm --fetch DIR --write DIR --calib FILE --L L \
            --pass-images M --cov-images N --out-dir profiles --command-fetch "..." --command-write "..."
        HBM bytes per image of each forward stage and of the covariance (counters averaged over
        the full-pass dispatches, scaled by the calibration), one file per stage, with the digest
        of the kernel sources the counters were taken on
    python -m paper_1412_0781_amd.prof_summary counters DIR --command "..." [--per N]
        every counter of a --pmc run averaged per dispatch, per kernel (full-pass dispatches),
        with MFMA utilisation when SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE were collected

rocprofv3 writes CSV files under DIR (possibly in a host / process subdirectory); they are
found by their suffixes (_kernel_stats.csv, _kernel_trace.csv, _counter_collection.csv).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources whose change invalidates stored counter readings of the expansion / covariance kernels
KERNEL_SOURCES = ["paper_1412_0781_amd/csrc/" + f for f in
                  ("nufft.hip", "fft_dev.h", "dev_common.h", "plan.h", "plan.cpp", "gemm.hip", "api.cpp")]
# benchmark stage -> kernels (name prefixes) that make it up
STAGES = {
    "fwd_rows": ("k_fwd_rows",),
    "fwd_cols": ("k_fwd_cols",),
    "fwd_gather": ("k_fwd_gather",),
    "fwd_angular": ("k_fwd_angular",),
    "radial_fwd": ("k_radial_fwd",),
    "covariance": ("k_covariance", "k_cov_reduce"),
    "radial_adj": ("k_radial_adj",),
    "adj_angular": ("k_adj_angular",),
    "adj_spread": ("k_adj_spread",),
    "adj_cols": ("k_adj_cols",),
    "adj_rows": ("k_adj_rows",),
}
SIMDS = 256 * 4  # MI355X: 256 compute units of 4 SIMDs
XCDS = 8         # GRBM_GUI_ACTIVE arrives summed over the 8 XCDs (each counts the same busy cycles)


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _csv(dirpath: str, suffix: str) -> list:
    files = sorted(glob.glob(os.path.join(dirpath, "**", f"*{suffix}"), recursive=True))
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name: str) -> str:
    """Kernel name without the namespace and the argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    if "(" in name:
        name = name[:name.index("(")]
    return name.replace("fb::", "")


def _grid(row: dict) -> int:
    for key in ("Grid_Size", "Grid_Size_X", "grid_size"):
        if key in row and row[key] not in ("", None):
            g = int(float(row[key]))
            for ky in ("Grid_Size_Y", "Grid_Size_Z"):
                if ky in row and row[ky] not in ("", None):
                    g *= max(1, int(float(row[ky])))
            return g
    return 0


def cmd_trace(a):
    stats = _csv(a.dir, "_kernel_stats.csv")
    trace = _csv(a.dir, "_kernel_trace.csv")
    print(f"# rocprofv3 kernel trace: {a.title}")
    print(f"command: {a.command}")
    print()
    print(f"{'kernel':44s} {'calls':>7s} {'total_ms':>10s} {'avg_ms':>9s} {'min_ms':>9s} {'max_ms':>9s}")
    rows = []
    for r in stats:
        name = _short(r.get("Name", r.get("KernelName", "")))
        calls = int(float(r["Calls"]))
        tot = float(r["TotalDurationNs"]) / 1e6
        rows.append((tot, name, calls, float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6))
    for tot, name, calls, avg, mn, mx in sorted(rows, reverse=True):
        if name.startswith("k_"):
            print(f"{name:44s} {calls:7d} {tot:10.3f} {avg:9.4f} {mn:9.4f} {mx:9.4f}")
    if trace:
        by = defaultdict(list)
        for r in trace:
            name = _short(r["Kernel_Name"])
            if any(name.startswith(p) for ps in STAGES.values() for p in ps):
                by[name].append((_grid(r), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6))
        print()
        print("full-pass dispatches only (largest grid of each forward and covariance kernel):")
        for name in sorted(by):
            g = max(x[0] for x in by[name])
            d = [x[1] for x in by[name] if x[0] == g]
            print(f"  {name:44s} grid={g:>10d} dispatches={len(d):5d} avg_ms={sum(d) / len(d):9.4f}")


def _counter_table(dirpath: str, ours: bool = True):
    """{kernel: (grid, dispatches, {counter: mean value per dispatch of the largest grid})}; ours:
    this library's kernels only (names k_*)"""
    rows = _csv(dirpath, "_counter_collection.csv")
    per = defaultdict(lambda: defaultdict(dict))  # kernel -> dispatch -> counter -> value
    grid = {}
    for r in rows:
        name = _short(r["Kernel_Name"])
        if ours and not name.startswith("k_"):
            continue
        d = r.get("Dispatch_Id", r.get("Correlation_Id"))
        per[name][d][r["Counter_Name"]] = per[name][d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        grid[(name, d)] = _grid(r)
    out = {}
    for name, disp in per.items():
        g = max(grid[(name, d)] for d in disp)
        full = [d for d in disp if grid[(name, d)] == g]
        cnt = defaultdict(list)
        for d in full:
            for c, v in disp[d].items():
                cnt[c].append(v)
        out[name] = (g, len(full), {c: sum(v) / len(v) for c, v in cnt.items()})
    return out


def cmd_calib(a):
    nbytes_kib = a.gib * (1 << 20)
    f = _counter_table(a.fetch, ours=False)
    w = _counter_table(a.write, ours=False)

    def total(t, c):
        # the copy is the only large dispatch: take the kernel with the largest counter value
        return max(v[2].get(c, 0.0) for v in t.values()) if t else 0.0
    fk, wk = total(f, "FETCH_SIZE"), total(w, "WRITE_SIZE")
    print(f"# HBM byte-counter calibration on a plain device copy of {a.gib:g} GiB (torch copy_, one dispatch)")
    print(f"command: {a.command_fetch}")
    print(f"FETCH_SIZE: {fk:.1f} KiB counted for {nbytes_kib:.0f} KiB read -> scale factor {nbytes_kib / fk:.4f}")
    print(f"command: {a.command_write}")
    print(f"WRITE_SIZE: {wk:.1f} KiB counted for {nbytes_kib:.0f} KiB written -> scale factor {nbytes_kib / wk:.4f}")


def _calib_factors(path: str):
    fs = ws = None
    with open(path) as f:
        for line in f:
            if line.startswith("FETCH_SIZE:"):
                fs = float(line.rsplit("factor", 1)[1])
            elif line.startswith("WRITE_SIZE:"):
                ws = float(line.rsplit("factor", 1)[1])
    return fs, ws


def algorithmic_bytes_per_image(L: int, grid_n: int, w: int, n_xi: int, H: int, k_max: int, p_half: int) -> dict:
    M2 = grid_n // 2 + 2 * (w // 2 + 1) + 1
    c8 = 8
    img, g1, g = 4 * L * L, c8 * M2 * L, c8 * M2 * grid_n
    P, fh, co = c8 * n_xi * H, c8 * (k_max + 1) * n_xi, c8 * p_half
    y, y1 = c8 * (grid_n // 2 + 1) * grid_n, c8 * (grid_n // 2 + 1) * L  # adjoint half-plane grid, column pass
    return {"fwd_rows": img + g1, "fwd_cols": g1 + g, "fwd_gather": g + P, "fwd_angular": P + fh,
            "radial_fwd": fh + co, "covariance": co, "radial_adj": co + fh, "adj_angular": fh + P,
            "adj_spread": P + y, "adj_cols": y + y1, "adj_rows": y1 + img}


def cmd_hbm(a):
    sys.path.insert(0, ROOT)
    from paper_1412_0781_amd import Plan
    pl = Plan(a.L, 0.5, a.L / 2, device=False)
    alg = algorithmic_bytes_per_image(pl.L, pl.grid_n, pl.kernel_w, pl.n_xi, pl.n_theta // 2, pl.k_max, pl.p_half)
    fs, ws = _calib_factors(a.calib)
    f = _counter_table(a.fetch)
    w = _counter_table(a.write)
    digest = source_digest()
    wanted = set(a.stages.split(",")) if a.stages else set(STAGES)
    for stage, prefixes in STAGES.items():
        if stage not in wanted:
            continue
        names = sorted(n for n in set(f) | set(w) if any(n.startswith(p) for p in prefixes))
        if not names:
            continue
        imgs = a.cov_images if stage == "covariance" else a.pass_images
        fk = sum(f[n][2].get("FETCH_SIZE", 0.0) for n in names if n in f)
        wk = sum(w[n][2].get("WRITE_SIZE", 0.0) for n in names if n in w)
        disp = max(f[n][1] for n in names if n in f) if any(n in f for n in names) else 0
        per_image = (fk * fs + wk * ws) * 1024 / imgs
        path = os.path.join(a.out_dir, f"{stage}_hbm_counters_L{a.L}.txt")
        with open(path, "w") as out:
            out.write(f"# HBM traffic of the {stage} stage ({', '.join(names)}), L = {a.L}, R = {a.L // 2}, "
                      f"c = 1/2, {a.form} form\n")
            out.write("# FETCH_SIZE and WRITE_SIZE in KiB per dispatch (average over the run's full-pass\n"
                      "# dispatches), each scaled by the plain-copy calibration factor; one run per counter.\n")
            out.write(f"command_fetch: {a.command_fetch}\n")
            out.write(f"command_write: {a.command_write}\n")
            out.write(f"command_summary: python3 -m paper_1412_0781_amd.prof_summary hbm (see this file's header)\n")
            out.write(f"source_digest: {digest}\n")
            out.write(f"dispatches_per_run: {disp}\n")
            out.write(f"images_per_dispatch: {imgs}\n")
            out.write(f"FETCH_SIZE_KiB_per_dispatch: {fk:.1f}\n")
            out.write(f"WRITE_SIZE_KiB_per_dispatch: {wk:.1f}\n")
            out.write(f"fetch_scale: {fs:.4f}\n")
            out.write(f"write_scale: {ws:.4f}\n")
            out.write(f"hbm_bytes_per_image: {per_image:.1f}\n")
            out.write(f"algorithmic_bytes_per_image: {alg[stage]}\n")
            out.write(f"traffic_over_algorithmic: {per_image / alg[stage]:.3f}\n")
        print(f"{stage}: {per_image / 1e6:.3f} MB per image ({per_image / alg[stage]:.3f} x algorithmic) -> {path}")


def cmd_counters(a):
    t = _counter_table(a.dir)
    print(f"# rocprofv3 counters per dispatch (average over the full-pass dispatches of each kernel): {a.title}")
    print(f"command: {a.command}")
    counters = sorted({c for v in t.values() for c in v[2]})
    print()
    head = f"{'kernel':44s} {'disp':>5s} " + " ".join(f"{c:>28s}" for c in counters)
    mfma = "SQ_VALU_MFMA_BUSY_CYCLES" in counters and "GRBM_GUI_ACTIVE" in counters
    mops = [c for c in counters if c.startswith("SQ_INSTS_VALU_MFMA_MOPS_")]
    if mfma:
        head += f" {'MFMA_busy_%':>12s}"
    if mops:
        head += f" {'MFMA_GFLOP':>11s}"
    print(head)
    for name in sorted(t, key=lambda n: -max(t[n][2].values(), default=0.0)):
        g, nd, v = t[name]
        line = f"{name:44s} {nd:5d} " + " ".join(f"{v.get(c, 0.0):28.1f}" for c in counters)
        if mfma and v.get("GRBM_GUI_ACTIVE", 0.0) > 0:
            # busy cycles summed over all SIMDs / (the kernel's active cycles x SIMDs)
            line += f" {100.0 * v['SQ_VALU_MFMA_BUSY_CYCLES'] / (v['GRBM_GUI_ACTIVE'] / XCDS * SIMDS):12.2f}"
        if mops:
            # each MOPS count is 512 flops
            line += f" {sum(v.get(c, 0.0) for c in mops) * 512 / 1e9:11.2f}"
        print(line)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("trace")
    p.add_argument("dir")
    p.add_argument("--command", required=True)
    p.add_argument("--title", default="")
    p = sub.add_parser("calib")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--gib", type=float, required=True)
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    p = sub.add_parser("hbm")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--calib", required=True)
    p.add_argument("--L", type=int, default=256)
    p.add_argument("--pass-images", type=int, required=True)
    p.add_argument("--cov-images", type=int, required=True)
    p.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    p.add_argument("--form", default="BF16x3")
    p.add_argument("--stages", default="", help="comma-separated stages to write (default: every stage found)")
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    p = sub.add_parser("counters")
    p.add_argument("dir")
    p.add_argument("--command", required=True)
    p.add_argument("--title", default="")
    a = ap.parse_args(argv)
    {"trace": cmd_trace, "calib": cmd_calib, "hbm": cmd_hbm, "counters": cmd_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
