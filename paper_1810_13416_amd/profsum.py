"""Summaries of rocprofv3 output for the pass kernels (text, a few KB).

    python -m paper_1810_13416_amd.profsum stats  <kernel_stats.csv> <out.md> <command...>
    python -m paper_1810_13416_amd.profsum traffic <fetch counter_collection.csv>
           <write counter_collection.csv> <calib MiB> <cells> <out.txt> <command...>
    python -m paper_1810_13416_amd.profsum counters <out.md> <title> <csv> [<csv> ...] -- <command...>
    python -m paper_1810_13416_amd.profsum dispatches <kernel_trace.csv> <out.md> <name part[,part...]>
           <min grid threads> <command...>

`stats` turns a `--kernel-trace --stats` run into a table of kernels by
total time; `counters` tabulates any `--pmc` counters per kernel (mean per
dispatch) from one or more runs.  `traffic` turns two `--pmc` runs (FETCH_SIZE, then WRITE_SIZE,
both in KiB per dispatch) into HBM bytes per launch of each pass kernel,
scaled by what the same counters read for one plain elementwise copy of
known size (`bench.py --calib-copy-mib M`, which reads M MiB and writes M
MiB), and records a hash of the pass sources so that a reader can tell
whether the figures still describe the kernels as built.  `dispatches`
summarises, from the per-dispatch trace of a `--kernel-trace` run, the
launches of the kernels whose name contains one of the given parts and whose grid has
at least a given number of work-items (so that launches of one problem size
are not averaged with those of another).
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_SOURCES = ["csrc/ppmb_sweep.hip", "csrc/ppmb_dev.h", "csrc/ppmb_internal.h", "build.py"]


def sweep_sources_hash() -> str:
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """'void ppmb::sweep_kernel<float, 1>(ppmb::BatchArgs<float>)' ->
    'sweep_kernel<float, 1>'; other kernels keep their name up to '('."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    n = n.replace("ppmb::", "")
    return re.sub(r"\s+", " ", n)


def _col(header, *keys):
    low = [h.lower() for h in header]
    for k in keys:
        for i, h in enumerate(low):
            if h == k:
                return i
    for k in keys:
        for i, h in enumerate(low):
            if k in h:
                return i
    raise KeyError(f"none of {keys} in {header}")


def read_kernel_stats(path):
    with open(path, newline="") as f:
        rows = list(csv.reader(f))
    hdr, body = rows[0], rows[1:]
    iname = _col(hdr, "name", "kernel_name")
    icalls = _col(hdr, "calls")
    itot = _col(hdr, "totaldurationns")
    iavg = _col(hdr, "averagens")
    imin = _col(hdr, "minns")
    imax = _col(hdr, "maxns")
    out = []
    for r in body:
        if not r:
            continue
        out.append({"name": short_name(r[iname]), "calls": int(r[icalls]),
                    "total_ms": float(r[itot]) * 1e-6, "avg_ms": float(r[iavg]) * 1e-6,
                    "min_ms": float(r[imin]) * 1e-6, "max_ms": float(r[imax]) * 1e-6})
    out.sort(key=lambda d: -d["total_ms"])
    return out


def write_stats(csv_path, out_path, command):
    rows = read_kernel_stats(csv_path)
    tot = sum(r["total_ms"] for r in rows) or 1.0
    lines = ["# Kernel time, rocprofv3 --kernel-trace --stats", "",
             "Command:", "", "    " + command, "",
             "| kernel | calls | total ms | avg ms | min ms | max ms | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['name']}` | {r['calls']} | {r['total_ms']:.3f} | {r['avg_ms']:.4f} | "
                     f"{r['min_ms']:.4f} | {r['max_ms']:.4f} | {100 * r['total_ms'] / tot:.1f} |")
    trace = os.path.join(os.path.dirname(csv_path), os.path.basename(csv_path).replace("kernel_stats", "kernel_trace"))
    if trace != csv_path and os.path.exists(trace):
        lines += _steady_table(trace)
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _steady_table(trace_csv):
    """The pass kernels' dispatches after the first of each: the first pass
    after a state is set updates every cell (the solid cells are not yet
    known to be equal in both buffers), the later ones only the cells within
    the stencil reach of the fluid; these are the launches the bench times."""
    with open(trace_csv, newline="") as f:
        rows = list(csv.reader(f))
    hdr, body = rows[0], rows[1:]
    iname, i0, i1 = _col(hdr, "kernel_name"), _col(hdr, "start_timestamp"), _col(hdr, "end_timestamp")
    per = {}
    for r in body:
        if r and short_name(r[iname]).startswith("sweep"):
            per.setdefault(short_name(r[iname]), []).append(int(r[i1]) - int(r[i0]))
    out = ["", "Pass kernels without their first dispatch (the launches the bench times):", "",
           "| kernel | dispatches | avg ms | median ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    for k in sorted(per):
        ns = per[k][1:]
        if ns:
            out.append(f"| `{k}` | {len(ns)} | {sum(ns) / len(ns) * 1e-6:.4f} | {_median(ns) * 1e-6:.4f} | "
                       f"{min(ns) * 1e-6:.4f} | {max(ns) * 1e-6:.4f} |")
    return out


def read_counters(path, counter):
    """Per kernel: list of counter values (one per dispatch)."""
    with open(path, newline="") as f:
        rows = list(csv.reader(f))
    hdr, body = rows[0], rows[1:]
    iname = _col(hdr, "kernel_name")
    icn = _col(hdr, "counter_name")
    icv = _col(hdr, "counter_value")
    idisp = _col(hdr, "dispatch_id", "correlation_id")
    per = {}
    seen = {}
    for r in body:
        if not r or r[icn] != counter:
            continue
        key = (r[idisp], r[iname])
        seen[key] = seen.get(key, 0.0) + float(r[icv])     # sum over instances if split
    for (disp, name), v in seen.items():
        per.setdefault(short_name(name), []).append(v)
    return per


def _calib_value(per, mib):
    """Counter reading of the calibration copy: the dispatch of an
    elementwise 'neg' kernel whose reading is closest to M MiB."""
    cands = [(k, v) for k, vs in per.items() for v in vs if "neg" in k.lower()]
    if not cands:
        cands = [(k, v) for k, vs in per.items() for v in vs if "elementwise" in k.lower()]
    if not cands:
        raise RuntimeError("calibration copy dispatch not found")
    want = mib * 1024.0
    k, v = min(cands, key=lambda kv: abs(kv[1] - want))
    return k, v


def _median(v):
    v = sorted(v)
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def write_traffic(fetch_csv, write_csv, mib, cells, out_path, command):
    fe = read_counters(fetch_csv, "FETCH_SIZE")
    wr = read_counters(write_csv, "WRITE_SIZE")
    ck, cf = _calib_value(fe, mib)
    _, cw = _calib_value(wr, mib)
    true_kib = mib * 1024.0
    sf, sw = true_kib / cf, true_kib / cw
    alg = (2 * 15 + 2) * 4 * cells
    lines = ["# HBM traffic of the FP32 pass kernels, spherical shell 512^3", "",
             "Counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch, the median over a",
             "kernel's dispatches: the first pass after the state is set writes every",
             "cell, later ones skip the solid cells beyond the stencil reach) from two",
             "separate rocprofv3 --pmc runs of the same command, scaled by what they read",
             f"for one plain elementwise copy of {mib} MiB in and {mib} MiB out.",
             f"Algorithmic bytes: 15 fields read and written once and the base rho0 and",
             f"p0 read once per updated (fluid) cell, {cells} cells.", "",
             "Command (run once with --pmc FETCH_SIZE, once with --pmc WRITE_SIZE):", "",
             "    " + command, "",
             f"sweep_sources_sha256: {sweep_sources_hash()}",
             f"calibration_kernel: {ck}",
             f"calibration: FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB for {true_kib:.0f} KiB each; "
             f"scale fetch {sf:.4f}, write {sw:.4f}",
             f"algorithmic_bytes_per_launch: {alg}", "",
             "| kernel | dispatches | FETCH KiB | WRITE KiB | HBM bytes/launch (scaled) | / algorithmic |",
             "|---|---|---|---|---|---|"]
    result = {}
    for k in sorted(set(fe) & set(wr)):
        f_kib = _median(fe[k])
        w_kib = _median(wr[k])
        b = (f_kib * sf + w_kib * sw) * 1024.0
        lines.append(f"| `{k}` | {len(fe[k])} | {f_kib:.0f} | {w_kib:.0f} | {b:.4g} | "
                     f"{b / alg:.3f} |")
        if k.startswith("sweep"):
            result[k] = b
    lines.append("")
    for k, b in result.items():
        lines.append(f"bytes_per_launch {k}: {b:.6g}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_dispatches(trace_csv, out_path, part, min_grid, command):
    with open(trace_csv, newline="") as f:
        rows = list(csv.reader(f))
    hdr, body = rows[0], rows[1:]
    iname = _col(hdr, "kernel_name")
    i0 = _col(hdr, "start_timestamp")
    i1 = _col(hdr, "end_timestamp")
    ig = [_col(hdr, "grid_size_" + a) for a in "xyz"]
    parts = [p for p in part.split(",") if p]
    per = {}
    for r in body:
        if not r or not any(p in r[iname] for p in parts):
            continue
        grid = 1
        for i in ig:
            grid *= int(r[i])
        if grid < min_grid:
            continue
        d = per.setdefault(short_name(r[iname]), {"grid": grid, "ns": []})
        d["ns"].append(int(r[i1]) - int(r[i0]))
    lines = ["# Kernel time per dispatch, rocprofv3 --kernel-trace", "",
             "Command:", "", "    " + command, "",
             "Dispatches of kernels named " + " or ".join(f"`*{p}*`" for p in parts) +
             f" with a grid of at least {min_grid} work-items.", "",
             "| kernel | grid work-items | dispatches | avg ms | min ms | max ms |",
             "|---|---|---|---|---|---|"]
    for k in sorted(per):
        ns = per[k]["ns"]
        lines.append(f"| `{k}` | {per[k]['grid']} | {len(ns)} | "
                     f"{sum(ns) / len(ns) * 1e-6:.4f} | {min(ns) * 1e-6:.4f} | {max(ns) * 1e-6:.4f} |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_all_counters(path):
    """{kernel: {counter: [value per dispatch]}} for every counter in a run."""
    with open(path, newline="") as f:
        rows = list(csv.reader(f))
    hdr, body = rows[0], rows[1:]
    iname = _col(hdr, "kernel_name")
    icn = _col(hdr, "counter_name")
    icv = _col(hdr, "counter_value")
    idisp = _col(hdr, "dispatch_id", "correlation_id")
    acc = {}
    for r in body:
        if not r:
            continue
        key = (r[idisp], short_name(r[iname]), r[icn])
        acc[key] = acc.get(key, 0.0) + float(r[icv])
    out = {}
    for (disp, k, c), v in acc.items():
        out.setdefault(k, {}).setdefault(c, []).append(v)
    return out


def write_counters(out_path, title, csvs, command, only_prefix=("sweep", "cfl_kernel")):
    per = {}
    for p in csvs:
        for k, cs in read_all_counters(p).items():
            per.setdefault(k, {}).update(cs)
    names = sorted({c for cs in per.values() for c in cs})
    lines = [f"# {title}", "", "Command (one run per counter group):", "", "    " + command, "",
             f"sweep_sources_sha256: {sweep_sources_hash()}", "",
             "Median per dispatch (the first pass after the state is set writes every",
             "cell; later passes skip the solid cells beyond the stencil reach).", "",
             "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for k in sorted(per):
        if only_prefix and not k.startswith(only_prefix):
            continue
        vals = []
        for c in names:
            v = per[k].get(c)
            vals.append(f"{_median(v):.4g}" if v else "")
        lines.append(f"| `{k}` | " + " | ".join(vals) + " |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_counters_summary(path):
    """{kernel: {counter: mean per dispatch}} and the recorded sources hash."""
    info = {"kernels": {}}
    names = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("sweep_sources_sha256:"):
                info["sweep_sources_sha256"] = line.split(":", 1)[1].strip()
            elif line.startswith("| kernel |"):
                names = [c.strip() for c in line.strip("|").split("|")][1:]
            elif names and line.startswith("| `"):
                cells = [c.strip() for c in line.strip("|").split("|")]
                k = cells[0].strip("`")
                info["kernels"][k] = {n: float(v) for n, v in zip(names, cells[1:]) if v}
    return info


def read_traffic_summary(path):
    info = {"bytes_per_launch": {}}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("sweep_sources_sha256:"):
                info["sweep_sources_sha256"] = line.split(":", 1)[1].strip()
            elif line.startswith("bytes_per_launch "):
                k, v = line[len("bytes_per_launch "):].rsplit(":", 1)
                info["bytes_per_launch"][k.strip()] = float(v)
    return info


def main(argv):
    if len(argv) >= 3 and argv[0] == "stats":
        write_stats(argv[1], argv[2], " ".join(argv[3:]))
    elif len(argv) >= 5 and argv[0] == "counters" and "--" in argv:
        j = argv.index("--")
        write_counters(argv[1], argv[2], argv[3:j], " ".join(argv[j + 1:]))
    elif len(argv) >= 5 and argv[0] == "dispatches":
        write_dispatches(argv[1], argv[2], argv[3], int(argv[4]), " ".join(argv[5:]))
    elif len(argv) >= 6 and argv[0] == "traffic":
        write_traffic(argv[1], argv[2], int(argv[3]), int(argv[4]), argv[5], " ".join(argv[6:]))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
