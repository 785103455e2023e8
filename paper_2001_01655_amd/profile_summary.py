"""Summaries of rocprofv3 output for the benchmark's profiles.

    python -m paper_2001_01655_amd.profile_summary stats  <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2001_01655_amd.profile_summary traffic <fetch_counter_collection.csv> \
           <write_counter_collection.csv> <out_dir> "<command>" <smoother> <sweeps>
    python -m paper_2001_01655_amd.profile_summary units <counter_collection.csv> <out.md> "<command>" "<title>"

`stats` writes the per-kernel time table.  `traffic` turns FETCH_SIZE and
WRITE_SIZE (KiB per dispatch) into HBM bytes per launch for the benchmark's
kernel classes, scaling each counter by what it reads for the benchmark's
256 MiB device-to-device copy (known bytes read and written).  `units`
tabulates any other counters (VALU and matrix-core activity, occupancy) as
the mean per launch of each kernel class.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20
CLASSES = {
    0: dict(match=["k_fine3sf64<3, 1>"], source=["kernels_fine.hip", "tm_device.h"],
            what="fine operator FP64, tensor-product form (q = K~p, outer loop)"),
    1: dict(match=["k_fine3sf<1, 1>", "k_fine3sf<2, 1>", "k_fine3sf<4, 1>", "k_fine3sf_pro<2, 1>",
                   "k_fine3sf_pro<4, 1>"],
            source=["kernels_fine.hip", "tm_device.h"],
            what="fine operator FP32, tensor-product form (V-cycle smoothing / residual; the first "
                 "post-smoothing step takes the prolongation in it)"),
    2: dict(match=["k_stencil_op<float, 3, 1, 4, 1>", "k_stencil_op<float, 3, 2, 4, 1>",
                   "k_stencil_op<float, 3, 4, 4, 1>"],
            source=["kernels_coarse.hip", "tm_device.h"], what="level-1 stencil operator FP32 (V-cycle)",
            largest_grid=True),
    3: dict(match=["k_fine3z2_mfma<1, 1>", "k_fine3z2_mfma<2, 1>", "k_fine3z2_mfma<4, 1>"],
            source=["kernels_fine.hip", "tm_device.h"],
            what="fine operator FP32 on the matrix cores (option fine_mfma)"),
    4: dict(match=["k_fine3z2<float, 1, 1>", "k_fine3z2<float, 2, 1>", "k_fine3z2<float, 4, 1>"],
            source=["kernels_fine.hip", "tm_device.h"],
            what="fine operator FP32, node gather (option fine_tensor = 0)"),
}


def _short(name: str) -> str:
    n = name.split("(")[0]
    return n.replace("void ", "").replace("tmi::", "")


def stats(path: str, out: str, command: str) -> None:
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# Kernel time summary", "", f"Command: `{command}`", "",
             f"Total kernel time: {tot / 1e6:.3f} ms", "",
             "| kernel | calls | avg us | total ms | share |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f}% |")
    open(out, "w").write("\n".join(lines) + "\n")


def _per_dispatch(path: str):
    rows = list(csv.DictReader(open(path)))
    return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"]) * 1024.0) for r in rows]


def traffic(fetch_csv: str, write_csv: str, out_dir: str, command: str, smoother: str, sweeps: int) -> None:
    fe, wr = _per_dispatch(fetch_csv), _per_dispatch(write_csv)
    cf = max((v for n, g, v in fe if "copyBuffer" in n), default=None)
    cw = max((v for n, g, v in wr if "copyBuffer" in n), default=None)
    if not cf or not cw:
        raise SystemExit("no calibration copy found (run the benchmark with --calibrate-copy)")
    kf, kw = COPY_BYTES / cf, COPY_BYTES / cw
    summary = [f"# HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
               f"Command (one run per counter): `{command}`", "",
               f"Calibration: a 256 MiB device copy reads as {cf / 2**20:.1f} MiB fetched and "
               f"{cw / 2**20:.1f} MiB written; factors {kf:.4f} (fetch) and {kw:.4f} (write).", "",
               "| class | kernel | launches | fetch MB | write MB | calibrated MB/launch |", "|---|---|---:|---:|---:|---:|"]
    for c, spec in CLASSES.items():
        sel = lambda rows: [(n, g, v) for n, g, v in rows if any(m in n for m in spec["match"])]
        f_rows, w_rows = sel(fe), sel(wr)
        if spec.get("largest_grid") and f_rows:
            g = max(gg for _, gg, _ in f_rows)
            f_rows = [r for r in f_rows if r[1] == g]
            w_rows = [r for r in w_rows if r[1] == g]
        if not f_rows or not w_rows:
            continue
        fb = sum(v for _, _, v in f_rows) / len(f_rows)
        wb = sum(v for _, _, v in w_rows) / len(w_rows)
        per = fb * kf + wb * kw
        h = hashlib.sha256()
        for n in spec["source"]:
            h.update(open(os.path.join(HERE, "csrc", n), "rb").read())
        rec = {"class": c, "kernel": spec["what"], "kernels": spec["match"], "launches": len(f_rows),
               "fetch_bytes_raw": fb, "write_bytes_raw": wb, "fetch_factor": kf, "write_factor": kw,
               "bytes_per_launch": per, "source": spec["source"],
               "source_sha": h.hexdigest()[:16], "mix": [smoother, sweeps], "command": command}
        json.dump(rec, open(os.path.join(out_dir, f"traffic_class{c}.json"), "w"), indent=1)
        summary.append(f"| {c} | {spec['what']} | {len(f_rows)} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {per / 1e6:.1f} |")
    open(os.path.join(out_dir, "traffic_cantilever3d.md"), "w").write("\n".join(summary) + "\n")


def units(path: str, out: str, command: str, title: str) -> None:
    rows = list(csv.DictReader(open(path)))
    names = sorted({r["Counter_Name"] for r in rows})
    lines = [f"# {title}", "", f"Command: `{command}`", "", "Mean per launch of each counter (rocprofv3 `--pmc`).",
             "", "| class | kernel | launches | " + " | ".join(names) + " |",
             "|---|---|---:|" + "---:|" * len(names)]
    for c, spec in CLASSES.items():
        sel = [r for r in rows if any(m in r["Kernel_Name"] for m in spec["match"])]
        if spec.get("largest_grid") and sel:
            g = max(int(r["Grid_Size"]) for r in sel)
            sel = [r for r in sel if int(r["Grid_Size"]) == g]
        if not sel:
            continue
        vals = collections.defaultdict(list)
        for r in sel:
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
        launches = max(len(v) for v in vals.values())
        cells = [f"{sum(vals[n]) / len(vals[n]):.4g}" if vals[n] else "" for n in names]
        lines.append(f"| {c} | {spec['what']} | {launches} | " + " | ".join(cells) + " |")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], int(sys.argv[7]))
    elif sys.argv[1] == "units":
        units(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        raise SystemExit(__doc__)
