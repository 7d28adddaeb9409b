"""Summaries of rocprofv3 runs of the CG kernels (writes the JSON the bench
reads for its ``traffic`` fields and prints the tables kept under profiles/).

    python3 -m paper_2602_07853_amd.profile_summary counters FETCH_DIR WRITE_DIR INFO_JSON OUT_JSON
    python3 -m paper_2602_07853_amd.profile_summary trace TRACE_DIR
    python3 -m paper_2602_07853_amd.profile_summary busy PMC_DIR [PMC_DIR ...]

``counters``: FETCH_DIR and WRITE_DIR hold the results databases of two
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
``python3 -m paper_2602_07853_amd.profile_hv`` (INFO_JSON is the last line it
printed).  Each counter is scaled by what it reads for profile_hv's final
plain device-to-device copy of known size (FETCH_SIZE and WRITE_SIZE are in
KiB per dispatch), and the per-launch bytes of the fused Hessian-vector
product and of the CG update kernel are the medians over their launches;
OUT_JSON keeps one entry per workload.

``trace``: the kernel dispatches of a ``rocprofv3 --kernel-trace --stats``
run (its results database), as a Markdown table of the top kernels.

``busy``: every counter of one or more ``rocprofv3 --pmc`` runs (for
instance VALUBusy, MfmaUtil, SQ_INSTS_VALU), as a Markdown table of the
median per dispatch of the two CG kernels.
"""
from __future__ import annotations

import glob
import json
import os
import sqlite3
import statistics
import sys


def _db(d):
    files = glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)
    if not files:
        raise SystemExit(f"no rocprofv3 results database under {d}")
    return sqlite3.connect(files[0])


def _counter(d, name):
    """[(kernel name, value)] in dispatch order for one counter."""
    con = _db(d)
    rows = con.execute("select dispatch_id, kernel_name, value from counters_collection "
                       "where counter_name = ? order by dispatch_id", (name,)).fetchall()
    return [(k, float(v)) for _, k, v in rows]


def counters(fetch_dir, write_dir, info_json, out_json):
    info = json.loads(open(info_json).read().strip().splitlines()[-1])
    res = {"workload": info["workload"], "kernel_version": info.get("kernel_version")}
    for cname, d, key in (("FETCH_SIZE", fetch_dir, "copy_bytes_read"),
                          ("WRITE_SIZE", write_dir, "copy_bytes_written")):
        vals = _counter(d, cname)
        copies = [v for k, v in vals if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"{cname}: no copy kernel to calibrate with")
        # profile_hv's 512 MiB copy is the largest copy dispatch of the run
        scale = info[key] / (max(copies) * 1024.0)
        res[f"{cname.lower()}_scale"] = scale
        for label, match in (("hv", "k_hv_fused"), ("update", "k_cg_step")):
            kv = [v for k, v in vals if match in k]
            if not kv:
                continue
            med = statistics.median(kv)
            res[f"{label}_{cname.lower()}_kib_median"] = med
            res[f"{label}_{cname.lower()}_launches"] = len(kv)
            res[f"{label}_{cname.lower()}_bytes"] = med * 1024.0 * scale
    for label in ("hv", "update"):
        f, w = res.get(f"{label}_fetch_size_bytes"), res.get(f"{label}_write_size_bytes")
        res[f"bytes_per_{label}"] = round(f + w) if f is not None and w is not None else None
    res.update({k: info[k] for k in ("active_cells", "active_nodes", "free_dofs", "tangent_cells")
                if k in info})
    # one entry per workload in OUT_JSON
    allres = {}
    if os.path.exists(out_json):
        with open(out_json) as fh:
            allres = json.load(fh)
    allres[res["workload"]] = res
    with open(out_json, "w") as fh:
        json.dump(allres, fh, indent=1)
    print(json.dumps(res, indent=1))


def trace(trace_dir, top=25):
    con = _db(trace_dir)
    rows = con.execute("select name, duration from kernels").fetchall()
    by = {}
    for name, dur in rows:
        short = name.replace("(anonymous namespace)::", "")
        short = short[5:] if short.startswith("void ") else short
        by.setdefault(short.split("(")[0], []).append(dur / 1e3)
    total = sum(sum(v) for v in by.values())
    print("| kernel | calls | total ms | avg us | median us | % |")
    print("|---|---:|---:|---:|---:|---:|")
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]:
        print(f"| `{name}` | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.2f} | "
              f"{statistics.median(v):.2f} | {100 * sum(v) / total:.1f} |")


def busy(dirs):
    rows = {}
    for d in dirs:
        con = _db(d)
        for name, kname, v in con.execute("select counter_name, kernel_name, value from counters_collection"):
            for label, match in (("k_hv_fused", "k_hv_fused"), ("k_cg_step", "k_cg_step")):
                if match in kname:
                    rows.setdefault(name, {}).setdefault(label, []).append(float(v))
    print("| counter | `k_hv_fused` (median per dispatch) | `k_cg_step` (median per dispatch) |")
    print("|---|---:|---:|")
    for name in sorted(rows):
        cells = []
        for label in ("k_hv_fused", "k_cg_step"):
            v = rows[name].get(label)
            cells.append(f"{statistics.median(v):.4g}" if v else "-")
        print(f"| {name} | {cells[0]} | {cells[1]} |")


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "counters" and len(sys.argv) == 6:
        counters(*sys.argv[2:])
    elif len(sys.argv) >= 2 and sys.argv[1] == "trace" and len(sys.argv) == 3:
        trace(sys.argv[2])
    elif len(sys.argv) >= 3 and sys.argv[1] == "busy":
        busy(sys.argv[2:])
    else:
        raise SystemExit(__doc__)
