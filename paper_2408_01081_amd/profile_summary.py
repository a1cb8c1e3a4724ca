"""Summaries of rocprofv3 output (CSV) for the lattice kernels.

  traffic: HBM bytes per launch of one kernel from two counter runs
      (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
      same counter reads for the plain copy kernel k_copy of known size in the
      same run; one entry per launch configuration in the output file;
  stats:   the per-kernel table of a --kernel-trace --stats run (with
      --by-grid, also per launch grid of the matching kernels).

    python -m paper_2408_01081_amd.profile_summary traffic \\
        --fetch DIR --write DIR --match 'k_tblock<0, 0, 1, 7>' --copy-bytes 2684354560 \\
        --algorithmic-bytes 2684354560 --kernel 'description' --kname k_tblock \\
        --launch 'T=7 seg=48 nt=0 pf=1' \\
        --command CMD --command CMD --out profiles/NAME.json
    python -m paper_2408_01081_amd.profile_summary stats --dir DIR --title T \\
        --command CMD --note LINE [--only k_batch] --out profiles/NAME.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os


def _short(name: str) -> str:
    i = name.find("k_")
    if i < 0:
        return name[:40]
    j = name.find("(", i)
    return name[i:j] if j > 0 else name[i:]


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern))
    if not hits:
        raise SystemExit("no file matches %s" % pattern)
    return hits[0]


def _counter_values(d: str, match: str):
    vals = []
    for r in csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))):
        if match in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit("no dispatch of %r in %s" % (match, d))
    return vals


def traffic(a):
    from . import build as B
    avg = lambda v: sum(v) / len(v)
    f, w = _counter_values(a.fetch, a.match), _counter_values(a.write, a.match)
    cf, cw = _counter_values(a.fetch, "k_copy"), _counter_values(a.write, "k_copy")
    # the copy kernel reads and writes copy_bytes / 2 each
    half = a.copy_bytes / 2 / 1024.0
    fs, ws = half / avg(cf), half / avg(cw)
    rd, wr = avg(f) * fs * 1024, avg(w) * ws * 1024
    out = {
        "kernel": a.kernel, "match": a.match, "launch": a.launch,
        "source_sha256": B.kernel_hash(a.kname),
        "commands": a.command,
        "fetch_kib_per_dispatch": round(avg(f), 2), "write_kib_per_dispatch": round(avg(w), 2),
        "dispatches": [len(f), len(w)],
        "calibration": {"kernel": "k_copy, %d B read + %d B written" % (half * 1024, half * 1024),
                        "fetch_kib_per_dispatch": round(avg(cf), 2),
                        "write_kib_per_dispatch": round(avg(cw), 2),
                        "fetch_scale": round(fs, 6), "write_scale": round(ws, 6)},
        "read_bytes_per_launch": int(rd), "write_bytes_per_launch": int(wr),
        "bytes_per_launch": int(rd + wr),
        "algorithmic_bytes_per_launch": a.algorithmic_bytes,
        "traffic_over_algorithmic": round((rd + wr) / a.algorithmic_bytes, 5),
        "read_over_algorithmic": round(rd / (a.algorithmic_bytes / 2), 5),
        "write_over_algorithmic": round(wr / (a.algorithmic_bytes / 2), 5),
    }
    # one file holds the entries of several launch configurations of the
    # same kernel and workload; an entry for the same launch is replaced
    doc = {"entries": []}
    if os.path.exists(a.out):
        old = json.load(open(a.out))
        doc["entries"] = [e for e in old.get("entries", []) if e.get("launch") != a.launch]
    doc["entries"].append(out)
    json.dump(doc, open(a.out, "w"), indent=1)
    print(json.dumps(out, indent=1))


def _by_grid(d: str, match: str):
    """(kernel, grid) -> durations (ns) of the matching dispatches of a
    --kernel-trace run; grid = workgroups (x, y, z)."""
    out = {}
    for r in csv.DictReader(open(_one(os.path.join(d, "*kernel_trace.csv")))):
        if match not in r["Kernel_Name"]:
            continue
        wg = [int(r["Workgroup_Size_%s" % c]) for c in "XYZ"]
        grid = tuple(int(r["Grid_Size_%s" % c]) // w for c, w in zip("XYZ", wg))
        key = (_short(r["Kernel_Name"]), grid)
        out.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def stats(a):
    rows = list(csv.DictReader(open(_one(os.path.join(a.dir, "*kernel_stats.csv")))))
    lines = ["# " + a.title, "", "Command (repo root, one MI355X, ROCm 7.2):", ""]
    for c in a.command:
        lines.append("    " + c)
    if a.only:
        lines += ["", "Kernels whose names start with %s (share: of all kernel time in the run):"
                  % ", ".join("`%s`" % o for o in a.only)]
    lines += ["", "| kernel | calls | avg (us) | min (us) | max (us) | share |",
              "|---|---|---|---|---|---|"]
    for r in rows:
        if "k_" not in r["Name"]:
            continue
        if a.only and not any(_short(r["Name"]).startswith(o) for o in a.only):
            continue
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.2f%% |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    for m in a.by_grid:
        g = _by_grid(a.dir, m)
        lines += ["", "Dispatches of `%s` by launch grid (workgroups x, y, z):" % m, "",
                  "| kernel | grid | calls | avg (us) | min (us) | max (us) |",
                  "|---|---|---|---|---|---|"]
        for (k, grid), v in sorted(g.items()):
            lines.append("| %s | %s | %d | %.1f | %.1f | %.1f |" % (
                k, "x".join(map(str, grid)), len(v), sum(v) / len(v) / 1e3, min(v) / 1e3,
                max(v) / 1e3))
    if a.note:
        lines.append("")
        lines += ["* " + n for n in a.note]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--match", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--algorithmic-bytes", type=int, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--kname", required=True, choices=["k_tblock", "k_step"])
    t.add_argument("--launch", default="",
                   help="launch configuration the counters belong to, e.g. "
                        "'T=7 seg=48 nt=0 pf=1'")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--note", action="append", default=[])
    s.add_argument("--by-grid", action="append", default=[],
                   help="also list the dispatches of kernels matching this string per "
                        "launch grid (from the kernel trace)")
    s.add_argument("--only", action="append", default=[],
                   help="list only the kernels whose names start with this prefix")
    s.add_argument("--out", required=True)
    a = ap.parse_args()
    traffic(a) if a.what == "traffic" else stats(a)


if __name__ == "__main__":
    main()
