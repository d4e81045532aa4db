"""Summaries of rocprofv3 output for the committed profiles.

    python profile_summary.py stats <prefix>_kernel_stats.csv [--top 20]
    python profile_summary.py trace <prefix>_kernel_trace.csv
        --kernel <name substring> --last N
    python profile_summary.py step <prefix>_kernel_trace.csv
        --marker <name substring of a step's last kernel>
    python profile_summary.py traffic --fetch <fetch counter csv>
        --write <write counter csv> --kernel <name substring> --last N [--copy-mib 256]

`trace` prints the average duration of the last N dispatches of one kernel in a kernel trace.
`step` prints the kernels of one step: the dispatches after the second-to-last dispatch of the
marker kernel (the step's last kernel) up to and including the last one, grouped by name.
`stats` prints the kernel table (calls, average and total duration, share) of a
`rocprofv3 --kernel-trace --stats --output-format csv` run. `traffic` reads two
`rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of profile_run.py (KiB per dispatch), takes
the last N dispatches of the named kernel, and scales each counter by the ratio of the known bytes of
the final plain device copy (copy-mib MiB read and written) to what the same counter read for it.
"""
from __future__ import annotations

import argparse
import csv
import json
import sys
from typing import Dict, List


def _rows(path: str) -> List[Dict[str, str]]:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats(path: str, top: int) -> None:
    rows = _rows(path)
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| Kernel | Calls | Avg (us) | Total (ms) | % |")
    print("|---|---:|---:|---:|---:|")
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        t = float(r["TotalDurationNs"])
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {t / 1e6:.2f} | "
              f"{100 * t / total:.1f} |")


def trace(path: str, kernel: str, last: int) -> None:
    ds = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    ds.sort(key=lambda r: int(r["Dispatch_Id"]))
    ds = ds[-last:]
    if len(ds) < last:
        sys.exit(f"only {len(ds)} dispatches of {kernel!r}")
    dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in ds]
    print(f"Kernel `{ds[-1]['Kernel_Name']}`: last {last} dispatches, average "
          f"{sum(dur) / len(dur) / 1e6:.4f} ms (min {min(dur) / 1e6:.4f}, max {max(dur) / 1e6:.4f}).")


def step(path: str, marker: str) -> None:
    ds = sorted(_rows(path), key=lambda r: int(r["Dispatch_Id"]))
    ends = [k for k, r in enumerate(ds) if marker in r["Kernel_Name"]]
    if len(ends) < 2:
        sys.exit(f"fewer than two dispatches of {marker!r}")
    one = ds[ends[-2] + 1:ends[-1] + 1]
    groups: Dict[str, List[int]] = {}
    for r in one:
        groups.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in groups.values())
    print("| Kernel | Launches | Total (us) | % |")
    print("|---|---:|---:|---:|")
    for name, v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        print(f"| `{name.replace('|', '/')}` | {len(v)} | {sum(v) / 1e3:.1f} | {100 * sum(v) / total:.1f} |")
    print(f"| all | | {total / 1e3:.1f} | 100 |")
    span = int(one[-1]["End_Timestamp"]) - int(one[0]["Start_Timestamp"])
    print(f"\nSum of kernel durations {total / 1e3:.1f} us; first start to last end {span / 1e3:.1f} us.")


def _dispatches(path: str, counter: str) -> List[Dict[str, object]]:
    out = []
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        out.append({"id": int(r["Dispatch_Id"]), "name": r["Kernel_Name"],
                    "kib": float(r["Counter_Value"])})
    out.sort(key=lambda d: d["id"])
    return out


def traffic(fetch: str, write: str, kernel: str, last: int, copy_mib: int) -> None:
    res = {}
    for counter, path in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
        ds = _dispatches(path, counter)
        copies = [d for d in ds if "copyBuffer" in str(d["name"])]
        if not copies:
            sys.exit(f"no copy dispatch in {path}")
        cal = copies[-1]["kib"] * 1024.0
        factor = copy_mib * 2**20 / cal
        ks = [d for d in ds if kernel in str(d["name"])][-last:]
        if len(ks) < last:
            sys.exit(f"only {len(ks)} dispatches of {kernel!r} in {path}")
        raw = sum(d["kib"] for d in ks) / len(ks) * 1024.0
        res[counter] = {"raw_bytes_per_dispatch": raw, "copy_raw_bytes": cal, "factor": factor,
                        "bytes_per_dispatch": raw * factor, "kernel": ks[-1]["name"],
                        "dispatches": len(ks)}
    tot = res["FETCH_SIZE"]["bytes_per_dispatch"] + res["WRITE_SIZE"]["bytes_per_dispatch"]
    print("| Counter | Raw (MB per dispatch) | Copy calibration (raw MB for "
          f"{copy_mib} MiB) | Factor | HBM (MB per dispatch) |")
    print("|---|---:|---:|---:|---:|")
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        r = res[c]
        print(f"| {c} | {r['raw_bytes_per_dispatch'] / 1e6:.1f} | {r['copy_raw_bytes'] / 1e6:.1f} | "
              f"{r['factor']:.3f} | {r['bytes_per_dispatch'] / 1e6:.1f} |")
    print(f"\nKernel: `{res['FETCH_SIZE']['kernel']}`, last {last} dispatches; "
          f"traffic {tot / 1e6:.1f} MB per dispatch.\n")
    print("JSON: " + json.dumps({"kernel": res["FETCH_SIZE"]["kernel"], "bytes_per_launch": tot,
                                 "fetch_factor": res["FETCH_SIZE"]["factor"],
                                 "write_factor": res["WRITE_SIZE"]["factor"]}))


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=20)
    r = sub.add_parser("trace")
    r.add_argument("csv")
    r.add_argument("--kernel", required=True)
    r.add_argument("--last", type=int, required=True)
    st = sub.add_parser("step")
    st.add_argument("csv")
    st.add_argument("--marker", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--last", type=int, required=True)
    t.add_argument("--copy-mib", type=int, default=256)
    a = ap.parse_args()
    if a.cmd == "stats":
        stats(a.csv, a.top)
    elif a.cmd == "trace":
        trace(a.csv, a.kernel, a.last)
    elif a.cmd == "step":
        step(a.csv, a.marker)
    else:
        traffic(a.fetch, a.write, a.kernel, a.last, a.copy_mib)


if __name__ == "__main__":
    main()
