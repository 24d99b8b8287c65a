"""rocprofv3 summaries for the solver's kernels: per-kernel times, HBM traffic.

HBM traffic of a kernel comes from two counter runs of the same command
(FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Each counter is scaled by
the ratio of the bytes a plain copy kernel of known size moves to what the
same counter reports for it (``bench.py --workload copy``), which calibrates
the counter's units on this device.  The stored summary carries a fingerprint
of the sources that define the kernels; ``bench.py`` reports the traffic only
while the sources still match.

Usage (after the rocprofv3 runs, on their CSV output):
  python -m paper_1701_04685_amd.profiling stats  RUN_kernel_stats.csv TITLE COMMAND > out.txt
  python -m paper_1701_04685_amd.profiling traffic --kernel NAME --fetch F.csv --write W.csv
         --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N --commands CMDS --out profiles/X
  python -m paper_1701_04685_amd.profiling passes --spec KERNEL=LABEL=READ=WRITE [--spec ...]
         --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N
         --title T --commands CMDS --out profiles/X
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# The files that hold the solver's device code, and the build script whose
# flags compile it.  lsh_solver.hip is host code only (it instantiates the
# kernel templates, whose arguments are part of the kernel's name, and
# launches them), so a change to its scheduling leaves the fingerprint alone.
KERNEL_SOURCES = ["csrc/lsh_kernels.hpp", "csrc/lsh_common.hpp", "csrc/lsh_fft.hpp", "csrc/lsh_green.hpp",
                  "csrc/lsh_twopass.hpp", "csrc/lsh_twopass.hip", "build.py"]


def source_fingerprint() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def kernel_stats_table(csv_path: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", "", f"command: {command}", "",
           f"{'kernel':60s} {'calls':>6s} {'avg us':>10s} {'total %':>8s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"{_short(r['Name'])[:60]:60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{100 * float(r['TotalDurationNs']) / tot:8.2f}")
    return "\n".join(out) + "\n"


def counter_kib(csv_path: str, counter: str, kernel: str):
    """Per-dispatch values (KiB) of `counter` for dispatches whose name contains `kernel`."""
    vals = []
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    return vals


def traffic_summary(kernel, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, commands):
    copy_name = "elementwise"
    cf = statistics.median(counter_kib(copy_fetch_csv, "FETCH_SIZE", copy_name)[1:])
    cw = statistics.median(counter_kib(copy_write_csv, "WRITE_SIZE", copy_name)[1:])
    kf = counter_kib(fetch_csv, "FETCH_SIZE", kernel)
    kw = counter_kib(write_csv, "WRITE_SIZE", kernel)
    fscale = copy_bytes / (cf * 1024.0)
    wscale = copy_bytes / (cw * 1024.0)
    fetch = statistics.median(kf) * 1024.0 * fscale
    write = statistics.median(kw) * 1024.0 * wscale
    return {"kernel": kernel, "fingerprint": source_fingerprint(), "dispatches": [len(kf), len(kw)],
            "fetch_kib_median": statistics.median(kf), "write_kib_median": statistics.median(kw),
            "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes_each_way": copy_bytes,
            "fetch_scale": fscale, "write_scale": wscale,
            "fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write, "commands": commands}


def pass_traffic_table(specs, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, title, commands):
    """Counted HBM traffic of several kernels of one run against their algorithmic
    bytes.  specs: (kernel name substring, label, algorithmic read bytes,
    algorithmic write bytes) per kernel.  Every kernel's counters are scaled by
    the same copy calibration, so kernels whose bytes are known exactly (the
    axis-2 passes read and write the state once) test that calibration on
    access patterns other than the copy's."""
    base = traffic_summary("elementwise", copy_fetch_csv, copy_write_csv, copy_fetch_csv, copy_write_csv,
                           copy_bytes, commands)
    fs, ws = base["fetch_scale"], base["write_scale"]
    out = [f"# {title}", "", "Commands (FETCH_SIZE run, WRITE_SIZE run, copy calibration runs):", "", "```",
           commands, "```", "",
           f"Copy calibration ({copy_bytes:.0f} B each way): FETCH_SIZE x {fs:.4f}, WRITE_SIZE x {ws:.4f}.",
           "Counted = the median dispatch's counter value times that scale; alg. = the bytes the pass must",
           "read and write (the state, the phase map, the previous iterate).", "",
           f"{'kernel':40s} {'pass':24s} {'n':>3s} {'read GB':>8s} {'alg.':>7s} {'ratio':>6s} "
           f"{'write GB':>8s} {'alg.':>7s} {'ratio':>6s}"]
    rows = []
    for kern, label, ar, aw in specs:
        kf = counter_kib(fetch_csv, "FETCH_SIZE", kern)
        kw = counter_kib(write_csv, "WRITE_SIZE", kern)
        if not kf or not kw:
            continue
        rd = statistics.median(kf) * 1024.0 * fs
        wr = statistics.median(kw) * 1024.0 * ws
        rows.append({"kernel": kern, "pass": label, "dispatches": [len(kf), len(kw)], "read_bytes": rd,
                     "write_bytes": wr, "alg_read_bytes": ar, "alg_write_bytes": aw})
        out.append(f"{kern[:40]:40s} {label[:24]:24s} {len(kf):3d} {rd / 1e9:8.4f} {ar / 1e9:7.4f} {rd / ar:6.3f} "
                   f"{wr / 1e9:8.4f} {aw / 1e9:7.4f} {wr / aw:6.3f}")
    out += ["", f"source fingerprint {source_fingerprint()}", ""]
    return "\n".join(out), {"title": title, "fingerprint": source_fingerprint(), "fetch_scale": fs,
                             "write_scale": ws, "rows": rows, "commands": commands}


def load_traffic(kernel_substr: str, profiles_dir: str = os.path.join(ROOT, "profiles")):
    """Stored traffic (bytes per launch) for a kernel, or None if absent or stale."""
    if not os.path.isdir(profiles_dir):
        return None
    fp = source_fingerprint()
    for f in sorted(os.listdir(profiles_dir)):
        if not f.endswith("_traffic.json"):
            continue
        d = json.load(open(os.path.join(profiles_dir, f)))
        if kernel_substr in d.get("kernel", "") and d.get("fingerprint") == fp:
            return d
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("title")
    s.add_argument("command")
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--commands", required=True)
    t.add_argument("--out", required=True, help="path prefix: writes PREFIX_traffic.json and PREFIX_traffic.md")
    pt = sub.add_parser("passes", help="counted vs algorithmic bytes of several kernels of one run")
    pt.add_argument("--spec", action="append", required=True,
                    help="KERNEL_SUBSTRING=LABEL=ALG_READ_BYTES=ALG_WRITE_BYTES (repeat per kernel)")
    for k in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--title", "--commands", "--out"):
        pt.add_argument(k, required=True)
    pt.add_argument("--copy-bytes", type=float, required=True)
    a = ap.parse_args()
    if a.cmd == "passes":
        specs = []
        for sp in a.spec:
            kern, label, ar, aw = sp.split("=")
            specs.append((kern, label, float(ar), float(aw)))
        text, d = pass_traffic_table(specs, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.title,
                                     a.commands)
        with open(a.out + ".md", "w") as fh:
            fh.write(text)
        with open(a.out + ".json", "w") as fh:
            json.dump(d, fh, indent=1)
        return
    if a.cmd == "stats":
        print(kernel_stats_table(a.csv, a.title, a.command), end="")
        return
    d = traffic_summary(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.commands)
    with open(a.out + "_traffic.json", "w") as fh:
        json.dump(d, fh, indent=1)
    lines = [f"# HBM traffic per launch: {a.kernel}", "",
             "Commands (FETCH_SIZE run, WRITE_SIZE run, copy calibration runs):", "", "```", a.commands, "```", "",
             f"- kernel FETCH_SIZE median {d['fetch_kib_median']:.1f} KiB, WRITE_SIZE median "
             f"{d['write_kib_median']:.1f} KiB over {d['dispatches']} dispatches",
             f"- copy kernel ({a.copy_bytes:.0f} B each way): FETCH_SIZE {d['copy_fetch_kib']:.1f} KiB, "
             f"WRITE_SIZE {d['copy_write_kib']:.1f} KiB -> scale {d['fetch_scale']:.4f} (fetch), "
             f"{d['write_scale']:.4f} (write)",
             f"- traffic: read {d['fetch_bytes'] / 1e9:.4f} GB + write {d['write_bytes'] / 1e9:.4f} GB = "
             f"{d['traffic_bytes'] / 1e9:.4f} GB per launch",
             f"- source fingerprint {d['fingerprint']}", ""]
    with open(a.out + "_traffic.md", "w") as fh:
        fh.write("\n".join(lines))


if __name__ == "__main__":
    main()
