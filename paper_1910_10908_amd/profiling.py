"""Summaries of rocprofv3 output for the tFFR kernels.

    python -m paper_1910_10908_amd.profiling trace <rocprofv3 -d dir>
        per-kernel calls / average / total duration from a --kernel-trace --stats run
    python -m paper_1910_10908_amd.profiling traffic <fetch dir> <write dir> --kernel NAME
        HBM bytes per dispatch of kernel NAME from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the
        plain copy kernel (__amd_rocclr_copyBuffer) of known size the run also launched;
        prints key: value lines that bench.py reads back (with the kernel-source hash, so a
        changed kernel is not reported with stale counters).
"""

import argparse
import collections
import csv
import glob
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in
                  ("tffr_device.h", "tffr_range.hip", "tffr_azimuth.hip", "tffr_entstep.hip",
                                                  "tffr_coord.hip", "tffr_misc.hip")]
COPY_BYTES = 64 << 20  # the calibration copy bench.py --profile-steps launches


def kernel_source_hash():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name):
    return name.split("(")[0].replace("void ", "").strip()


def trace_table(path):
    dbs = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    con = sqlite3.connect(dbs[0])
    rows = con.execute("select name, total_calls, average, total_duration from top_kernels").fetchall()
    return [(_short(n), c, a, t) for n, c, a, t in rows]


def trace_summary(path, only=None):
    lines = [f"{'kernel':72s} {'calls':>6s} {'avg_us':>10s} {'total_us':>12s}"]
    for n, c, a, t in trace_table(path):
        if only and not any(o in n for o in only):
            continue
        lines.append(f"{n[:72]:72s} {c:6d} {a:10.3f} {t:12.1f}")
    return "\n".join(lines)


def _pmc_dispatches(path, counter):
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {path}")
    per = collections.defaultdict(dict)
    for r in csv.DictReader(open(files[0])):
        if r["Counter_Name"] != counter:
            continue
        key = (_short(r["Kernel_Name"]), r["Dispatch_Id"])
        per[key][counter] = per[key].get(counter, 0.0) + float(r["Counter_Value"])
    out = collections.defaultdict(list)
    for (name, _), v in per.items():
        out[name].append(v[counter])
    return out


def traffic(fetch_dir, write_dir, kernel, copy_bytes=COPY_BYTES):
    fetch = _pmc_dispatches(fetch_dir, "FETCH_SIZE")
    write = _pmc_dispatches(write_dir, "WRITE_SIZE")

    def pick(d, sub, reduce):
        keys = [k for k in d if sub in k]
        if not keys:
            raise KeyError(f"{sub} not in {sorted(d)}")
        return reduce(d[keys[0]])

    mean = lambda v: sum(v) / len(v)  # noqa: E731
    # the calibration copy is the largest copyBuffer dispatch of the run
    copy_f = pick(fetch, "copyBuffer", max)
    copy_w = pick(write, "copyBuffer", max)
    f_scale = copy_bytes / (copy_f * 1024.0)
    w_scale = copy_bytes / (copy_w * 1024.0)
    kf = pick(fetch, kernel, mean) * 1024.0 * f_scale
    kw = pick(write, kernel, mean) * 1024.0 * w_scale
    return {"kernel": kernel, "fetch_bytes": kf, "write_bytes": kw, "traffic_bytes": kf + kw,
            "copy_fetch_scale": f_scale, "copy_write_scale": w_scale, "source_hash": kernel_source_hash()}


def read_traffic(path):
    """key: value lines written by `traffic` (bench.py reads them back)."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--only", nargs="*")
    p = sub.add_parser("traffic")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("--kernel", required=True)
    p.add_argument("--copy-bytes", type=int, default=COPY_BYTES)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_summary(a.dir, a.only))
    else:
        for k, v in traffic(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes).items():
            print(f"{k}: {v}")


if __name__ == "__main__":
    sys.exit(main())
