"""Summaries of rocprofv3 output for the tFFR kernels.

    python -m paper_1910_10908_amd.profiling trace <rocprofv3 -d dir>
        per-kernel calls / average / total duration from a --kernel-trace --stats run
    python -m paper_1910_10908_amd.profiling traffic <fetch dir> <write dir> --kernel NAME
        HBM bytes per dispatch of kernel NAME from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for the
        plain copy kernel (__amd_rocclr_copyBuffer) of known size the run also launched;
        prints key: value lines that bench.py reads back (with the kernel-source hash, so a
        changed kernel is not reported with stale counters).
    python -m paper_1910_10908_amd.profiling counters <pmc dir> [<pmc dir> ...] --kernel NAME
        per-dispatch means of every SQ / GRBM counter the runs collected for kernel NAME,
        and the compute ceilings they give (same key: value format):
        with C = the dispatch's duration (its trace timestamps) times the published 2.4 GHz
        clock, the fraction of each unit's peak the kernel used:
          valu_busy   = SQ_ACTIVE_INST_VALU / (CUs * C)   (quad-cycles per CU-cycle: the share
                        of SIMD cycles issuing vector ALU work)
          valu_issue  = 4 (SQ_INSTS_VALU + 3 SQ_INSTS_VALU_TRANS_F32 + 3 SQ_INSTS_VALU_TRANS_F64)
                        / (4 CUs * C)   (wave64 instructions at 4 cycles each on a 16-lane SIMD,
                        transcendentals at a quarter rate)
          lds_util    = SQ_LDS_IDX_ACTIVE / (CUs * C)   (LDS busy share per CU)
          lds_conflict_share = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE
          occupancy   = 4 SQ_WAVE_CYCLES / (32 CUs * C)  (resident waves over the 32 slots)
          gui_clock_GHz = GRBM_GUI_ACTIVE / 8 / duration (the CSV sums the 8 XCDs)
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
                                                  "tffr_coord.hip", "tffr_ffr.hip", "tffr_misc.hip")]
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
    lines.append(f"source_hash: {kernel_source_hash()}")
    return "\n".join(lines)


def read_trace_avg(path, kernel):
    """Average traced duration (us) of `kernel` (name up to its template list) in a committed
    kernel-trace summary, and the summary's kernel-source hash: (avg_us or None, hash or None)."""
    avg, src = None, None
    if not os.path.exists(path):
        return avg, src
    with open(path) as f:
        for line in f:
            if line.startswith("source_hash:"):
                src = line.split(":", 1)[1].strip()
            elif line.startswith(f"tffr::{kernel}<"):
                avg = float(line[72:].split()[1])
    return avg, src


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


CU_NUM = 256
XCD_NUM = 8
PEAK_CLOCK_GHZ = 2.4


def counters(dirs, kernel):
    """Per-dispatch means of the counters in one or more --pmc runs for kernel NAME, and the
    derived compute fractions (see the module docstring)."""
    vals = {}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise FileNotFoundError(f"no counter_collection.csv under {d}")
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        dur = {}
        for r in csv.DictReader(open(files[0])):
            if kernel not in _short(r["Kernel_Name"]):
                continue
            per[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
            dur[r["Dispatch_Id"]] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
            for key in ("VGPR_Count", "SGPR_Count", "LDS_Block_Size", "Workgroup_Size", "Grid_Size", "Scratch_Size"):
                vals.setdefault(key, float(r[key]))
        for cname, disp in per.items():
            v = sum(disp.values()) / len(disp)
            # GRBM_GUI_ACTIVE is collected in every pass: keep the first
            vals.setdefault(cname, v)
        if dur:
            vals.setdefault("dispatch_ns", sum(dur.values()) / len(dur))
    if not vals:
        raise KeyError(f"{kernel}: no dispatches")
    out = {"kernel": kernel}
    out.update({k: vals[k] for k in sorted(vals)})
    # capacity: the kernel's dispatch duration at the published 2.4 GHz clock (the peak the
    # fractions are quoted against).  The CSV's GRBM_GUI_ACTIVE sums the 8 XCDs' graphics
    # blocks; an eighth of it over the duration is the clock the kernel actually ran at.
    cyc = vals.get("dispatch_ns", 0.0) * PEAK_CLOCK_GHZ
    if vals.get("GRBM_GUI_ACTIVE") and vals.get("dispatch_ns"):
        out["gui_clock_GHz"] = vals["GRBM_GUI_ACTIVE"] / XCD_NUM / vals["dispatch_ns"]
    if cyc:
        if "SQ_ACTIVE_INST_VALU" in vals:
            out["valu_busy"] = vals["SQ_ACTIVE_INST_VALU"] / (CU_NUM * cyc)
        if "SQ_INSTS_VALU" in vals:
            trans = vals.get("SQ_INSTS_VALU_TRANS_F32", 0.0) + vals.get("SQ_INSTS_VALU_TRANS_F64", 0.0)
            out["valu_issue"] = 4.0 * (vals["SQ_INSTS_VALU"] + 3.0 * trans) / (4.0 * CU_NUM * cyc)
        if "SQ_LDS_IDX_ACTIVE" in vals:
            out["lds_util"] = vals["SQ_LDS_IDX_ACTIVE"] / (CU_NUM * cyc)
            if vals["SQ_LDS_IDX_ACTIVE"] > 0 and "SQ_LDS_BANK_CONFLICT" in vals:
                out["lds_conflict_share"] = vals["SQ_LDS_BANK_CONFLICT"] / vals["SQ_LDS_IDX_ACTIVE"]
        if "SQ_WAVE_CYCLES" in vals:
            out["occupancy"] = 4.0 * vals["SQ_WAVE_CYCLES"] / (32.0 * CU_NUM * cyc)
    out["source_hash"] = kernel_source_hash()
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
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_summary(a.dir, a.only))
    elif a.cmd == "counters":
        for k, v in counters(a.dirs, a.kernel).items():
            print(f"{k}: {v}")
    else:
        for k, v in traffic(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes).items():
            print(f"{k}: {v}")


if __name__ == "__main__":
    sys.exit(main())
