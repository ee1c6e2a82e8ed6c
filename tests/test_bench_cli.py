"""bench.py on the host: more than one GPU is refused with a message before anything
touches a device, and the committed trace summaries it reads are current."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_trace_summaries_parse_and_match_kernel_sources():
    """Every committed kernel-trace summary names the kernel sources it was taken on, and the
    bench can read the step kernels' traced durations from it."""
    from paper_1910_10908_amd import profiling

    for wl in ("ffr_vs_tffr_c64", "full_swath_4k"):
        path = os.path.join(ROOT, "profiles", f"kernel_trace_{wl}.md")
        for k in ("k_fwd_rows_run", "k_ent_cols", "k_adj_rows"):
            us, src = profiling.read_trace_avg(path, k)
            assert us is not None and us > 0, (wl, k)
            assert src == profiling.kernel_source_hash(), (wl, src)
    assert profiling.read_trace_avg(os.path.join(ROOT, "profiles", "missing.md"), "k_ent_cols") == (None, None)
