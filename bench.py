"""Benchmark of the tFFR hot path on one MI355X.

One step = one pass of the whole path over one batch of resident synthetic input:
coordinate prep + tFFR weights and threshold (fused into the range kernels), range
and azimuth gridding + inverse FFTs + deapodisation (forward image), image-entropy
loss and its gradient, and the adjoint with gradients w.r.t. the samples and the
per-pulse phase / along-track errors.  The same step is timed for plain FFR (banded
weights solved inside the step) and plain NUFFT (trapezoid weights) on the same GPU.

Prints one JSON line.  Default workload: 512 x 1024 samples, 1024^2 image (plain FFR vs
tFFR in complex64).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Msamples/s tFFR fwd+adjoint vs plain FFR at rel-L2≤1e-5 vs FP64; HBM %"
HBM_PEAK_GBS = 8000.0
ORACLE_WORKERS = 16  # oracle threads for the accuracy references (the GPU machine's CPU share)


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ffr_vs_tffr_c64")
    ap.add_argument("--width", type=int, default=None, help="kernel width (default: workload's)")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain FFR / NUFFT steps")
    ap.add_argument("--cpu-cols", type=int, default=48, help="image columns in the CPU oracle sample")
    ap.add_argument("--sweep", action="store_true",
                    help="one JSON line per workload: tFFR step, plain NUFFT and plain FFR (where the frame "
                         "product is invertible), accuracy vs the oracle, peak memory, oracle timing")
    ap.add_argument("--no-full-swath", action="store_true", help="skip the 4096 x 8192 leg")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many eager steps of the tFFR path (for profilers) and exit")
    ap.add_argument("--profile-ffr", action="store_true",
                    help="with --profile-steps: steps of plain FFR with D re-solved in every step")
    return ap.parse_args()


class Step:
    """Buffers and launches of one step for one weighting method."""

    def __init__(self, T, plan, samples, phase, dalong, ffr=False, fused=True):
        import torch

        self.T, self.plan, self.s, self.ph, self.da, self.ffr = T, plan, samples, phase, dalong, ffr
        self.fused = fused
        dev = samples.device
        self.img = torch.empty(plan.shape_image, dtype=plan.ctype, device=dev)
        self.gI = torch.empty_like(self.img)
        self.gs = torch.empty(plan.shape_samples, dtype=plan.ctype, device=dev)
        self.D = torch.empty(plan.shape_samples + (2 * plan.params.band_r + 1,), dtype=plan.rtype,
                             device=dev) if ffr else None
        self.loss = torch.empty((), dtype=torch.float64, device=dev)
        self.gph = torch.empty(plan.params.n_pulses, dtype=plan.rtype, device=dev)
        self.gda = torch.empty_like(self.gph)

    def __call__(self):
        T, P = self.T, self.plan
        lib, h, work = P.lib, P.handle, T._ptr(P.work)
        st = T._stream()
        if self.ffr:
            T._lib.check(lib.tffr_weights(h, T._ptr(self.D), work, st))
        if self.fused:
            T._lib.check(lib.tffr_entropy_step(h, T._ptr(self.s), T._ptr(self.ph), T._ptr(self.da), T._ptr(self.D),
                                               T._ptr(self.img), T._ptr(self.loss), T._ptr(self.gs),
                                               T._ptr(self.gph), T._ptr(self.gda), work, st))
            return
        T._lib.check(lib.tffr_forward(h, T._ptr(self.s), T._ptr(self.ph), T._ptr(self.da), T._ptr(self.D),
                                      T._ptr(self.img), work, st))
        T._lib.check(lib.tffr_entropy(h, T._ptr(self.img), T._ptr(self.loss), T._ptr(self.gI), work, st))
        T._lib.check(lib.tffr_adjoint(h, T._ptr(self.gI), T._ptr(self.s), T._ptr(self.ph), T._ptr(self.da),
                                      T._ptr(self.D), T._ptr(self.gs), T._ptr(self.gph), T._ptr(self.gda), work, st))


def time_step(torch, fn, steps, warmup, graph):
    """ms per step: warmup, then `steps` steps bracketed by synchronisations and events."""
    stream = torch.cuda.current_stream()
    runner = fn
    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            fn()  # warm the allocator / attributes outside capture
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=side):
                fn()
        stream.wait_stream(side)
        runner = g.replay
    for _ in range(warmup):
        runner()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        runner()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, runner


def kernel_time(torch, fn, reps=200):
    """Average duration of one launch of fn() (back-to-back launches, events on the stream)."""
    for _ in range(10):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3  # seconds


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """GB/s of a plain device-to-device copy (read + write bytes over its duration): the
    bandwidth a streaming kernel reaches on this GPU, a second denominator beside the
    published HBM peak."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    t = kernel_time(torch, lambda: dst.copy_(src), reps)
    del src, dst
    return 2 * nbytes / t / 1e9


def cpu_baseline(wl, k, ku, s, phase, dalong, cols, threads=None):
    """The FP64 oracle timed on a bounded sample of the same step, scaled to Msamples/s.
    With `threads` the BLAS pool is limited to that many threads for the timed work."""
    if threads is not None:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=threads):
            return _cpu_baseline(wl, k, ku, s, phase, dalong, cols, str(threads))
    return _cpu_baseline(wl, k, ku, s, phase, dalong, cols,
                         os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count()))


def _cpu_baseline(wl, k, ku, s, phase, dalong, cols, threads):
    from oracle import entropy as OE
    from oracle import pipeline as OP

    cpu_model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]["name"]
    except Exception:  # noqa: BLE001 - informational only
        blas = "unknown BLAS"
    prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    rng = np.random.default_rng(5)
    col_idx = np.sort(rng.choice(wl.m, cols, replace=False))
    rows = max(1, int(round(wl.n_pulses * cols / wl.m)))
    row_idx = np.sort(rng.choice(wl.n_pulses, rows, replace=False))
    t0 = time.perf_counter()
    kx, ky, lam, X, Y = prob.geometry()
    w = OP.sample_weights(prob)
    t_w = time.perf_counter() - t0
    t0 = time.perf_counter()
    img_cols = OP.image_columns(prob, s, col_idx, phase, dalong)  # forward on a column subset
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    gI = OE.entropy_grad(img_cols)  # stands in for the full-image loss gradient
    yfull = np.zeros((wl.m, wl.m), complex)
    yfull[col_idx] = gI
    sub = OP.Problem(k=k, ku=ku[row_idx], mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    OP.backward(sub, yfull, s[row_idx], phase[row_idx], dalong[row_idx])  # adjoint on a pulse subset
    t_a = time.perf_counter() - t0
    full = t_w + t_f * wl.m / cols + t_a * wl.n_pulses / rows
    return {
        "value": wl.n_samples / full / 1e6,
        "unit": "Msamples/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"FP64 NumPy oracle on {cpu_model} ({blas} with {threads} threads for the matrix products; "
                   f"NumPy's elementwise exponentials run on one core): weights for all {wl.n_samples} samples "
                   f"({t_w:.2f} s), forward on {cols}/{wl.m} image columns ({t_f:.2f} s), entropy gradient + "
                   f"adjoint on {rows}/{wl.n_pulses} pulses ({t_a:.2f} s); full step extrapolated linearly to "
                   f"{full:.1f} s"),
    }, img_cols, col_idx


def accuracy(got, ref):
    """rel-L2 and peak error (dB of the largest error over the largest reference value)."""
    return {"rel_l2_vs_fp64": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "peak_db": float(20 * np.log10(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))}


def sweep(args):
    """Every workload at its own size and precision: the tFFR entropy step, the plain-NUFFT
    (quadrature) step and the plain-FFR step (weights solved inside the step), each timed
    as the faster of graph replay and eager launches; accuracy of the tFFR image against
    the FP64 oracle on sampled columns; peak device memory of one tFFR step; the oracle's
    own time for the step on the host (bounded sample, extrapolated)."""
    import torch

    from oracle import pipeline as OP
    from paper_1910_10908_amd import scenes
    from paper_1910_10908_amd import tffr as T

    dev = "cuda:0"
    torch.cuda.set_device(0)
    for name in scenes.WORKLOAD_ORDER:
        wl = scenes.WORKLOADS[name]
        dtype = T.C128 if wl.dtype == "c128" else T.C64
        ctype, rtype = (torch.complex128, torch.float64) if dtype == T.C128 else (torch.complex64, torch.float32)
        inp = scenes.make_inputs(wl, device=dev, scene=True)
        k, ku = inp["k"], inp["ku"]
        s = inp["samples"].to(ctype).contiguous()
        ph = torch.zeros(wl.n_pulses, dtype=rtype, device=dev)
        da = torch.zeros_like(ph)
        steps = max(10, min(200, int(4e8 / wl.n_samples)))
        rec = {"workload": name, "n_pulses": wl.n_pulses, "n_freq": wl.n_freq, "image": [wl.m, wl.m],
               "dtype": wl.dtype, "kernel_width": wl.kernel_width, "steps": steps}
        for label, wt in (("tffr", T.W_TFFR), ("plain_nufft_quad", T.W_QUAD), ("plain_ffr", T.W_FFR)):
            prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                                   fov_y=wl.fov, weighting=wt, kernel_width=wl.kernel_width, dtype=dtype)
            try:
                plan = T.Plan(prm, k, ku, dev)
            except RuntimeError as e:
                rec[label] = {"error": str(e)}
                continue
            st = Step(T, plan, s, ph, da, ffr=(wt == T.W_FFR))
            ms_e, _ = time_step(torch, st, steps, 5, graph=False)
            ms_g, _ = time_step(torch, st, steps, 5, graph=True)
            ms = min(ms_e, ms_g)
            rec[label] = {"ms_per_step": ms, "Msamples_per_s": wl.n_samples / (ms * 1e-3) / 1e6,
                          "timing": "hip_graph" if ms_g < ms_e else "eager"}
            if wt == T.W_TFFR:
                rec[label]["range_kernel"] = "k_fwd_rows_run" if plan.range_mode >= 1 else "k_fwd_rows"
                torch.cuda.synchronize()
                torch.cuda.reset_peak_memory_stats()
                st()
                torch.cuda.synchronize()
                rec[label]["peak_device_MiB"] = torch.cuda.max_memory_allocated() / 2 ** 20
                img = st.img.cpu().numpy().astype(np.complex128)
            del plan, st
        img16 = None
        if dtype == T.C64 and wl.name == "precision_2k":
            # the same step on samples stored as two IEEE halves (FP32 arithmetic)
            h = torch.view_as_real(s).to(torch.float16).contiguous()
            prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                                   fov_y=wl.fov, weighting=T.W_TFFR, kernel_width=wl.kernel_width,
                                   dtype=T.C64_FP16IN)
            plan = T.Plan(prm, k, ku, dev)
            st = Step(T, plan, h, ph, da)
            ms_e, _ = time_step(torch, st, steps, 5, graph=False)
            ms_g, _ = time_step(torch, st, steps, 5, graph=True)
            ms = min(ms_e, ms_g)
            rec["tffr_fp16_samples"] = {"ms_per_step": ms, "Msamples_per_s": wl.n_samples / (ms * 1e-3) / 1e6,
                                        "timing": "hip_graph" if ms_g < ms_e else "eager"}
            st()
            torch.cuda.synchronize()
            img16 = st.img.cpu().numpy().astype(np.complex128)
            hr = h.cpu().numpy().astype(np.float64)
            s16 = hr[..., 0] + 1j * hr[..., 1]
            del plan, st, h
        cols = max(2, min(48, int(48 * 524288 / wl.n_samples)))
        s_np = s.cpu().numpy().astype(np.complex128)
        zeros = np.zeros(wl.n_pulses)
        base, ref_cols, col_idx = cpu_baseline(wl, k, ku, s_np, zeros, zeros, cols)
        rec["accuracy"] = dict(accuracy(img[col_idx], ref_cols), sample=f"{len(col_idx)} of {wl.m} image columns")
        rec["cpu_oracle"] = base
        if wl.n_samples <= 524288:
            # the oracle on one core too, for context against the paper's serial timings
            rec["cpu_oracle_1core"] = cpu_baseline(wl, k, ku, s_np, zeros, zeros, cols, threads=1)[0]
        if img16 is not None:
            prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
            ref16 = OP.image_columns(prob, s16, col_idx, zeros, zeros)
            rec["tffr_fp16_samples"]["accuracy_vs_rounded_inputs"] = accuracy(img16[col_idx], ref16)
            rec["tffr_fp16_samples"]["accuracy_vs_fp64_inputs"] = accuracy(img16[col_idx], ref_cols)
        print(json.dumps(rec), flush=True)
        del inp, s, img


def counter_file(name, wl_name, kind):
    """Committed counter summary of kernel `name` at workload `wl_name`, if it was taken on
    the current kernel sources (key: value dict), else {}."""
    from paper_1910_10908_amd import profiling

    tr = profiling.read_traffic(os.path.join(ROOT, "profiles", f"{kind}_{name}_{wl_name}.txt"))
    return tr if tr.get("source_hash") == profiling.kernel_source_hash() else {}


def pass_report(name, us, alg_bytes, wl_name):
    """Time, algorithmic bytes and every ceiling's fraction for one kernel of the step: HBM
    (algorithmic bytes, and counter-measured bytes where the counters are current), VALU
    busy and LDS busy (committed SQ counters); `binding` names the largest."""
    from paper_1910_10908_amd import profiling

    t = us * 1e-6
    rec = {"us": us, "alg_bytes": alg_bytes, "achieved_GBps": alg_bytes / t / 1e9,
           "hbm_frac": alg_bytes / t / 1e9 / HBM_PEAK_GBS}
    tr = counter_file(name, wl_name, "hbm_traffic")
    rec["traffic"] = float(tr["traffic_bytes"]) if "traffic_bytes" in tr else None
    fr = {"hbm": rec["hbm_frac"]}
    if rec["traffic"] is not None:
        fr["hbm_counters"] = rec["traffic"] / t / 1e9 / HBM_PEAK_GBS
    sq = counter_file(name, wl_name, "sq_counters")
    for key, label in (("valu_busy", "valu"), ("lds_util", "lds")):
        if key in sq:
            fr[label] = float(sq[key])
    for key in ("valu_issue", "lds_conflict_share", "occupancy"):
        if key in sq:
            rec[key] = float(sq[key])
    rec["fractions"] = fr
    # the committed rocprofv3 trace of the same workload, where taken on the current sources
    tus, th = profiling.read_trace_avg(os.path.join(ROOT, "profiles", f"kernel_trace_{wl_name}.md"), name)
    if tus is not None and th == profiling.kernel_source_hash():
        rec["us_trace"] = tus
        rec["us_over_trace"] = us / tus
    top = max(fr, key=fr.get)
    rec["binding"] = {"ceiling": "hbm" if top.startswith("hbm") else top, "frac": fr[top]}
    return rec


def alg_bytes_of(name, wl):
    """Algorithmic HBM bytes of one launch of a step kernel (complex64): every input read
    once, every output written once."""
    N, nb, img = wl.n_samples, wl.n_pulses * wl.m, wl.m * wl.m
    return {"k_fwd_rows": 8 * N + 8 * nb,            # samples in, range spectra out
            "k_fwd_rows_run": 8 * N + 8 * nb,
            "k_ent_cols": 8 * nb + 8 * img + 16 * nb,  # spectra in; image, two interleaved fields out
            "k_fwd_cols": 8 * nb + 8 * img,            # spectra in, image out
            "k_adj_cols": 8 * img + 8 * nb,            # image in, spectra cotangent out
            "k_entropy_stats": 0,
            "k_adj_rows": None}.get(name)


def step_passes(T, plan, step, wl, fused, nsteps, step_us):
    """Each launch of the step, in the step's own order, data flow and caches.
    "us_events": the time between HIP events recorded between the step's launches.  Each
    event makes the next launch wait for the previous one's completion to be recorded,
    which adds about the same few microseconds to every launch, so "us" takes the excess
    of their sum over the plain step (`step_us`, no events inside) off every launch in
    equal shares.  "us_marginal": what one more launch adds to the step (plain steps
    against steps that issue that launch twice, events around the loops only); the
    repeated launch finds its inputs in cache, so on small steps it reads low."""
    outs = (step.img, step.loss, step.gs, step.gph, step.gda)
    times_ev = plan.tffr_debug_step_kernel_times(step.s, step.ph, step.da, None, out=outs, nsteps=nsteps)
    times_mg = plan.tffr_debug_step_kernel_marginal_times(step.s, step.ph, step.da, None, out=outs, nsteps=nsteps)
    share = max(0.0, sum(times_ev.values()) - step_us) / len(times_ev)
    out = {}
    for name, us_ev in times_ev.items():
        us = max(us_ev - share, 0.5 * us_ev)
        b = alg_bytes_of(name, wl)
        if name == "k_adj_rows":  # samples in, sample gradient out, plus its spectra input
            b = 16 * wl.n_samples + (16 if fused else 8) * wl.n_pulses * wl.m
        out[name] = pass_report(name, us, b, wl.name) if b else {"us": us}
        out[name]["us_events"] = us_ev
        out[name]["us_marginal"] = times_mg.get(name)
    return out


def oracle_columns(wl, k, ku, s, cols, weighting, thresh_mode=0, user_w=None):
    """The FP64 oracle's image on the columns `cols` (threads over slice ranges)."""
    from oracle import pipeline as OP

    prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov, weighting=weighting,
                      thresh_mode=thresh_mode)
    return OP.image_columns(prob, s, cols, np.zeros(wl.n_pulses), np.zeros(wl.n_pulses), user_w=user_w,
                            workers=ORACLE_WORKERS)


def full_swath_leg(T, torch, steps):
    """The 4096 x 8192 -> 4096^2 step (seeded random phase history; the kernels' work does
    not depend on the values): time, kept count, per-launch times, and the image on two
    sampled columns against the oracle."""
    from paper_1910_10908_amd import scenes

    wl = scenes.WORKLOADS["full_swath_4k"]
    dev = "cuda:0"
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    s_np = scenes.random_samples(wl.n_pulses, wl.n_freq, 4096)
    s = torch.as_tensor(s_np, dtype=torch.complex64, device=dev)
    ph = torch.zeros(wl.n_pulses, dtype=torch.float32, device=dev)
    da = torch.zeros_like(ph)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    plan = T.Plan(prm, k, ku, dev)
    st = Step(T, plan, s, ph, da)
    ms_e, _ = time_step(torch, st, steps, 3, graph=False)
    ms_g, _ = time_step(torch, st, steps, 3, graph=True)
    ms = min(ms_e, ms_g)
    passes = step_passes(T, plan, st, wl, plan.ent_fused, steps, ms_e * 1e3)
    st()
    torch.cuda.synchronize()
    log("4096 x 8192: oracle on two columns")
    cols = np.sort(np.random.default_rng(44).choice(wl.m, 2, replace=False))
    got = st.img.cpu().numpy()[cols].astype(np.complex128)
    from oracle import geometry as OG
    from oracle import weights as OW

    kx, _ = OG.stolt(k, ku)
    lam = OG.lattice_coordinate(kx, wl.fov)
    w = np.concatenate([OW.tffr_weights(lam[r:r + 256])[0] for r in range(0, wl.n_pulses, 256)])  # bounded memory
    ref = oracle_columns(wl, k, ku, s_np.astype(np.complex64).astype(np.complex128), cols, 4, user_w=w)
    rec = {"workload": wl.name, "n_pulses": wl.n_pulses, "n_freq": wl.n_freq, "image": [wl.m, wl.m],
           "ms_per_step": ms, "Msamples_per_s": wl.n_samples / (ms * 1e-3) / 1e6,
           "timing": "hip_graph" if ms_g < ms_e else "eager", "kept_count": plan.tffr_kept_count(),
           "passes": passes, "accuracy": dict(accuracy(got, ref), sample="2 of 4096 image columns, full height"),
           "launch": {"range_mode": plan.range_mode, "az_cols": plan.az_cols, "entropy_fused": plan.ent_fused}}
    del plan, st, s
    torch.cuda.empty_cache()
    return rec


def stolt_and_front_end(T, torch, wl, plan, k, ku, s, s_np, acc_cols, ms_step, args):
    """The Stolt-interpolation baseline image and the tFFR image alone (image formation
    only, as the paper's timing table compares), and the range-migration front end on
    raw echoes of the same geometry (J = 2 N_u positions)."""
    from paper_1910_10908_amd import scenes

    res = {}
    steps = max(20, args.steps // 2)
    graph = not args.eager
    log("comparison: stolt_interpolation, tffr image only")
    img = torch.empty((wl.m, wl.m), dtype=torch.complex64, device=s.device)
    ms_stolt, _ = time_step(torch, lambda: plan.tffr_stolt_image(s, out=img), steps, 5, graph=graph)
    ms_fwd, _ = time_step(torch, lambda: plan.tffr_forward(s, out=img), steps, 5, graph=graph)
    rec = {"ms_per_image": ms_stolt, "Msamples_per_s": wl.n_samples / (ms_stolt * 1e-3) / 1e6,
           "tffr_image_ms": ms_fwd, "tffr_image_over_stolt": ms_fwd / ms_stolt, "over_tffr_step": ms_stolt / ms_step,
           "note": "linear interpolation per slice onto the integer lattice, inverse FFT of the fine row, "
                   "azimuth stage as tFFR; image formation only"}
    if not args.no_cpu_baseline:
        from oracle import pipeline as OP
        from oracle import rma as ORMA

        got = plan.tffr_stolt_image(s).cpu().numpy()[acc_cols].astype(np.complex128)
        prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
        ref = ORMA.stolt_image(prob, s_np, cols=acc_cols)
        rec["accuracy"] = dict(accuracy(got, ref), sample=f"{len(acc_cols)} of {wl.m} image columns",
                               reference="oracle Stolt image")
    res["stolt_interpolation"] = rec
    log("comparison: rma_front_end")
    J, du = scenes.rma_positions(wl.n_pulses)
    gen = torch.Generator(s.device).manual_seed(17)
    echoes = torch.randn((J, wl.n_freq), dtype=torch.complex64, device=s.device, generator=gen)
    smp = torch.empty_like(s)
    xc = 2000.0
    ms_fe, _ = time_step(torch, lambda: plan.tffr_rma_front_end(echoes, du, xc, out=smp), steps, 5, graph=graph)
    rec = {"ms": ms_fe, "raw_positions": J, "Msamples_per_s": wl.n_samples / (ms_fe * 1e-3) / 1e6,
           "alg_bytes": (J + wl.n_pulses) * wl.n_freq * 8,
           "achieved_GBps": (J + wl.n_pulses) * wl.n_freq * 8 / (ms_fe * 1e-3) / 1e9,
           "note": "azimuth FFT of the raw echoes (J positions), centred N_u bins, reference multiply "
                   "exp(+i kx X_c) in FP64 phase, X_c = 2 km; output samples per second"}
    rec["hbm_frac"] = rec["achieved_GBps"] / HBM_PEAK_GBS
    if not args.no_cpu_baseline:
        from oracle import rma as ORMA

        plan.tffr_rma_front_end(echoes, du, xc, out=smp)
        cols = acc_cols[acc_cols < wl.n_freq]
        ct = torch.as_tensor(cols, device=s.device)
        ein = echoes[:, ct].cpu().numpy().astype(np.complex128)
        ref, _ = ORMA.front_end(ein, k[cols], du, xc, wl.n_pulses)
        rec["accuracy"] = dict(accuracy(smp[:, ct].cpu().numpy().astype(np.complex128), ref),
                               sample=f"{len(cols)} of {wl.n_freq} fast-time columns, all pulses")
    res["rma_front_end"] = rec
    # the same front end with per-pulse along-track position errors: a smooth platform
    # drift of up to 0.4 du (three random-phase sinusoids over the aperture), so the true
    # positions stay about du apart; a type-1 NUFFT along azimuth instead of the FFT.  The
    # call copies the positions after synchronising its stream, so it is timed eagerly,
    # with the copy.
    log("comparison: rma_front_end with position errors")
    rng_d = np.random.default_rng(18)
    jj = np.arange(J) / J
    drift = sum(np.sin(2 * np.pi * (f * jj + rng_d.uniform())) / f for f in (1.0, 2.0, 3.0))
    dpos = 0.4 * du * drift / np.max(np.abs(drift))
    ms_fp, _ = time_step(torch, lambda: plan.tffr_rma_front_end(echoes, du, xc, out=smp, dpos=dpos), steps, 5,
                         graph=False)
    rec = {"ms": ms_fp, "raw_positions": J, "Msamples_per_s": wl.n_samples / (ms_fp * 1e-3) / 1e6,
           "over_uniform_front_end": ms_fp / ms_fe,
           "note": "echoes recorded at u_j + d_j, a smooth drift with |d_j| <= 0.4 du: ES spreading of the J "
                   "echoes at their true positions onto a periodic grid of >= 2 N_u cells (sub-passes), FFT, "
                   "deapodisation, reference multiply; eager launches including the per-call position copy"}
    if not args.no_cpu_baseline:
        from oracle import rma as ORMA

        plan.tffr_rma_front_end(echoes, du, xc, out=smp, dpos=dpos)
        ref, _ = ORMA.front_end(ein, k[cols], du, xc, wl.n_pulses, dpos=dpos)
        rec["accuracy"] = dict(accuracy(smp[:, ct].cpu().numpy().astype(np.complex128), ref),
                               sample=f"{len(cols)} of {wl.n_freq} fast-time columns, all pulses")
    res["rma_front_end_position_errors"] = rec
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU slab design is described but not "
              "built, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        return sweep(args)
    import torch

    from paper_1910_10908_amd import scenes
    from paper_1910_10908_amd import tffr as T

    wl = scenes.WORKLOADS[args.workload]
    width = args.width or wl.kernel_width
    dev = "cuda:0"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    if args.profile_steps:
        # profiler runs: the kernels' work does not depend on the sample values, and a
        # seeded random phase history keeps the traced process to a handful of launches
        k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
        s = torch.as_tensor(scenes.random_samples(wl.n_pulses, wl.n_freq, 1), dtype=torch.complex64, device=dev)
    else:
        inp = scenes.make_inputs(wl, device=dev, scene=True)
        k, ku = inp["k"], inp["ku"]
        s = inp["samples"].to(torch.complex64).contiguous()
    torch.cuda.synchronize()
    t_synth = time.perf_counter() - t0
    # autofocus-style estimates: start from zero phase / position error
    ph = torch.zeros(wl.n_pulses, dtype=torch.float32, device=dev)
    da = torch.zeros_like(ph)

    def params(weighting, w=width, gridding=T.GRID_ES, **kw):
        return T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                                fov_y=wl.fov, weighting=weighting, kernel_width=w, dtype=T.C64, gridding=gridding,
                                **kw)

    if args.profile_steps and args.profile_ffr:
        plan = T.Plan(params(T.W_FFR), k, ku, dev)
        step = Step(T, plan, s, ph, da, ffr=True)
    else:
        plan = T.Plan(params(T.W_TFFR), k, ku, dev)
        step = Step(T, plan, s, ph, da)
    if args.profile_steps:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        # calibration: a plain device copy of known size for the HBM byte counters
        from paper_1910_10908_amd import profiling

        src = torch.empty(profiling.COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": wl.name, "ffr": args.profile_ffr,
                          "copy_bytes": profiling.COPY_BYTES}))
        return

    # the step timed both ways, as a HIP graph replay and as eager launches on one stream;
    # `value` is the faster (config.timing names it), both are reported
    log(f"{wl.name}: timing {args.steps} steps (eager, then graph replay)")
    ms_eager, _ = time_step(torch, step, args.steps, args.warmup, graph=False)
    ms_graph, replay_ok = None, None
    if not args.eager:
        ms_graph, runner = time_step(torch, step, args.steps, args.warmup, graph=True)
        # graph replays must reproduce the eager result
        step()
        torch.cuda.synchronize()
        ref_img, ref_gph = step.img.clone(), step.gph.clone()
        runner()
        torch.cuda.synchronize()
        replay_ok = bool(torch.equal(step.img, ref_img) or float((step.img - ref_img).abs().max()) <=
                         1e-5 * float(ref_img.abs().max()))
        replay_ok = replay_ok and float((step.gph - ref_gph).abs().max()) <= 1e-4 * float(
            ref_gph.abs().max() + 1e-30)
    use_graph = ms_graph is not None and ms_graph < ms_eager
    ms = ms_graph if use_graph else ms_eager

    # every launch of the step, timed with HIP events between the step's own launches (same
    # order, data flow and caches as the timed steps), less an equal share of the events'
    # own cost; the slowest is the roofline kernel
    log("per-launch times inside the step")
    passes = step_passes(T, plan, step, wl, plan.ent_fused, max(50, args.steps), ms_eager * 1e3)
    timed = {n: r for n, r in passes.items() if "alg_bytes" in r}
    kname = max(timed, key=lambda n: timed[n]["us"])
    kr = timed[kname]
    copy_gbs = copy_bandwidth(torch)
    kept = plan.tffr_kept_count()

    out = {
        "metric": METRIC,
        "value": wl.n_samples / (ms * 1e-3) / 1e6,
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_pulses": wl.n_pulses, "n_freq": wl.n_freq, "image": [wl.m, wl.m],
                   "fine_grid": list(plan.nfine), "kernel_width": width, "weighting": "tffr", "tau": 0.97,
                   "threshold": "literal", "window_a": 0.01, "q": 3,
                   "timing": "hip_graph" if use_graph else "eager", "parallelism": "single_gpu"},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": kr["achieved_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kr["hbm_frac"], "traffic": kr["traffic"], "kernel_us": kr["us"],
                     "alg_bytes": kr["alg_bytes"], "copy_GBps": copy_gbs,
                     "frac_of_copy": kr["achieved_GBps"] / copy_gbs, "binding": kr["binding"],
                     "fractions": kr["fractions"], "kernel_us_trace": kr.get("us_trace"),
                     "kernel_us_over_trace": kr.get("us_over_trace")},
        "passes": passes,
        "launch": {"range_mode": plan.range_mode, "az_cols": plan.az_cols, "entropy_fused": plan.ent_fused},
        "kept_count": kept,
        "graph_replay_matches_eager": replay_ok,
        "eager_ms_per_step": ms_eager,
        "graph_ms_per_step": ms_graph,
        "input_synthesis_s": t_synth,
    }

    s_np = s.cpu().numpy().astype(np.complex128)
    col_idx = np.sort(np.random.default_rng(5).choice(wl.m, args.cpu_cols, replace=False))
    if not args.no_compare:
        comp = {}
        acc_cols = col_idx[: min(16, len(col_idx))]
        for name, prm, ffr_in_step in (
                ("plain_ffr_D_solved_in_step", params(T.W_FFR), True),
                ("plain_ffr_D_cached_by_plan", params(T.W_FFR), False),
                ("plain_nufft_quad", params(T.W_QUAD), False),
                ("tffr_correlation_threshold", params(T.W_TFFR, thresh_mode=T.THRESH_CORRELATION), False),
                ("tffr_width6", params(T.W_TFFR, 6), False),
                ("tffr_literal_algorithm1", params(T.W_TFFR, width, T.GRID_LITERAL), False)):
            log(f"comparison: {name}")
            try:
                p2 = T.Plan(prm, k, ku, dev)
            except RuntimeError as e:
                comp[name] = {"error": str(e)}
                continue
            st2 = Step(T, p2, s, ph, da, ffr=ffr_in_step)
            ms2, _ = time_step(torch, st2, max(20, args.steps // 2), 5, graph=not args.eager)
            rec = {"ms_per_step": ms2, "Msamples_per_s": wl.n_samples / (ms2 * 1e-3) / 1e6,
                   "kernel_width": prm.kernel_width, "over_tffr_step": ms2 / ms}
            if name.startswith("plain_ffr"):
                rec["note"] = ("banded D = B_2(pinv(Psi W)) re-solved on the GPU inside every step" if ffr_in_step
                               else "D solved once per geometry at plan creation, applied in every step")
            if name == "tffr_correlation_threshold":
                rec["kept_count"] = p2.tffr_kept_count()
                rec["note"] = "keep iff g >= tau (the correlation reading of R_tau); removed samples skip their taps"
            if name == "tffr_literal_algorithm1":
                rec["note"] = ("range gridding with the window's own transform truncated to |l - lam| < q on the "
                               "image lattice, / w(x) (Eq. (8) as printed); azimuth as tFFR")
            if not args.no_cpu_baseline and name in ("plain_ffr_D_cached_by_plan", "tffr_correlation_threshold",
                                                     "tffr_width6", "tffr_literal_algorithm1"):
                img2 = p2.tffr_forward(s, ph, da).cpu().numpy()[acc_cols].astype(np.complex128)
                if name == "plain_ffr_D_cached_by_plan":
                    from oracle import geometry as OG
                    from oracle import weights as OW

                    kx, _ = OG.stolt(k, ku)
                    wf = OW.ffr_weights(OG.lattice_coordinate(kx, wl.fov), 0.01, 3.0, 2, workers=ORACLE_WORKERS)
                    ref2 = oracle_columns(wl, k, ku, s_np, acc_cols, 4, user_w=wf)
                elif name == "tffr_correlation_threshold":
                    ref2 = oracle_columns(wl, k, ku, s_np, acc_cols, 3, thresh_mode=1)
                else:  # the exact weighted sum (tFFR weights): the width-6 kernel's and the literal method's error
                    ref2 = oracle_columns(wl, k, ku, s_np, acc_cols, 3)
                rec["accuracy"] = dict(accuracy(img2, ref2), sample=f"{len(acc_cols)} of {wl.m} image columns",
                                       reference=("oracle with its own FFR weights" if name.startswith("plain_ffr")
                                                  else "oracle with the same threshold" if "correlation" in name
                                                  else "oracle exact weighted sum, tFFR weights"))
            comp[name] = rec
            del p2, st2
        comp.update(stolt_and_front_end(T, torch, wl, plan, k, ku, s, s_np, acc_cols, ms, args))
        out["comparisons"] = comp

    # accuracy against the FP64 oracle on sampled image columns (and CPU timing of the oracle)
    if not args.no_cpu_baseline:
        log("oracle on the host cores (bounded sample)")
        base, ref_cols, col_idx = cpu_baseline(wl, k, ku, s_np, np.zeros(wl.n_pulses), np.zeros(wl.n_pulses),
                                               args.cpu_cols)
        out["cpu_baseline"] = base
        step()
        torch.cuda.synchronize()
        got = step.img.cpu().numpy()[col_idx].astype(np.complex128)
        out["accuracy"] = dict(accuracy(got, ref_cols), sample=f"{len(col_idx)} of {wl.m} image columns, full height")
    if not args.no_full_swath and wl.name != "full_swath_4k":
        log("4096 x 8192 leg")
        out["full_swath_4k"] = full_swath_leg(T, torch, max(10, args.steps // 4))
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
