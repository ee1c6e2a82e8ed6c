"""GPU parity at the full workload sizes, on outputs the FP64 oracle computes one by one
(sampled image columns, sampled samples of the adjoint), plus properties that hold at
any size.  Inputs are seeded CN(0,1) phase histories on the workloads' exact geometry."""

import numpy as np
import pytest
import torch

from oracle import nudft as ON
from oracle import pipeline as OP
from oracle import weights as OW
from paper_1910_10908_amd import scenes
from paper_1910_10908_amd import tffr as T
from tests.gpu_helpers import DEV, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(gpu):
    print(flush=True)
    yield


def _setup(name, dtype=T.C64, width=7, seed=0):
    wl = scenes.WORKLOADS[name]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                           fov_y=wl.fov, kernel_width=width, dtype=dtype)
    plan = T.Plan(prm, k, ku, DEV)
    prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    s = scenes.random_samples(wl.n_pulses, wl.n_freq, 777 + seed)
    return wl, plan, prob, s


def _oracle_weights_chunked(prob, rows=256):
    """tFFR weights of every sample, computed slice-chunk by slice-chunk (memory bound)."""
    kx, ky, lam, X, Y = prob.geometry()
    w = np.empty_like(lam)
    for r0 in range(0, lam.shape[0], rows):
        w[r0:r0 + rows] = OW.tffr_weights(lam[r0:r0 + rows], prob.a, prob.q, prob.tau, prob.thresh_mode)[0]
    return w


def _oracle_columns(prob, s, cols, phase=None):
    kx, ky, lam, X, Y = prob.geometry()
    psi = OP.row_phase(ky, phase, None)
    c = _oracle_weights_chunked(prob) * (s * np.exp(1j * psi)[:, None])
    return ON.forward_columns(c, kx, ky, X, Y, cols)


@pytest.mark.parametrize("name", ["ffr_vs_tffr_c64", "autofocus_1k"])
def test_forward_sampled_columns(name):
    wl, plan, prob, s = _setup(name)
    print(f"{name}: forward, sampled columns", flush=True)
    rng = np.random.default_rng(1)
    phase = rng.normal(0, 0.5, wl.n_pulses)
    pt = torch.as_tensor(phase, dtype=torch.float32, device=DEV)
    img = plan.tffr_forward(torch.as_tensor(s, dtype=torch.complex64, device=DEV), pt).cpu().numpy()
    cols = np.sort(rng.choice(wl.m, 6, replace=False))
    s32 = s.astype(np.complex64).astype(np.complex128)
    ref = _oracle_columns(prob, s32, cols, pt.cpu().double().numpy())
    err = rel_l2(img[cols], ref)
    print(f"  rel-L2 over {len(cols)} full columns: {err:.3e}", flush=True)
    assert err < 1e-5


def test_adjoint_sampled_samples_bench_config():
    wl, plan, prob, s = _setup("ffr_vs_tffr_c64")
    print("bench config: adjoint at sampled samples", flush=True)
    rng = np.random.default_rng(2)
    y = (rng.standard_normal((wl.m, wl.m)) + 1j * rng.standard_normal((wl.m, wl.m))).astype(np.complex64)
    gs, _, _ = plan.tffr_adjoint(torch.as_tensor(y, device=DEV))
    gs = gs.cpu().numpy()
    kx, ky, lam, X, Y = prob.geometry()
    w = _oracle_weights_chunked(prob)
    picks = [(int(rng.integers(wl.n_pulses)), int(rng.integers(wl.n_freq))) for _ in range(12)]
    ref = ON.adjoint_samples(y.astype(np.complex128), kx, ky, X, Y, picks)
    ref = ref * np.array([w[n, p] for n, p in picks])
    got = np.array([gs[n, p] for n, p in picks])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  rel-L2 over {len(picks)} samples: {err:.3e}", flush=True)
    assert err < 1e-5


def test_precision_study_fp32_and_fp16_2k():
    """2048 x 4096 samples -> 2048^2 image: FP32 samples and FP16-stored samples (FP32
    accumulation) against the FP64 oracle on the same (rounded) inputs, sampled columns."""
    wl = scenes.WORKLOADS["precision_2k"]
    _, plan32, prob, s = _setup("precision_2k")
    rng = np.random.default_rng(3)
    cols = np.sort(rng.choice(wl.m, 3, replace=False))
    img32 = plan32.tffr_forward(torch.as_tensor(s, dtype=torch.complex64, device=DEV)).cpu().numpy()
    ref32 = _oracle_columns(prob, s.astype(np.complex64).astype(np.complex128), cols)
    e32 = rel_l2(img32[cols], ref32)
    del plan32
    _, plan16, _, _ = _setup("precision_2k", dtype=T.C64_FP16IN)
    h = np.stack([s.real, s.imag], axis=-1).astype(np.float16)
    img16 = plan16.tffr_forward(torch.as_tensor(h, device=DEV)).cpu().numpy()
    s16 = h[..., 0].astype(np.float64) + 1j * h[..., 1].astype(np.float64)
    ref16 = _oracle_columns(prob, s16, cols)
    e16 = rel_l2(img16[cols], ref16)
    ref_full = _oracle_columns(prob, s, cols)
    e16_in = rel_l2(img16[cols], ref_full)
    print(f"  FP32 rel-L2 {e32:.3e}; FP16-stored vs rounded inputs {e16:.3e}; vs FP64 inputs {e16_in:.3e}",
          flush=True)
    assert e32 < 1e-5 and e16 < 1e-5
    assert e16_in < 1e-3  # the input rounding itself (~2^-11 relative per sample)


def test_launch_configuration_by_density():
    """Sparse slices (512 x 1024: ~3.1-3.6 fine cells apart) and dense ones (2048 x 4096:
    0.8-0.9 cells apart) take the run range kernel at width 7, the densest (4096 x 8192:
    under half a cell apart) its paired form; 512 slices of two parts each (two waves per
    SIMD with one workgroup per slice) grid both parts at once; the literal lattice taps
    take the sub-pass kernel; every full-size plan runs the fused entropy azimuth kernel."""
    for name, mode in (("ffr_vs_tffr_c64", 3), ("autofocus_1k", 1), ("precision_2k", 1), ("full_swath_4k", 2)):
        wl = scenes.WORKLOADS[name]
        k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
        prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                               fov_y=wl.fov)
        plan = T.Plan(prm, k, ku, DEV)
        print(f"  {name}: range mode {plan.range_mode}, azimuth columns {plan.az_cols}, fused {plan.ent_fused}",
              flush=True)
        assert plan.range_mode == mode and plan.ent_fused
    wl = scenes.WORKLOADS["ffr_vs_tffr_c64"]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov,
                           gridding=T.GRID_LITERAL)
    assert T.Plan(prm, k, ku, DEV).range_mode == 0


def test_full_swath_sampled_columns_and_memory():
    wl, plan, prob, s = _setup("full_swath_4k")
    print("full swath: forward, sampled columns, peak memory", flush=True)
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    img, loss, gs, gph, gda = plan.tffr_entropy_step(st, torch.zeros(wl.n_pulses, device=DEV),
                                                     torch.zeros(wl.n_pulses, device=DEV))
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    print(f"  peak device memory of one step (inputs, outputs, workspace): {peak / 2**20:.0f} MiB", flush=True)
    rng = np.random.default_rng(4)
    cols = np.sort(rng.choice(wl.m, 2, replace=False))
    ref = _oracle_columns(prob, s.astype(np.complex64).astype(np.complex128), cols)
    err = rel_l2(img.cpu().numpy()[cols], ref)
    print(f"  rel-L2 over {len(cols)} full columns: {err:.3e}", flush=True)
    assert err < 1e-5
    assert peak < 4 * 2**30


def test_autofocus_gradient_properties_1k():
    """At 1024 x 2048 samples: the phase gradient of the entropy sums to ~0 (a global phase
    leaves |I| unchanged), the position gradient is ky times it, and a central difference
    of the GPU loss along a random direction matches <grad, v>."""
    wl, plan, prob, s = _setup("autofocus_1k")
    rng = np.random.default_rng(5)
    phase = rng.normal(0, 0.5, wl.n_pulses)
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    ph = torch.as_tensor(phase, dtype=torch.float32, device=DEV)
    da = torch.zeros(wl.n_pulses, dtype=torch.float32, device=DEV)
    img, loss, gs, gph, gda = plan.tffr_entropy_step(st, ph, da)
    g = gph.double().cpu().numpy()
    assert abs(g.sum()) < 1e-3 * np.abs(g).sum()
    ky = plan.ku
    assert np.allclose(gda.double().cpu().numpy(), ky * g, rtol=1e-5, atol=1e-6 * np.abs(ky * g).max())
    v = rng.standard_normal(wl.n_pulses)
    v -= v.mean()
    h = 2e-2
    lp = plan.tffr_entropy_step(st, ph + h * torch.as_tensor(v, dtype=torch.float32, device=DEV), da)[1]
    lm = plan.tffr_entropy_step(st, ph - h * torch.as_tensor(v, dtype=torch.float32, device=DEV), da)[1]
    fd = (float(lp) - float(lm)) / (2 * h)
    an = float(np.dot(g, v))
    print(f"  directional derivative: central difference {fd:.6e}, gradient {an:.6e}", flush=True)
    assert abs(fd - an) < 2e-2 * abs(an) + 1e-6
