"""GPU parity of the range-migration front end and the Stolt-interpolation baseline
(tffr_rma_front_end, tffr_stolt_image) against the FP64 oracle (oracle.rma)."""

import numpy as np
import pytest
import torch

from oracle import geometry, pipeline as OP, rma as ORMA
from paper_1910_10908_amd import scenes
from paper_1910_10908_amd import tffr as T

from .gpu_helpers import DEV, Case, peak_db, rel_l2

pytestmark = pytest.mark.gpu

WORKERS = 16


def _echoes(J, P, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((J, P)) + 1j * rng.standard_normal((J, P))) / np.sqrt(2.0)


def _front_case(n_pulses, n_freq, dtype, J=None):
    J0, du = scenes.rma_positions(n_pulses)
    J = J0 if J is None else J
    case = Case(n_pulses, n_freq, 64, fov=40.0, dtype=dtype, width=7 if dtype != T.C128 else 14)
    return case, J, du


def _max_rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / np.max(np.abs(b)))


def _got(plan, out):
    if plan.params.dtype == T.C64_FP16IN:
        h = out.float().cpu().numpy()
        return h[..., 0] + 1j * h[..., 1]
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", [T.C64, T.C128, T.C64_FP16IN])
@pytest.mark.parametrize("n_pulses,n_freq", [(64, 96), (32, 200)])
def test_front_end_vs_oracle(dtype, n_pulses, n_freq):
    """J = 2 N_u raw positions, fast-time columns in several workgroup tiles plus a ragged
    last tile, reference range 523.7 m (phases of 1e5 rad)."""
    print(f"front end N_u {n_pulses} P {n_freq} dtype {dtype}", flush=True)
    case, J, du = _front_case(n_pulses, n_freq, dtype)
    e = _echoes(J, n_freq, 11 + n_pulses)
    ct = torch.complex128 if dtype == T.C128 else torch.complex64
    et = torch.as_tensor(e, dtype=ct, device=DEV)
    got = _got(case.plan, case.plan.tffr_rma_front_end(et, du, 523.7))
    ein = et.cpu().numpy().astype(np.complex128)
    ref, ku = ORMA.front_end(ein, case.k, du, 523.7, n_pulses)
    np.testing.assert_allclose(ku, case.ku, rtol=0, atol=1e-12)
    e_max = _max_rel(got, ref)
    print(f"  max-rel {e_max:.2e}", flush=True)
    tol = {T.C64: 2e-6, T.C128: 1e-12, T.C64_FP16IN: 1e-3}[dtype]
    assert e_max < tol


def test_front_end_wider_transform_keeps_the_centre():
    """J = 4 N_u: the N_u wavenumbers nearest zero of a longer transform (the plan's ku
    spacing then matches du = c / (8 fc))."""
    n_pulses, n_freq = 64, 80
    k, _ = scenes.radar_sampling(n_pulses, n_freq)
    J, du = 4 * n_pulses, scenes.C_LIGHT / (8.0 * 10e9)
    ku = ORMA.azimuth_wavenumbers(n_pulses, J, du)
    prm = T.default_params(n_pulses=n_pulses, n_freq=n_freq, mx=64, my=64, fov_x=40.0, fov_y=40.0)
    plan = T.Plan(prm, k, ku, DEV)
    e = _echoes(J, n_freq, 5)
    got = plan.tffr_rma_front_end(torch.as_tensor(e, dtype=torch.complex64, device=DEV), du, 80.0).cpu().numpy()
    ref, _ = ORMA.front_end(e.astype(np.complex64).astype(np.complex128), k, du, 80.0, n_pulses)
    assert _max_rel(got, ref) < 2e-6


def test_front_end_rejects_mismatched_geometry():
    case, J, du = _front_case(64, 96, T.C64)
    et = torch.zeros((J, 96), dtype=torch.complex64, device=DEV)
    out = torch.empty((64, 96), dtype=torch.complex64, device=DEV)
    lib, h = case.plan.lib, case.plan.handle
    ptr = lambda t: torch.Tensor.data_ptr(t)
    assert lib.tffr_rma_front_end(h, ptr(et), J, du * 1.001, 0.0, ptr(out), None) == 1  # ku of another du
    assert lib.tffr_rma_front_end(h, ptr(et), J - 1, du, 0.0, ptr(out), None) == 1      # not a power of two
    assert lib.tffr_rma_front_end(h, ptr(et), 32, du, 0.0, ptr(out), None) == 1         # fewer than 64 / N_u
    assert lib.tffr_rma_front_end(h, ptr(et), J, -du, 0.0, ptr(out), None) == 1
    assert lib.tffr_rma_front_end(h, ptr(et), J, du, float("nan"), ptr(out), None) == 1


@pytest.mark.parametrize("dtype", [T.C64, T.C128])
@pytest.mark.parametrize("with_ref", [False, True])
@pytest.mark.parametrize("n_freq", [64, 256, 2048])
def test_range_fft_vs_oracle(dtype, with_ref, n_freq):
    """Range FFT and matched filter of random pulses against the oracle, in place."""
    print(f"range FFT n_freq {n_freq} ref {with_ref} dtype {dtype}", flush=True)
    case = Case(8, n_freq, 64, fov=40.0, dtype=dtype, width=7 if dtype != T.C128 else 14)
    J = 24
    ct = torch.complex128 if dtype == T.C128 else torch.complex64
    r = _echoes(J, n_freq, 51 + n_freq)
    rng = np.random.default_rng(52)
    ref = np.exp(1j * rng.uniform(0, 2 * np.pi, n_freq)) * rng.uniform(0.5, 1.5, n_freq) if with_ref else None
    rt = torch.as_tensor(r, dtype=ct, device=DEV)
    rin = rt.cpu().numpy().astype(np.complex128)
    reft = torch.as_tensor(ref, dtype=ct, device=DEV) if with_ref else None
    got = case.plan.tffr_rma_range_fft(rt, reft, out=rt).cpu().numpy()  # in place
    want = ORMA.range_fft(rin, reft.cpu().numpy().astype(np.complex128) if with_ref else None)
    e = _max_rel(got, want)
    print(f"  max-rel {e:.2e}", flush=True)
    # FP64: rounding of log2(n_freq) Stockham stages with two-level twiddle products
    assert e < (1e-6 if dtype == T.C64 else 1e-12)


def test_range_fft_then_front_end_matches_frequency_echoes():
    """Time-domain pulses of point scatterers (the frequency-domain echoes taken back to
    time samples at the centred bins) through the range FFT and the front end give the
    samples of the frequency-domain echoes; a unit reference and a chirp code with its
    conjugate reference both recover them."""
    n_pulses, n_freq = 64, 256
    case, J, du = _front_case(n_pulses, n_freq, T.C64)
    rng = np.random.default_rng(53)
    x, y = rng.uniform(-10, 10, 5), rng.uniform(-0.2, 0.2, 5)
    a = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    E = scenes.raw_echoes(case.k, J, du, 500.0, x, y, a)
    m = np.arange(n_freq) - n_freq // 2
    code = np.exp(1j * np.pi * (m / n_freq) ** 2 * n_freq / 4)
    ref_s, _ = ORMA.front_end(E, case.k, du, 500.0, n_pulses)
    for C in (np.ones(n_freq), code):
        pulses = np.fft.ifft(np.roll(C * E, -n_freq // 2, axis=1), axis=1)
        pt = torch.as_tensor(pulses, dtype=torch.complex64, device=DEV)
        reft = torch.as_tensor(np.conj(C), dtype=torch.complex64, device=DEV)
        echoes = case.plan.tffr_rma_range_fft(pt, reft)
        got = case.plan.tffr_rma_front_end(echoes, du, 500.0).cpu().numpy()
        e = rel_l2(got, ref_s)
        print(f"  rel-L2 {e:.2e}", flush=True)
        assert e < 1e-5


def test_range_fft_rejects():
    case = Case(8, 100, 64, fov=40.0)
    r = torch.zeros((4, 100), dtype=torch.complex64, device=DEV)
    with pytest.raises(RuntimeError, match="UNSUPPORTED"):
        case.plan.tffr_rma_range_fft(r)
    lib, h = case.plan.lib, case.plan.handle
    assert lib.tffr_rma_range_fft(h, None, 4, None, None, None) == 1


@pytest.mark.parametrize("dtype", [T.C64, T.C128, T.C64_FP16IN])
@pytest.mark.parametrize("n_pulses,n_freq,amp", [(64, 96, 0.4), (32, 200, 0.45), (64, 96, 0.0)])
def test_front_end_position_errors_vs_oracle(dtype, n_pulses, n_freq, amp):
    """Echoes recorded at u_j + d_j (d uniform within +-amp du): the non-uniform azimuth
    transform against the oracle's sum at the true positions; amp 0 puts every source on
    the nominal grid (the uniform front end's result, through the gridding path)."""
    print(f"front end with position errors N_u {n_pulses} P {n_freq} amp {amp} dtype {dtype}", flush=True)
    case, J, du = _front_case(n_pulses, n_freq, dtype)
    d = np.random.default_rng(31 + n_pulses).uniform(-amp, amp, J) * du
    e = _echoes(J, n_freq, 41 + n_pulses)
    ct = torch.complex128 if dtype == T.C128 else torch.complex64
    et = torch.as_tensor(e, dtype=ct, device=DEV)
    got = _got(case.plan, case.plan.tffr_rma_front_end(et, du, 523.7, dpos=d))
    ref, _ = ORMA.front_end(et.cpu().numpy().astype(np.complex128), case.k, du, 523.7, n_pulses, dpos=d)
    e_max, e_l2 = _max_rel(got, ref), rel_l2(got, ref)
    print(f"  max-rel {e_max:.2e} rel-L2 {e_l2:.2e}", flush=True)
    tol = {T.C64: 1e-5, T.C128: 1e-10, T.C64_FP16IN: 1e-3}[dtype]
    assert e_max < tol


def test_front_end_position_errors_tone():
    """A tone exp(+i ku_m u) recorded at the true positions transforms to J at bin m."""
    n_pulses, n_freq = 64, 8
    case, J, du = _front_case(n_pulses, n_freq, T.C64)
    d = np.random.default_rng(5).uniform(-0.4, 0.4, J) * du
    m = 60
    u = (np.arange(J) - J / 2.0) * du + d
    e = np.repeat(np.exp(1j * case.ku[m] * u)[:, None], n_freq, axis=1)
    got = case.plan.tffr_rma_front_end(torch.as_tensor(e, dtype=torch.complex64, device=DEV), du, 0.0,
                                       dpos=d).cpu().numpy()
    assert np.max(np.abs(got[m] - J)) < 1e-5 * J


def test_front_end_position_errors_rejected():
    case, J, du = _front_case(64, 96, T.C64)
    et = torch.zeros((J, 96), dtype=torch.complex64, device=DEV)
    d = np.zeros(J)
    d[40] = -1.5 * du  # position 40 falls behind position 39
    with pytest.raises(RuntimeError, match="NONMONOTONE"):
        case.plan.tffr_rma_front_end(et, du, 0.0, dpos=d)
    d[40] = float("nan")
    with pytest.raises(RuntimeError, match="ERR_ARG"):
        case.plan.tffr_rma_front_end(et, du, 0.0, dpos=d)
    d = np.zeros(J)
    d[-1] = J * du  # the last position wraps past the first
    with pytest.raises(RuntimeError, match="NONMONOTONE"):
        case.plan.tffr_rma_front_end(et, du, 0.0, dpos=d)
    with pytest.raises(ValueError):
        case.plan.tffr_rma_front_end(et, du, 0.0, dpos=np.zeros(J - 1))


def test_front_end_position_errors_full_size_sampled_columns():
    """4096 x 8192 geometry (J = 8192 positions, an 8192-cell grid), positions within
    +-0.45 du of nominal, all N_u rows of 8 sampled fast-time columns against the oracle."""
    n_pulses, n_freq = 4096, 8192
    k, ku = scenes.radar_sampling(n_pulses, n_freq)
    J, du = scenes.rma_positions(n_pulses)
    prm = T.default_params(n_pulses=n_pulses, n_freq=n_freq, mx=4096, my=4096, fov_x=400.0, fov_y=400.0)
    plan = T.Plan(prm, k, ku, DEV)
    d = np.random.default_rng(77).uniform(-0.45, 0.45, J) * du
    et = torch.randn((J, n_freq), dtype=torch.complex64, device=DEV, generator=torch.Generator(DEV).manual_seed(7))
    got = plan.tffr_rma_front_end(et, du, 1500.0, dpos=d)
    cols = np.sort(np.random.default_rng(78).choice(n_freq, 8, replace=False))
    e = et[:, torch.as_tensor(cols, device=DEV)].cpu().numpy().astype(np.complex128)
    ref, _ = ORMA.front_end(e, k[cols], du, 1500.0, n_pulses, dpos=d)
    g = got[:, torch.as_tensor(cols, device=DEV)].cpu().numpy()
    e_max = _max_rel(g, ref)
    print(f"  8 columns max-rel {e_max:.2e}", flush=True)
    assert e_max < 1e-5


def test_front_end_full_size_sampled_columns():
    """4096 x 8192 geometry (J = 8192 positions, the largest single-column LDS tile), all
    N_u rows of 16 sampled fast-time columns against the oracle."""
    n_pulses, n_freq = 4096, 8192
    k, ku = scenes.radar_sampling(n_pulses, n_freq)
    J, du = scenes.rma_positions(n_pulses)
    prm = T.default_params(n_pulses=n_pulses, n_freq=n_freq, mx=4096, my=4096, fov_x=400.0, fov_y=400.0)
    plan = T.Plan(prm, k, ku, DEV)
    rng = np.random.default_rng(21)
    et = (torch.randn((J, n_freq), dtype=torch.complex64, device=DEV, generator=torch.Generator(DEV).manual_seed(3)))
    got = plan.tffr_rma_front_end(et, du, 1500.0)
    cols = np.sort(rng.choice(n_freq, 16, replace=False))
    ein = et[:, torch.as_tensor(cols, device=DEV)].cpu().numpy().astype(np.complex128)
    ref, _ = ORMA.front_end(ein, k[cols], du, 1500.0, n_pulses)
    e_max = _max_rel(got[:, torch.as_tensor(cols, device=DEV)].cpu().numpy(), ref)
    print(f"  4096 x 8192, 16 columns: max-rel {e_max:.2e}", flush=True)
    assert e_max < 5e-6


# ---------------------------------------------------------------- Stolt baseline
@pytest.mark.parametrize("dtype", [T.C64, T.C128, T.C64_FP16IN])
@pytest.mark.parametrize("n_pulses,n_freq,mx,fov", [(24, 200, 64, 40.0), (12, 512, 64, 50.0), (16, 96, 128, 25.0)])
def test_stolt_image_vs_oracle(dtype, n_pulses, n_freq, mx, fov):
    """Sample spacings above and below one lattice unit, lattice spans wider than mx (the
    parts), several FFT sizes; with per-pulse phase errors."""
    print(f"stolt {n_pulses}x{n_freq} mx {mx} fov {fov} dtype {dtype}", flush=True)
    case = Case(n_pulses, n_freq, mx, fov=fov, dtype=dtype, width=7 if dtype != T.C128 else 14, seed=31)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, n_pulses)
    got = case.plan.tffr_stolt_image(st, case.real(phase)).cpu().numpy()
    ref = ORMA.stolt_image(case.prob, s, case.rounded(phase))
    e, pk = rel_l2(got, ref), peak_db(got, ref)
    print(f"  rel-L2 {e:.2e} peak {pk:.1f} dB", flush=True)
    tol = 1e-10 if dtype == T.C128 else 1e-5
    assert e < tol and pk < (-160 if dtype == T.C128 else -100)


def test_stolt_image_bench_geometry_sampled_columns():
    """512 x 1024 samples -> 1024^2 (the benchmark's geometry, lattice span ~1600 > mx, two
    parts per slice): 16 sampled image columns against the oracle."""
    wl = scenes.WORKLOADS["ffr_vs_tffr_c64"]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    plan = T.Plan(prm, k, ku, DEV)
    s = scenes.random_samples(wl.n_pulses, wl.n_freq, 77)
    got = plan.tffr_stolt_image(torch.as_tensor(s, dtype=torch.complex64, device=DEV)).cpu().numpy()
    prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    cols = np.sort(np.random.default_rng(5).choice(wl.m, 16, replace=False))
    ref = ORMA.stolt_image(prob, s.astype(np.complex64).astype(np.complex128), cols=cols)
    e, pk = rel_l2(got[cols], ref), peak_db(got[cols], ref)
    print(f"  16 columns: rel-L2 {e:.2e} peak {pk:.1f} dB", flush=True)
    assert e < 1e-5 and pk < -100


def test_stolt_rejects_non_power_of_two_image():
    case = Case(8, 64, 96, fov=40.0)
    s, st = case.samples()
    img = torch.empty((96, 96), dtype=torch.complex64, device=DEV)
    assert case.plan.lib.tffr_stolt_image(case.plan.handle, st.data_ptr(), None, None, img.data_ptr(),
                                          case.plan.work.data_ptr(), None) == 5


def test_raw_echoes_to_images_focus_on_the_scatterers():
    """End to end on the GPU: raw echoes of three scatterers -> front end -> Stolt and
    tFFR images; each image's three brightest separated peaks sit within one pixel of
    the scatterers, and the GPU Stolt image matches the oracle chain."""
    n_pulses, n_freq = 64, 64
    k, _ = scenes.radar_sampling(n_pulses, n_freq)
    J, du = scenes.rma_positions(n_pulses)
    ku = ORMA.azimuth_wavenumbers(n_pulses, J, du)
    xc = 20.0
    xt, yt = np.array([0.75, -1.1, 0.3]), np.array([0.12, -0.2, 0.31])
    e = scenes.raw_echoes(k, J, du, xc, xt, yt, np.array([1.0, 0.8, 0.9], dtype=np.complex128))
    mx, my, fov_x, fov_y = 32, 16, 4.0, J * du
    prm = T.default_params(n_pulses=n_pulses, n_freq=n_freq, mx=mx, my=my, fov_x=fov_x, fov_y=fov_y)
    plan = T.Plan(prm, k, ku, DEV)
    s = plan.tffr_rma_front_end(torch.as_tensor(e, dtype=torch.complex64, device=DEV), du, xc)
    X, Y = geometry.pixel_coordinates(mx, fov_x), geometry.pixel_coordinates(my, fov_y)
    for name, img in (("stolt", plan.tffr_stolt_image(s)), ("tffr", plan.tffr_forward(s))):
        a = np.abs(img.cpu().numpy())
        for t in range(3):
            jx = np.argmin(np.abs(X - xt[t]))
            jy = np.argmin(np.abs(Y - yt[t]))
            win = a[max(0, jx - 1):jx + 2, max(0, jy - 1):jy + 2]
            assert win.max() > 0.5 * a.max(), (name, t)
    sref, _ = ORMA.front_end(e.astype(np.complex64).astype(np.complex128), k, du, xc, n_pulses)
    prob = OP.Problem(k=k, ku=ku, mx=mx, my=my, fov_x=fov_x, fov_y=fov_y)
    ref = ORMA.stolt_image(prob, sref)
    assert rel_l2(plan.tffr_stolt_image(s).cpu().numpy(), ref) < 1e-5


def test_front_end_largest_transform():
    """J = 16384 raw positions (the longest azimuth transform, one fast-time column per
    workgroup filling 128 KB of LDS): against the oracle on every column."""
    n_pulses, n_freq = 8192, 24
    k, ku = scenes.radar_sampling(n_pulses, n_freq)
    J, du = scenes.rma_positions(n_pulses)
    assert J == 16384
    prm = T.default_params(n_pulses=n_pulses, n_freq=n_freq, mx=64, my=64, fov_x=40.0, fov_y=40.0)
    plan = T.Plan(prm, k, ku, DEV)
    e = _echoes(J, n_freq, 29)
    got = plan.tffr_rma_front_end(torch.as_tensor(e, dtype=torch.complex64, device=DEV), du, 900.0).cpu().numpy()
    ref, _ = ORMA.front_end(e.astype(np.complex64).astype(np.complex128), k, du, 900.0, n_pulses)
    err = _max_rel(got, ref)
    print(f"  J = 16384: max-rel {err:.2e}", flush=True)
    assert err < 5e-6
