"""GPU parity of the HIP path against the FP64 oracle (and of single stages against
independent CPU references of that stage).  Every call goes through the C ABI."""

import numpy as np
import pytest
import torch

import oracle
from oracle import entropy as OE
from oracle import literal as OL
from oracle import pipeline as OP
from oracle import weights as OW
from paper_1910_10908_amd import tffr as T
from tests.gpu_helpers import DEV, Case, peak_db, rel_l2, tol_for

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(gpu):
    print(flush=True)
    yield


# ---------------------------------------------------------------- single stages
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("log2n", [6, 7, 8, 9, 10, 11, 12, 13])
@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("max_radix", [8, 16])
def test_lds_fft_vs_numpy(log2n, sign, dtype, max_radix):
    print(f"fft log2n={log2n} sign={sign} {dtype} max radix {max_radix}", flush=True)
    rng = np.random.default_rng(log2n)
    n = 1 << log2n
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    xt = torch.as_tensor(x, dtype=dtype, device=DEV)
    got = T.tffr_debug_fft(xt, sign, max_radix).cpu().numpy()
    xr = xt.cpu().numpy().astype(np.complex128)
    ref = np.fft.ifft(xr, axis=-1) * n if sign > 0 else np.fft.fft(xr, axis=-1)
    tol = 1e-6 if dtype == torch.complex64 else 1e-13
    assert rel_l2(got, ref) < tol


def es_spread_rows_cpu(case, c):
    """Independent FP64 reference of the range gridding: c[n,p] spread with the plan's
    ES kernel (beta, width from the plan) onto the periodic fine row."""
    kx, ky, lam, X, Y = case.prob.geometry()
    nf = case.plan.nfine[0]
    W, beta = case.prm.kernel_width, case.plan.beta
    t = kx * case.prm.fov_x / (2 * np.pi * case.prm.mx)
    u = (t - np.floor(t)) * nf
    out = np.zeros((kx.shape[0], nf), complex)
    for n in range(kx.shape[0]):
        for p in range(kx.shape[1]):
            for g in range(int(np.floor(u[n, p] - W / 2)) - 1, int(np.ceil(u[n, p] + W / 2)) + 2):
                z = (g - u[n, p]) / (W / 2)
                if abs(z) < 1:
                    out[n, g % nf] += c[n, p] * np.exp(beta * (np.sqrt(1 - z * z) - 1))
    return out


@pytest.mark.parametrize("weighting", [T.W_NONE, T.W_TFFR, T.W_QUAD])
def test_range_gridding_stage(weighting):
    print(f"gridding stage weighting={weighting}", flush=True)
    case = Case(6, 40, 32, weighting=weighting, seed=3)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 6)
    got = case.plan.tffr_debug_rows(st, stage=0, phase=case.real(phase)).cpu().numpy()
    c = OP.weighted_samples(case.prob, s, case.rounded(phase))
    ref = es_spread_rows_cpu(case, c)
    assert rel_l2(got, ref) < 2e-6


# Dense slices (consecutive samples ~0.3-1.3 fine cells apart at fov 40 m) through both
# range kernels: TFFR_RANGE_MODE forces the sub-pass (0) or the run kernel (1) at plan
# creation.  Rows wider than the fine row are cut into several parts.
DENSE = [(6, 256, 32), (4, 1000, 64), (3, 777, 128)]


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("size", DENSE)
def test_range_gridding_modes_dense(size, mode, monkeypatch):
    print(f"gridding stage, dense rows size={size} range mode={mode}", flush=True)
    monkeypatch.setenv("TFFR_RANGE_MODE", mode)
    case = Case(*size, weighting=T.W_TFFR, seed=5)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, size[0])
    got = case.plan.tffr_debug_rows(st, stage=0, phase=case.real(phase)).cpu().numpy()
    c = OP.weighted_samples(case.prob, s, case.rounded(phase))
    ref = es_spread_rows_cpu(case, c)
    assert rel_l2(got, ref) < 2e-6


# The run kernel at rows long enough for several waves of runs (NT = 256 on 2048- and
# 4096-cell rows: the first run of each wave goes through its halo) and for several parts
# (span beyond the row), dense and sparse, in both precisions, one part at a time and two
# at once (range mode 3, twice the threads, one LDS row per part; an odd last part leaves
# half the threads idle); on 4096-cell complex64 rows with samples under half a cell
# apart, its paired form (range mode 2).
@pytest.mark.parametrize("n_freq,fov,mx,dtype,mode", [
    (4000, 200.0, 1024, T.C64, 1), (6000, 300.0, 1024, T.C64, 1), (600, 200.0, 1024, T.C64, 1),
    (4000, 200.0, 1024, T.C128, 1), (6000, 300.0, 1024, T.C128, 1),
    (6600, 300.0, 2048, T.C64, 2), (13000, 600.0, 2048, T.C64, 2), (13000, 600.0, 2048, T.C128, 1)])
@pytest.mark.parametrize("parts", ["1", "2"])
def test_range_gridding_run_kernel_many_waves(n_freq, fov, mx, dtype, mode, parts, monkeypatch):
    print(f"gridding stage, run kernel n_freq={n_freq} fov={fov} mx={mx} dtype={dtype} parts={parts}",
          flush=True)
    monkeypatch.setenv("TFFR_RANGE_MODE", "1")
    monkeypatch.setenv("TFFR_RUN_PARTS", parts)
    case = Case(2, n_freq, mx, fov=fov, weighting=T.W_TFFR, dtype=dtype, seed=17)
    print(f"  range mode {case.plan.range_mode}", flush=True)
    # two parts at once (mode 3) on rows of at most 4096 cells, never with pairs
    assert case.plan.range_mode == (3 if parts == "2" and mode == 1 else mode)
    assert case.plan.nfine[0] == 2 * mx
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 2)
    got = case.plan.tffr_debug_rows(st, stage=0, phase=case.real(phase)).cpu().numpy()
    c = OP.weighted_samples(case.prob, s, case.rounded(phase))
    ref = es_spread_rows_cpu(case, c)
    err = rel_l2(got, ref)
    print(f"  rel-L2 {err:.3e}", flush=True)
    assert err < (2e-6 if dtype == T.C64 else 1e-11)


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("weighting,dtype,n_freq", [(T.W_TFFR, T.C64, 600), (T.W_QUAD, T.C64, 600),
                                                    (T.W_TFFR, T.C128, 600), (T.W_TFFR, T.C64_FP16IN, 600),
                                                    (T.W_FFR, T.C64, 145)])
def test_forward_dense_rows_both_range_modes(weighting, dtype, n_freq, mode, monkeypatch):
    print(f"forward, dense rows, weighting={weighting} dtype={dtype} n_freq={n_freq} range mode={mode}",
          flush=True)
    monkeypatch.setenv("TFFR_RANGE_MODE", mode)
    # plain FFR needs a full-rank frame product: ~1.1 lattice units (2.2 fine cells) apart
    case = Case(5, n_freq, 64, weighting=weighting, dtype=dtype, width=7, seed=13)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 5)
    dal = case.rng.normal(0, 0.004, 5)
    got = case.plan.tffr_forward(st, case.real(phase), case.real(dal)).cpu().numpy()
    ref = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    err = rel_l2(got, ref)
    print(f"  rel-L2 {err:.3e}", flush=True)
    # width 7 in complex128 is limited by the kernel (~1e-6), not by the arithmetic
    assert err < 1e-5


# ---------------------------------------------------------------- weights
@pytest.mark.parametrize("tau,mode", [(0.97, OW.THRESH_LITERAL), (1.03, OW.THRESH_LITERAL),
                                      (0.97, OW.THRESH_CORRELATION), (0.9, OW.THRESH_CORRELATION)])
@pytest.mark.parametrize("dtype", [T.C64, T.C128])
def test_tffr_weights_and_kept_count(tau, mode, dtype):
    print(f"tffr weights tau={tau} mode={mode} dtype={dtype}", flush=True)
    case = Case(64, 512, 128, fov=400.0, weighting=T.W_TFFR, tau=tau, thresh_mode=mode, dtype=dtype)
    got = case.plan.tffr_weights().cpu().numpy()
    kx, ky, lam, X, Y = case.prob.geometry()
    ref, kept = OW.tffr_weights(lam, 0.01, 3.0, tau, mode)
    # decisions are taken in FP64 near the threshold: identical kept sets
    assert np.array_equal(got != 0, kept)
    assert case.plan.tffr_kept_count() == int(kept.sum())
    # FP64: the closed forms cancel a(1 - e^{-a/2}) ~ a^2/2 out of terms of size a near
    # d = 0, a condition number ~ 2/a = 200, so two correct FP64 evaluations that round
    # sin/cos differently agree to ~ 200 * 16 eps ~ 1e-12; the kernels also form lam
    # in a different order (a few ulp of lam ~ 3e4), which moves 1/g by |d(1/g)/dlam| <= 1
    # times that.  FP32: polynomial + rounding.
    lam_ulp = np.spacing(np.max(lam))
    tol = 1e-12 + 8 * lam_ulp if dtype == T.C128 else 3e-7
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)) + 1e-300


def test_quad_weights():
    case = Case(16, 300, 64, fov=400.0, weighting=T.W_QUAD)
    got = case.plan.tffr_weights().cpu().numpy()
    kx, ky, lam, X, Y = case.prob.geometry()
    ref = OW.quad_weights(lam)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-6
    assert case.plan.tffr_kept_count() == 16 * 300


@pytest.mark.parametrize("dtype", [T.C64, T.C128])
def test_ffr_weights(dtype):
    print(f"ffr weights dtype={dtype}", flush=True)
    case = Case(8, 128, 128, fov=40.0, weighting=T.W_FFR, dtype=dtype)
    got = case.plan.tffr_weights().cpu().numpy()
    kx, ky, lam, X, Y = case.prob.geometry()
    ref = OW.ffr_weights(lam, 0.01, 3.0, 2)
    tol = 1e-12 if dtype == T.C128 else 1e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


# ---------------------------------------------------------------- forward / adjoint
SIZES = [(8, 16, 16), (64, 128, 128), (33, 100, 50), (5, 257, 34)]


@pytest.mark.parametrize("size", SIZES)
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
@pytest.mark.parametrize("weighting", [T.W_TFFR, T.W_QUAD, T.W_NONE])
def test_forward_parity(size, dtype, width, weighting):
    print(f"forward size={size} dtype={dtype} w={width} weighting={weighting}", flush=True)
    case = Case(*size, weighting=weighting, dtype=dtype, width=width, seed=11)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, size[0])
    dal = case.rng.normal(0, 0.004, size[0])
    got = case.plan.tffr_forward(st, case.real(phase), case.real(dal)).cpu().numpy()
    ref = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    err = rel_l2(got, ref)
    print(f"  rel-L2 {err:.3e} peak {peak_db(got, ref):.1f} dB", flush=True)
    assert err < tol_for(case)
    assert peak_db(got, ref) < 20 * np.log10(tol_for(case))


@pytest.mark.parametrize("size", SIZES)
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
@pytest.mark.parametrize("weighting", [T.W_TFFR, T.W_QUAD])
def test_adjoint_parity(size, dtype, width, weighting):
    print(f"adjoint size={size} dtype={dtype} w={width} weighting={weighting}", flush=True)
    case = Case(*size, weighting=weighting, dtype=dtype, width=width, seed=12)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, size[0])
    dal = case.rng.normal(0, 0.004, size[0])
    y = case.image_np()
    yt = torch.as_tensor(y, dtype=case.ctype, device=DEV)
    gs, gph, gda = case.plan.tffr_adjoint(yt, st, case.real(phase), case.real(dal), want_phase=True,
                                          want_dalong=True)
    yr = yt.cpu().numpy().astype(np.complex128)
    rgs, rgph, rgda = OP.backward(case.prob, yr, s, case.rounded(phase), case.rounded(dal))
    e1 = rel_l2(gs.cpu().numpy(), rgs)
    e2 = np.max(np.abs(gph.cpu().numpy() - rgph)) / np.max(np.abs(rgph))
    e3 = np.max(np.abs(gda.cpu().numpy() - rgda)) / np.max(np.abs(rgda))
    print(f"  grad_s rel-L2 {e1:.3e}  dphi {e2:.3e}  ddu {e3:.3e}", flush=True)
    tol = tol_for(case)
    assert e1 < tol and e2 < tol and e3 < tol


@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
def test_ffr_forward_adjoint(dtype, width):
    print(f"ffr fwd/adj dtype={dtype}", flush=True)
    case = Case(64, 128, 128, weighting=T.W_FFR, dtype=dtype, width=width, seed=13)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 64)
    got = case.plan.tffr_forward(st, case.real(phase)).cpu().numpy()
    ref = OP.image(case.prob, s, case.rounded(phase))
    assert rel_l2(got, ref) < tol_for(case)
    y = case.image_np()
    yt = torch.as_tensor(y, dtype=case.ctype, device=DEV)
    gs, gph, _ = case.plan.tffr_adjoint(yt, st, case.real(phase), want_phase=True)
    rgs, rgph, _ = OP.backward(case.prob, yt.cpu().numpy().astype(np.complex128), s, case.rounded(phase))
    assert rel_l2(gs.cpu().numpy(), rgs) < tol_for(case)
    assert np.max(np.abs(gph.cpu().numpy() - rgph)) < tol_for(case) * np.max(np.abs(rgph))
    # the explicit weights of tffr_weights give the same image as the plan's cached D
    D = case.plan.tffr_weights()
    got2 = case.plan.tffr_forward(st, case.real(phase), user_w=D).cpu().numpy()
    assert rel_l2(got2, got) < 1e-6


def test_adjoint_identity_gpu():
    case = Case(48, 200, 96, fov=100.0, seed=14)
    s, st = case.samples()
    y = torch.as_tensor(case.image_np(), dtype=case.ctype, device=DEV)
    Ax = case.plan.tffr_forward(st)
    Ahy, _, _ = case.plan.tffr_adjoint(y)
    lhs = torch.vdot(y.flatten().to(torch.complex128), Ax.flatten().to(torch.complex128))
    rhs = torch.vdot(Ahy.flatten().to(torch.complex128), st.flatten().to(torch.complex128))
    rel = float(abs(lhs - rhs) / (torch.linalg.norm(Ax.double()) * torch.linalg.norm(y.double())))
    assert rel < 1e-6


def test_entropy_and_gradients():
    print("entropy + autograd", flush=True)
    case = Case(64, 128, 128, seed=15)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 64)
    dal = case.rng.normal(0, 0.004, 64)
    pt = case.real(phase).requires_grad_(True)
    dt = case.real(dal).requires_grad_(True)
    st = st.requires_grad_(True)
    img = T.tffr_image(case.plan, st, pt, dt)
    loss = T.image_entropy(case.plan, img)
    loss.backward()
    ref_img = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    assert abs(float(loss) - OE.entropy(ref_img)) < 1e-5 * abs(OE.entropy(ref_img))
    gI = OE.entropy_grad(ref_img)
    rgs, rgph, rgda = OP.backward(case.prob, gI, s, case.rounded(phase), case.rounded(dal))
    assert rel_l2(st.grad.cpu().numpy(), rgs) < 1e-5
    assert np.max(np.abs(pt.grad.cpu().numpy() - rgph)) < 1e-5 * np.max(np.abs(rgph))
    assert np.max(np.abs(dt.grad.cpu().numpy() - rgda)) < 1e-5 * np.max(np.abs(rgda))
    # a global phase leaves |I| unchanged
    assert abs(float(pt.grad.double().sum())) < 1e-4 * float(pt.grad.double().abs().sum())


def test_entropy_kernel_values():
    case = Case(4, 8, 64, seed=16)
    I = case.image_np()
    It = torch.as_tensor(I, dtype=case.ctype, device=DEV)
    loss, grad = case.plan.tffr_entropy(It)
    Ir = It.cpu().numpy().astype(np.complex128)
    assert abs(float(loss) - OE.entropy(Ir)) < 1e-6
    assert rel_l2(grad.cpu().numpy(), OE.entropy_grad(Ir)) < 1e-5


def test_fp16_samples():
    case = Case(64, 128, 128, dtype=T.C64_FP16IN, seed=17)
    s16, st = case.samples()
    got = case.plan.tffr_forward(st).cpu().numpy()
    ref = OP.image(case.prob, s16)  # oracle on the FP16-rounded samples
    assert rel_l2(got, ref) < 1e-5


# ---------------------------------------------------------------- edge cases
def test_single_frequency_and_single_pulse():
    for size in [(1, 40, 32), (7, 1, 32)]:
        case = Case(*size, weighting=T.W_QUAD, seed=18)
        s, st = case.samples()
        got = case.plan.tffr_forward(st).cpu().numpy()
        ref = OP.image(case.prob, s)
        assert rel_l2(got, ref) < 1e-5


def test_everything_thresholded_gives_zero_image():
    case = Case(8, 64, 32, tau=5.0, seed=19)
    s, st = case.samples()
    assert case.plan.tffr_kept_count() == 0
    img = case.plan.tffr_forward(st)
    assert float(img.abs().max()) == 0.0


def test_nonsquare_image():
    case = Case(40, 90, 48, my=80, fov=40.0, fov_y=25.0, seed=20)
    s, st = case.samples()
    got = case.plan.tffr_forward(st).cpu().numpy()
    assert got.shape == (48, 80)
    assert rel_l2(got, OP.image(case.prob, s)) < 1e-5


# ---------------------------------------------------------------- fused step and graphs
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14), (T.C64_FP16IN, 7)])
def test_entropy_step_matches_separate_calls_and_oracle(dtype, width):
    print(f"entropy step dtype={dtype}", flush=True)
    case = Case(48, 160, 96, fov=60.0, dtype=dtype, width=width, seed=21)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 48)
    dal = case.rng.normal(0, 0.004, 48)
    ph, da = case.real(phase), case.real(dal)
    img, loss, gs, gph, gda = case.plan.tffr_entropy_step(st, ph, da)
    img2 = case.plan.tffr_forward(st, ph, da)
    loss2, gI = case.plan.tffr_entropy(img2)
    gs2, gph2, gda2 = case.plan.tffr_adjoint(gI, st, ph, da, want_phase=True, want_dalong=True)
    assert torch.equal(img, img2)
    assert abs(float(loss) - float(loss2)) < 1e-12 * abs(float(loss2))
    tol = tol_for(case)
    assert rel_l2(gs.cpu().numpy(), gs2.cpu().numpy()) < tol
    assert rel_l2(gph.cpu().numpy(), gph2.cpu().numpy()) < 10 * tol
    ref_img = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    assert rel_l2(img.cpu().numpy(), ref_img) < tol
    assert abs(float(loss) - OE.entropy(ref_img)) < 10 * tol * abs(OE.entropy(ref_img))
    rgs, rgph, rgda = OP.backward(case.prob, OE.entropy_grad(ref_img), s, case.rounded(phase), case.rounded(dal))
    assert rel_l2(gs.cpu().numpy(), rgs) < tol
    assert np.max(np.abs(gph.cpu().numpy() - rgph)) < tol * np.max(np.abs(rgph))
    assert np.max(np.abs(gda.cpu().numpy() - rgda)) < tol * np.max(np.abs(rgda))


def test_marginal_launch_timing_leaves_one_step_outputs():
    """The marginal per-launch timing issues each launch of the step twice in turn; every
    launch overwrites its outputs, so afterwards they equal one plain step's bit for bit,
    and it reports the same launches, in order, as the event timing."""
    print("marginal per-launch timing", flush=True)
    case = Case(64, 128, 128, weighting=T.W_TFFR, seed=24)
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, 64))
    da = case.real(case.rng.normal(0, 0.004, 64))
    ref = [t.clone() for t in case.plan.tffr_entropy_step(st, ph, da)]
    out = tuple(torch.full_like(t, 7.0) for t in ref)
    marg = case.plan.tffr_debug_step_kernel_marginal_times(st, ph, da, out=out, nsteps=5)
    ev = case.plan.tffr_debug_step_kernel_times(st, ph, da, out=tuple(torch.empty_like(t) for t in ref), nsteps=5)
    print(f"  marginal {marg}  events {ev}", flush=True)
    assert list(marg) == list(ev) and len(marg) >= 3
    for a, b in zip(out, ref):
        assert torch.equal(a, b)


@pytest.mark.parametrize("weighting", [T.W_TFFR, T.W_FFR])
def test_graph_replays_match_eager(weighting):
    """The fused step captured in a HIP graph gives the eager result on every replay,
    with other eager work and synchronisations between the replays."""
    print(f"graph replay weighting={weighting}", flush=True)
    case = Case(64, 128, 128, weighting=weighting, seed=22)
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, 64))
    out = (torch.empty(case.plan.shape_image, dtype=case.ctype, device=DEV),
           torch.empty((), dtype=torch.float64, device=DEV),
           torch.empty(case.plan.shape_samples, dtype=case.ctype, device=DEV),
           torch.empty(64, dtype=case.rtype, device=DEV), torch.empty(64, dtype=case.rtype, device=DEV))
    eager = [t.clone() for t in case.plan.tffr_entropy_step(st, ph, out=out)]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        case.plan.tffr_entropy_step(st, ph, out=out)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            case.plan.tffr_entropy_step(st, ph, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in out:
            t.zero_()
        case.plan.tffr_forward(st)  # unrelated eager work that reuses the workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert torch.equal(a, b), f"replay {rep}"


# ---------------------------------------------------------------- explicit coordinates
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
def test_plan_from_coordinates_equals_stolt_plan(dtype, width):
    """tffr_plan_create_xy with the Stolt map's own coordinates: the same image and
    gradients as the plan made from (k, ku) (the host forms kx with the kernels'
    operation order, so the values and every kernel decision coincide)."""
    print(f"xy plan == Stolt plan, dtype={dtype}", flush=True)
    case = Case(16, 200, 64, fov=40.0, dtype=dtype, width=width, seed=21)
    kx, ky, lam, X, Y = case.prob.geometry()
    pxy = T.Plan(case.prm, None, None, DEV, kx=kx, ky=np.repeat(ky[:, None], kx.shape[1], axis=1))
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, 16))
    da = case.real(case.rng.normal(0, 0.004, 16))
    a = case.plan.tffr_forward(st, ph, da)
    b = pxy.tffr_forward(st, ph, da)
    assert torch.equal(a, b)
    ga = case.plan.tffr_entropy_step(st, ph, da)
    gb = pxy.tffr_entropy_step(st, ph, da)
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)


@pytest.mark.parametrize("weighting", [T.W_TFFR, T.W_QUAD, T.W_NONE, T.W_FFR])
def test_plan_from_jittered_coordinates_vs_oracle(weighting):
    """A non-Stolt geometry with the slice structure (kx jittered along every slice,
    ky shifted): forward and adjoint against the oracle on the same coordinates."""
    print(f"xy plan, jittered geometry, weighting={weighting}", flush=True)
    case = Case(12, 100, 64, fov=40.0, weighting=weighting, seed=22)
    kx, ky, lam, X, Y = case.prob.geometry()
    rng = np.random.default_rng(23)
    jit = kx + rng.uniform(-0.3, 0.3, kx.shape) * np.min(np.diff(kx, axis=1))
    kyj = ky + 0.37
    plan = T.Plan(case.prm, None, None, DEV, kx=jit, ky=np.repeat(kyj[:, None], kx.shape[1], axis=1))
    prob = OP.Problem(k=case.k, ku=case.ku, mx=64, my=64, fov_x=40.0, fov_y=40.0, weighting=weighting,
                      kx_explicit=jit, ky_explicit=kyj)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 12)
    dal = case.rng.normal(0, 0.004, 12)
    got = plan.tffr_forward(st, case.real(phase), case.real(dal)).cpu().numpy()
    ref = OP.image(prob, s, case.rounded(phase), case.rounded(dal))
    e = rel_l2(got, ref)
    y = case.image_np()
    yt = torch.as_tensor(y, dtype=case.ctype, device=DEV)
    gs, gph, gda = plan.tffr_adjoint(yt, st, case.real(phase), case.real(dal), want_phase=True, want_dalong=True)
    rgs, rgph, rgda = OP.backward(prob, yt.cpu().numpy().astype(np.complex128), s, case.rounded(phase),
                                  case.rounded(dal))
    e1 = rel_l2(gs.cpu().numpy(), rgs)
    e2 = np.max(np.abs(gph.cpu().numpy() - rgph)) / np.max(np.abs(rgph))
    e3 = np.max(np.abs(gda.cpu().numpy() - rgda)) / np.max(np.abs(rgda))
    print(f"  forward {e:.3e}  grad_s {e1:.3e}  dphi {e2:.3e}  ddu {e3:.3e}", flush=True)
    assert e < 1e-5 and e1 < 1e-5 and e2 < 1e-5 and e3 < 1e-5


@pytest.mark.parametrize("dtype", [T.C64, T.C128, T.C64_FP16IN])
def test_row_phase_grad(dtype):
    """tffr_row_phase_grad on the adjoint's sample cotangent reproduces the phase and
    position gradients the adjoint reduces itself, and the oracle's."""
    print(f"row phase grad dtype={dtype}", flush=True)
    case = Case(10, 150, 32, dtype=dtype, width=7 if dtype != T.C128 else 14, seed=24)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 10)
    dal = case.rng.normal(0, 0.004, 10)
    yt = torch.as_tensor(case.image_np(), dtype=case.ctype, device=DEV)
    gs, gph, gda = case.plan.tffr_adjoint(yt, st, case.real(phase), case.real(dal), want_phase=True,
                                          want_dalong=True)
    gph2, gda2 = case.plan.tffr_row_phase_grad(st, gs)
    scale = float(gph.abs().max())
    assert float((gph2 - gph).abs().max()) <= 1e-6 * scale
    assert float((gda2 - gda).abs().max()) <= 1e-6 * float(gda.abs().max())
    # the formula itself, in FP64 on the same inputs
    gsn = gs.cpu().numpy().astype(np.complex128)
    ref = np.sum(gsn.imag * s.real - gsn.real * s.imag, axis=1)
    assert np.max(np.abs(gph2.cpu().numpy() - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("size", [(64, 128, 128), (33, 100, 50)])
def test_fused_azimuth_stage_fields(size):
    """The entropy step's fused azimuth kernel alone: its image equals the forward
    azimuth kernel's bit for bit, and its two adjoint fields are the adjoint azimuth
    transforms (FP64 reference of the type-2 sum over the image pixels) of I and of
    I (ln|I|^2 - c_b), with c_b = ln of the block's mean |I|^2."""
    print(f"fused azimuth stage size={size}", flush=True)
    case = Case(*size, seed=31)
    s, st = case.samples()
    hx = case.plan.tffr_debug_rows(st, stage=1)
    img_ref = T.tffr_debug_cols(case.plan, hx)
    img, h1, h2 = T.tffr_debug_ent_cols(case.plan, hx)
    assert torch.equal(img, img_ref)
    kx, ky, lam, X, Y = case.prob.geometry()
    I = img.cpu().numpy().astype(np.complex128)
    # adjoint azimuth transform: h[n][jx] = sum_jy f[jx][jy] exp(-i ky_n Y_jy)
    E = np.exp(-1j * np.outer(ky, Y))  # [n_pulses][my]
    r2 = (E @ I.T)
    assert rel_l2(h2.cpu().numpy(), r2) < 1e-5
    a = np.abs(I) ** 2
    mx, my = case.prm.mx, case.prm.my
    lg = np.where(a > 0, np.log(np.where(a > 0, a, 1.0)), 0.0)
    # the kernel centres per column block of the plan's width (each block's constant is
    # fixed by the image alone)
    w = case.plan.az_cols
    cbk = np.array([np.log(a[j0:j0 + w].sum() / (min(w, mx - j0) * my)) for j0 in range(0, mx, w)])
    cc = np.repeat(cbk, w)[:mx]
    r1 = E @ (I * (lg - cc[:, None])).T
    assert rel_l2(h1.cpu().numpy(), r1) < 1e-5


# ---------------------------------------------------------------- literal Algorithm-1 range gridding
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
@pytest.mark.parametrize("weighting,size", [(T.W_TFFR, (16, 200, 64)), (T.W_NONE, (9, 333, 128)),
                                            (T.W_QUAD, (5, 64, 64))])
def test_literal_gridding_vs_oracle(dtype, width, weighting, size):
    """TFFR_GRID_LITERAL: the window's own truncated transform on the image lattice,
    inverse FFT, division by w (Eq. (8) as printed), against the oracle of that
    definition; and the method's truncation error (literal vs the exact sum) is far
    above the kernel's error."""
    print(f"literal gridding size={size} dtype={dtype} weighting={weighting}", flush=True)
    case = Case(*size, fov=40.0, weighting=weighting, dtype=dtype, width=width, seed=51, gridding=T.GRID_LITERAL)
    assert case.plan.nfine[0] == size[2]
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, size[0])
    dal = case.rng.normal(0, 0.004, size[0])
    got = case.plan.tffr_forward(st, case.real(phase), case.real(dal)).cpu().numpy()
    ref = OL.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    err = rel_l2(got, ref)
    exact = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    trunc = rel_l2(ref, exact)
    print(f"  rel-L2 vs literal oracle {err:.3e}; literal method vs exact sum {trunc:.3e}", flush=True)
    assert err < tol_for(case)
    assert trunc > 100 * tol_for(case)


@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
def test_literal_gridding_adjoint_identity(dtype, width):
    """<A x, y> = <x, A^H y> for the literal plan (its adjoint gathers with the same
    lattice taps and the same division by w)."""
    case = Case(12, 150, 64, fov=40.0, dtype=dtype, width=width, seed=52, gridding=T.GRID_LITERAL)
    s, st = case.samples()
    y = case.image_np()
    yt = torch.as_tensor(y, dtype=case.ctype, device=DEV)
    Ax = case.plan.tffr_forward(st).cpu().numpy().astype(np.complex128)
    Ahy = case.plan.tffr_adjoint(yt)[0].cpu().numpy().astype(np.complex128)
    yr = yt.cpu().numpy().astype(np.complex128)
    sr = st.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(yr, Ax)
    rhs = np.vdot(Ahy, sr)
    tol = 1e-5 if dtype == T.C64 else 1e-11
    assert abs(lhs - rhs) <= tol * abs(lhs)


# ---------------------------------------------------------------- coordinate gradients
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
@pytest.mark.parametrize("weighting", [T.W_TFFR, T.W_QUAD, T.W_FFR])
def test_coordinate_gradients_vs_oracle(dtype, width, weighting):
    """tffr_coord_grad: dL/dkx per sample and dL/dky per slice for an image cotangent,
    weights held fixed, against the oracle's adjoint sums of the X- and Y-weighted
    cotangent."""
    print(f"coordinate gradients dtype={dtype} weighting={weighting}", flush=True)
    case = Case(12, 100, 64, my=48, fov=40.0, fov_y=30.0, weighting=weighting, dtype=dtype, width=width, seed=61)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 12)
    dal = case.rng.normal(0, 0.004, 12)
    G = case.rng.standard_normal((64, 48)) + 1j * case.rng.standard_normal((64, 48))
    Gt = torch.as_tensor(G, dtype=case.ctype, device=DEV)
    gkx, gky = case.plan.tffr_coord_grad(Gt, st, case.real(phase), case.real(dal))
    rkx, rky = OP.coordinate_gradients(case.prob, Gt.cpu().numpy().astype(np.complex128), s, case.rounded(phase),
                                       case.rounded(dal))
    e1 = rel_l2(gkx.cpu().numpy(), rkx)
    e2 = np.max(np.abs(gky.cpu().numpy() - rky)) / np.max(np.abs(rky))
    print(f"  dL/dkx rel-L2 {e1:.3e}  dL/dky {e2:.3e}", flush=True)
    tol = tol_for(case)
    assert e1 < 2 * tol and e2 < 20 * tol


def test_operator_classes_match_functions():
    """TFFR(plan).apply / TFFRAdjoint(plan).apply: the same values and gradients as the
    functional wrappers (autograd through the C ABI)."""
    case = Case(10, 80, 32, seed=71)
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, 10)).requires_grad_(True)
    img = T.TFFR(case.plan).apply(st, ph, None)
    ref = T.tffr_image(case.plan, st, ph.detach(), None)
    assert torch.equal(img.detach(), ref)
    loss = (img.abs() ** 2).sum()
    loss.backward()
    y = torch.as_tensor(case.image_np(), dtype=case.ctype, device=DEV)
    g = T.TFFRAdjoint(case.plan).apply(y)
    assert torch.equal(g, T.tffr_adjoint_op(case.plan, y))
    # d/dphi of sum |I|^2 is zero only for a single pulse; here it is a real, finite gradient
    assert torch.isfinite(ph.grad).all() and float(ph.grad.abs().sum()) > 0


def test_entropy_step_range_adjoint_alone_repeats_the_step():
    """tffr_debug_ent_adj_rows on the workspace an entropy step left behind reproduces that
    step's loss and gradients bit for bit (it only reads the workspace)."""
    case = Case(20, 90, 64, seed=81)
    s, st = case.samples()
    ph = case.real(case.rng.normal(0, 0.5, 20))
    da = case.real(case.rng.normal(0, 0.004, 20))
    img, loss, gs, gph, gda = case.plan.tffr_entropy_step(st, ph, da)
    loss2 = torch.empty_like(loss)
    gs2, gph2, gda2 = torch.empty_like(gs), torch.empty_like(gph), torch.empty_like(gda)
    p = case.plan
    for _ in range(2):
        T._lib.check(p.lib.tffr_debug_ent_adj_rows(p.handle, T._ptr(st), T._ptr(ph), T._ptr(da), None, T._ptr(loss2),
                                                   T._ptr(gs2), T._ptr(gph2), T._ptr(gda2), T._ptr(p.work),
                                                   T._stream()))
        torch.cuda.synchronize()
        assert torch.equal(loss2, loss) and torch.equal(gs2, gs) and torch.equal(gph2, gph) and torch.equal(gda2, gda)
