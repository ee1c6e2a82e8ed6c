"""GPU parity at the launch configurations the benchmark times, against the FP64 oracle:

* every azimuth block width (range columns per workgroup, forced with TFFR_AZ_COLS at plan
  creation and checked on the plan), including image widths that leave a partial block;
* the fused entropy step at 512 x 1024 -> 1024^2 (the benchmark's workload and launch) and
  the entropy gradient at 1024 x 2048 -> 1024^2 (the differentiation workload), against
  the oracle's loss and gradients;
* plain FFR at the 512 x 1024 geometry (weights and image);
* the correlation reading of the threshold, which keeps about half the samples.

Inputs are seeded CN(0,1) phase histories on the workloads' exact geometry.  The oracle
evaluates its row sums on threads (`workers`), which changes nothing but the wall time.

Tolerances.  The image target is rel-L2 <= 1e-5 (kernel error ~1.1e-6 at width 7 plus
FP32 rounding).  The entropy gradient -(2/S)(ln p + E) I inherits the image error scaled
by (|ln p + E| + 2)/|ln p + E| pixel by pixel (the logarithm's sensitivity is 2|dI|/|I|
times |I|), about twice the image error on speckle; the adjoint adds its own ~1e-6.
Measured: sample gradients 1.0-2.6e-6 and per-pulse phase gradients 0.9-3.5e-6 of their
largest value (images 0.5-1.4e-6).  Both are held to the 1e-5 target.
"""

import os

import numpy as np
import pytest
import torch

from oracle import entropy as OE
from oracle import geometry as OG
from oracle import pipeline as OP
from oracle import weights as OW
from paper_1910_10908_amd import scenes
from paper_1910_10908_amd import tffr as T
from tests.gpu_helpers import DEV, Case, peak_db, rel_l2

pytestmark = pytest.mark.gpu

WORKERS = 16  # oracle threads (the GPU machine's CPU share)
GRAD_S_TOL = 1e-5
DPHI_TOL = 1e-5


@pytest.fixture(autouse=True)
def _need_gpu(gpu):
    print(flush=True)
    yield


def _max_rel(got, ref):
    return float(np.max(np.abs(np.asarray(got) - ref)) / np.max(np.abs(ref)))


def _oracle_step(prob, s, phase, dal, workers=WORKERS):
    """Image, entropy and its gradients (samples, phase, position) from the oracle."""
    img = OP.image(prob, s, phase, dal, workers=workers)
    gI = OE.entropy_grad(img)
    gs, gph, gda = OP.backward(prob, gI, s, phase, dal, workers=workers)
    return img, OE.entropy(img), gs, gph, gda


def _check_step(tag, got, ref, tol_img=1e-5):
    img, loss, gs, gph, gda = (x.cpu().numpy() if torch.is_tensor(x) else x for x in got)
    rimg, rloss, rgs, rgph, rgda = ref
    e_img, e_pk = rel_l2(img, rimg), peak_db(img, rimg)
    e_loss = abs(float(loss) - rloss) / abs(rloss)
    e_gs, e_ph, e_da = rel_l2(gs, rgs), _max_rel(gph, rgph), _max_rel(gda, rgda)
    print(f"  {tag}: image rel-L2 {e_img:.3e} peak {e_pk:.1f} dB, loss {e_loss:.2e}, grad_s {e_gs:.3e}, "
          f"dphi {e_ph:.3e}, ddu {e_da:.3e}", flush=True)
    assert e_img < tol_img and e_pk < 20 * np.log10(tol_img)
    assert e_loss < tol_img
    assert e_gs < GRAD_S_TOL and e_ph < DPHI_TOL and e_da < DPHI_TOL


# ---------------------------------------------------------------- every azimuth block width
@pytest.mark.parametrize("mx", [96, 94])
@pytest.mark.parametrize("cb", [1, 2, 4])
def test_entropy_step_each_block_width(cb, mx, monkeypatch):
    """The fused entropy step with CB range columns per azimuth workgroup (94 columns leave
    a partial last block for CB = 4): image, loss and gradients against the oracle, and the
    fused azimuth kernel's two fields with the plan's own CB."""
    print(f"entropy step, block width {cb}, mx {mx}", flush=True)
    monkeypatch.setenv("TFFR_AZ_COLS", str(cb))
    case = Case(48, 160, mx, my=96, fov=60.0, seed=101)
    assert case.plan.az_cols == cb and case.plan.ent_fused
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 48)
    dal = case.rng.normal(0, 0.004, 48)
    got = case.plan.tffr_entropy_step(st, case.real(phase), case.real(dal))
    ref = _oracle_step(case.prob, s, case.rounded(phase), case.rounded(dal), workers=1)
    _check_step(f"CB={cb}", got, ref)
    # the fused kernel's fields for this CB: h2 = A_y^H I, h1 = A_y^H (I (ln|I|^2 - c_b)),
    # c_b = ln of block b's mean |I|^2 (FP64 type-2 sums over the GPU image)
    hx = case.plan.tffr_debug_rows(st, stage=1)
    img, h1, h2 = T.tffr_debug_ent_cols(case.plan, hx)
    kx, ky, lam, X, Y = case.prob.geometry()
    I = img.cpu().numpy().astype(np.complex128)
    E = np.exp(-1j * np.outer(ky, Y))
    a = np.abs(I) ** 2
    lg = np.where(a > 0, np.log(np.where(a > 0, a, 1.0)), 0.0)
    cbk = np.array([np.log(a[j0:j0 + cb].sum() / (min(cb, mx - j0) * 96)) for j0 in range(0, mx, cb)])
    cc = np.repeat(cbk, cb)[:mx]
    assert rel_l2(h2.cpu().numpy(), E @ I.T) < 1e-5
    assert rel_l2(h1.cpu().numpy(), E @ (I * (lg - cc[:, None])).T) < 1e-5


@pytest.mark.parametrize("cb", [1, 2, 4])
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
def test_forward_adjoint_each_block_width(cb, dtype, width, monkeypatch):
    print(f"forward / adjoint, block width {cb}, dtype {dtype}", flush=True)
    monkeypatch.setenv("TFFR_AZ_COLS", str(cb))
    case = Case(33, 100, 50, dtype=dtype, width=width, seed=102)
    assert case.plan.az_cols == cb
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 33)
    dal = case.rng.normal(0, 0.004, 33)
    ph, da = case.real(phase), case.real(dal)
    got = case.plan.tffr_forward(st, ph, da).cpu().numpy()
    ref = OP.image(case.prob, s, case.rounded(phase), case.rounded(dal))
    tol = 1e-10 if dtype == T.C128 else 1e-5
    assert rel_l2(got, ref) < tol and peak_db(got, ref) < 20 * np.log10(tol)
    yt = torch.as_tensor(case.image_np(), dtype=case.ctype, device=DEV)
    gs, gph, gda = case.plan.tffr_adjoint(yt, st, ph, da, want_phase=True, want_dalong=True)
    rgs, rgph, rgda = OP.backward(case.prob, yt.cpu().numpy().astype(np.complex128), s, case.rounded(phase),
                                  case.rounded(dal))
    e1, e2 = rel_l2(gs.cpu().numpy(), rgs), _max_rel(gph.cpu().numpy(), rgph)
    print(f"  forward {rel_l2(got, ref):.3e}, grad_s {e1:.3e}, dphi {e2:.3e}", flush=True)
    assert e1 < tol and e2 < 3 * tol


# ---------------------------------------------------------------- the benchmark's workload
def _workload_case(name, weighting=T.W_TFFR, cb=None, monkeypatch=None, **kw):
    wl = scenes.WORKLOADS[name]
    if cb is not None:
        monkeypatch.setenv("TFFR_AZ_COLS", str(cb))
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov,
                           fov_y=wl.fov, weighting=weighting, **kw)
    plan = T.Plan(prm, k, ku, DEV)
    if cb is not None:
        monkeypatch.delenv("TFFR_AZ_COLS")
    okw = {"thresh_mode": prm.thresh_mode, "tau": prm.tau}
    prob = OP.Problem(k=k, ku=ku, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov, weighting=weighting, **okw)
    return wl, plan, prob


def test_entropy_step_bench_workload_vs_oracle(monkeypatch):
    """512 x 1024 samples -> 1024^2: the fused step in the plan's own launch (two columns
    per azimuth workgroup) and with one and four, against the oracle's image, entropy and
    gradients on every sample and every pulse."""
    wl, plan, prob = _workload_case("ffr_vs_tffr_c64")
    assert plan.az_cols == 2 and plan.range_mode == 3 and plan.ent_fused
    s = scenes.random_samples(wl.n_pulses, wl.n_freq, 901)
    rng = np.random.default_rng(902)
    phase = rng.normal(0, 0.5, wl.n_pulses)
    dal = rng.normal(0, 0.004, wl.n_pulses)
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    ph = torch.as_tensor(phase, dtype=torch.float32, device=DEV)
    da = torch.as_tensor(dal, dtype=torch.float32, device=DEV)
    outs = {2: [x.clone() for x in plan.tffr_entropy_step(st, ph, da)]}
    for cb in (1, 4):
        _, p2, _ = _workload_case("ffr_vs_tffr_c64", cb=cb, monkeypatch=monkeypatch)
        assert p2.az_cols == cb
        outs[cb] = [x.clone() for x in p2.tffr_entropy_step(st, ph, da)]
        del p2
    print("  oracle: full image, entropy gradient, adjoint on every sample", flush=True)
    ref = _oracle_step(prob, s.astype(np.complex64).astype(np.complex128), ph.double().cpu().numpy(),
                       da.double().cpu().numpy())
    for cb, got in outs.items():
        _check_step(f"512x1024 CB={cb}", got, ref)


def test_entropy_gradient_autofocus_workload_vs_oracle():
    """1024 x 2048 samples -> 1024^2 with per-pulse phase errors ~ N(0, 0.5^2): the fused
    step's image and entropy against the oracle's, and d(entropy)/d(phi), d/d(du) and the
    sample gradient on 48 sampled pulses against the oracle's gradient."""
    wl, plan, prob = _workload_case("autofocus_1k")
    assert plan.range_mode == 1 and plan.ent_fused
    s = scenes.random_samples(wl.n_pulses, wl.n_freq, 911)
    rng = np.random.default_rng(912)
    phase = rng.normal(0, wl.phase_sigma, wl.n_pulses)
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    ph = torch.as_tensor(phase, dtype=torch.float32, device=DEV)
    da = torch.zeros(wl.n_pulses, dtype=torch.float32, device=DEV)
    img, loss, gs, gph, gda = (x.cpu().numpy() for x in plan.tffr_entropy_step(st, ph, da))
    s64 = s.astype(np.complex64).astype(np.complex128)
    phr = ph.double().cpu().numpy()
    print("  oracle: full image and entropy gradient", flush=True)
    rimg = OP.image(prob, s64, phr, workers=WORKERS)
    gI = OE.entropy_grad(rimg)
    sel = np.sort(rng.choice(wl.n_pulses, 48, replace=False))
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    sub = OP.Problem(k=k, ku=ku[sel], mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
    rgs, rgph, rgda = OP.backward(sub, gI, s64[sel], phr[sel], np.zeros(len(sel)), workers=WORKERS)
    e_img = rel_l2(img, rimg)
    e_loss = abs(float(loss) - OE.entropy(rimg)) / OE.entropy(rimg)
    e_gs = rel_l2(gs[sel], rgs)
    e_ph = float(np.max(np.abs(gph[sel] - rgph)) / np.max(np.abs(rgph)))
    e_da = float(np.max(np.abs(gda[sel] - rgda)) / np.max(np.abs(rgda)))
    print(f"  image {e_img:.3e} peak {peak_db(img, rimg):.1f} dB, loss {e_loss:.2e}, grad_s (48 pulses) "
          f"{e_gs:.3e}, dphi {e_ph:.3e}, ddu {e_da:.3e}", flush=True)
    assert e_img < 1e-5 and peak_db(img, rimg) < -100 and e_loss < 1e-5
    assert e_gs < GRAD_S_TOL and e_ph < DPHI_TOL and e_da < DPHI_TOL


# ---------------------------------------------------------------- plain FFR at the benchmark's geometry
def test_ffr_bench_geometry():
    """Plain FFR on the 512 x 1024 geometry (1.56-1.83 lattice units between samples):
    D = B_2(pinv(Psi W)) of four sampled slices against the oracle's dense pseudo-inverse,
    and the image of 32 of the workload's slices (same per-slice geometry) against the
    oracle's image with its own weights."""
    wl, plan, prob = _workload_case("ffr_vs_tffr_c64", weighting=T.W_FFR)
    D = plan.tffr_weights().cpu().numpy()
    kx, ky, lam, X, Y = prob.geometry()
    rng = np.random.default_rng(921)
    for n in np.sort(rng.choice(wl.n_pulses, 4, replace=False)):
        ref = OW.ffr_weights(lam[n:n + 1], 0.01, 3.0, 2)[0]
        e = _max_rel(D[n], ref)
        print(f"  slice {n}: D max-rel {e:.2e}", flush=True)
        assert e < 1e-6
    sel = np.sort(rng.choice(wl.n_pulses, 32, replace=False))
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=32, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov,
                           weighting=T.W_FFR)
    sub = T.Plan(prm, k, ku[sel], DEV)
    s = scenes.random_samples(32, wl.n_freq, 922)
    phase = rng.normal(0, 0.5, 32)
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    ph = torch.as_tensor(phase, dtype=torch.float32, device=DEV)
    got = sub.tffr_forward(st, ph).cpu().numpy()
    oprob = OP.Problem(k=k, ku=ku[sel], mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov, weighting=OP.WEIGHT_USER)
    w = OW.ffr_weights(lam[sel], 0.01, 3.0, 2, workers=WORKERS)
    ref = OP.image(oprob, s.astype(np.complex64).astype(np.complex128), ph.double().cpu().numpy(), user_w=w,
                   workers=WORKERS)
    e = rel_l2(got, ref)
    print(f"  32-slice image: rel-L2 {e:.3e} peak {peak_db(got, ref):.1f} dB", flush=True)
    assert e < 1e-5 and peak_db(got, ref) < -100


@pytest.mark.parametrize("dtype", [T.C64, T.C128])
def test_ffr_band_wider_than_frame_product(dtype):
    """B_r with r above the frame product's half-band (r = 7 at a 1.3-1.5 lattice-unit
    spacing, half-band ~4): every entry of the band is the pseudo-inverse's."""
    case = Case(6, 96, 64, fov=40.0, weighting=T.W_FFR, band_r=7, dtype=dtype)
    assert case.plan.ffr_halfband < 7
    got = case.plan.tffr_weights().cpu().numpy()
    kx, ky, lam, X, Y = case.prob.geometry()
    ref = OW.ffr_weights(lam, 0.01, 3.0, 7)
    tol = 1e-12 if dtype == T.C128 else 1e-6
    assert _max_rel(got, ref) < tol


# ---------------------------------------------------------------- correlation threshold
@pytest.mark.parametrize("dtype,width", [(T.C64, 7), (T.C128, 14)])
@pytest.mark.parametrize("size", [(64, 128, 128), (33, 100, 50)])
def test_correlation_threshold_forward_adjoint(size, dtype, width):
    """Threshold on the correlation (keep iff g >= tau = 0.97, about half the samples at
    q = 3): the kept count, the image and the adjoint against the oracle."""
    print(f"correlation threshold size={size} dtype={dtype}", flush=True)
    case = Case(*size, fov=400.0, dtype=dtype, width=width, seed=131, thresh_mode=T.THRESH_CORRELATION)
    kx, ky, lam, X, Y = case.prob.geometry()
    _, kept = OW.tffr_weights(lam, 0.01, 3.0, 0.97, OW.THRESH_CORRELATION)
    c = case.plan.tffr_kept_count()
    print(f"  kept {c} of {kept.size}", flush=True)
    assert c == int(kept.sum()) and 0.3 * kept.size < c < 0.7 * kept.size
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, size[0])
    got = case.plan.tffr_forward(st, case.real(phase)).cpu().numpy()
    ref = OP.image(case.prob, s, case.rounded(phase))
    tol = 1e-10 if dtype == T.C128 else 1e-5
    assert rel_l2(got, ref) < tol and peak_db(got, ref) < 20 * np.log10(tol)
    yt = torch.as_tensor(case.image_np(), dtype=case.ctype, device=DEV)
    gs, gph, _ = case.plan.tffr_adjoint(yt, st, case.real(phase), want_phase=True)
    rgs, rgph, _ = OP.backward(case.prob, yt.cpu().numpy().astype(np.complex128), s, case.rounded(phase))
    assert rel_l2(gs.cpu().numpy(), rgs) < tol
    # thresholded samples receive exactly zero gradient
    assert np.all(gs.cpu().numpy()[~kept] == 0)


def test_correlation_threshold_bench_workload():
    """512 x 1024 -> 1024^2 with the correlation threshold: the kept count equals the
    oracle's exactly, and sampled image columns match the oracle."""
    wl, plan, prob = _workload_case("ffr_vs_tffr_c64", thresh_mode=T.THRESH_CORRELATION)
    kx, ky, lam, X, Y = prob.geometry()
    _, kept = OW.tffr_weights(lam, 0.01, 3.0, 0.97, OW.THRESH_CORRELATION)
    assert plan.tffr_kept_count() == int(kept.sum())
    s = scenes.random_samples(wl.n_pulses, wl.n_freq, 931)
    st = torch.as_tensor(s, dtype=torch.complex64, device=DEV)
    got = plan.tffr_forward(st).cpu().numpy()
    cols = np.sort(np.random.default_rng(932).choice(wl.m, 16, replace=False))
    ref = OP.image_columns(prob, s.astype(np.complex64).astype(np.complex128), cols, workers=WORKERS)
    e = rel_l2(got[cols], ref)
    print(f"  kept {int(kept.sum())} of {kept.size}; 16 columns rel-L2 {e:.3e}", flush=True)
    assert e < 1e-5 and peak_db(got[cols], ref) < -100


# ---------------------------------------------------------------- plain FFR where the frame product is rank deficient
@pytest.mark.parametrize("fov,spacing", [(50.0, "0.39-0.46 (the 2048 x 4096 spacing)"),
                                         (25.0, "0.20-0.23 (the 4096 x 8192 spacing)")])
@pytest.mark.parametrize("dtype", [T.C64, T.C128])
def test_ffr_rank_deficient_vs_pseudo_inverse(fov, spacing, dtype):
    """512 samples per slice at the dense workloads' lattice spacing: more samples than
    lattice points, so the frame product Psi W has rank L < P.  D = B_2(pinv(Psi W)) from
    the factored route (band of (Sa Sb)^-1 by selected inversion) against the oracle's SVD
    pseudo-inverse of the dense product, and the image against the oracle with its own D."""
    print(f"ffr rank-deficient, spacing {spacing}, dtype {dtype}", flush=True)
    case = Case(12, 512, 64, fov=fov, weighting=T.W_FFR, dtype=dtype, width=7 if dtype == T.C64 else 14, seed=141)
    assert case.plan.ffr_route == 1
    kx, ky, lam, X, Y = case.prob.geometry()
    assert lam.shape[1] > lam[0, -1] - lam[0, 0] + 6  # more samples than lattice points
    D = case.plan.tffr_weights().cpu().numpy()
    ref = OW.ffr_weights(lam, 0.01, 3.0, 2, workers=WORKERS)
    e = _max_rel(D, ref)
    print(f"  D max-rel {e:.2e} (max |D| {np.max(np.abs(ref)):.3e})", flush=True)
    # Normal-equation route: the error bound grows with the condition number of Sa Sb after
    # equilibration (~1e8 here), 1e-8 of max |D| in FP64; FP32 storage adds 6e-8.
    assert e < (1e-7 if dtype == T.C128 else 1e-6)
    s, st = case.samples()
    phase = case.rng.normal(0, 0.5, 12)
    got = case.plan.tffr_forward(st, case.real(phase)).cpu().numpy()
    prob = OP.Problem(k=case.k, ku=case.ku, mx=64, my=64, fov_x=fov, fov_y=fov, weighting=OP.WEIGHT_USER)
    img = OP.image(prob, s, case.rounded(phase), user_w=ref)
    tol = 1e-7 if dtype == T.C128 else 1e-5  # the error of D above carries over
    print(f"  image rel-L2 {rel_l2(got, img):.3e}", flush=True)
    assert rel_l2(got, img) < tol


@pytest.mark.parametrize("n,tol", [(1024, 1e-6), (44, 3e-5), (344, 1e-2)])
def test_ffr_precision_workload_sampled_slices(n, tol):
    """Plain FFR on the 2048 x 4096 geometry (4096 samples over ~1610-1850 lattice points
    per slice): D of one slice against the oracle's SVD pseudo-inverse.  Slice 1024 is
    well scaled (cond(A) 75).  Slice 44: its last lattice point is reached by two samples
    with taps of 3e-3, so Sa Sb has a condition number of 4e15 (1e11 after
    equilibration) and the product Psi W one of 6e7; the normal-equation route keeps
    ~5 digits of max |D|.  Slice 344, the worst of the geometry: its last lattice point
    lies 2.9996 lattice units from the only sample that reaches it (q = 3), the product's
    condition number is 6e10 and D is not determined by FP64 arithmetic away from that
    point (the oracle's SVD and a QR evaluation of B (B^T B)^-1 (A^T A)^-1 A^T differ by
    O(1) in the middle of the slice); the point sets max |D| = 6.6e9, and the comparison,
    relative to it, holds to 1e-2."""
    wl, plan, prob = _workload_case("precision_2k", weighting=T.W_FFR)
    assert plan.ffr_route == 1 and plan.ffr_solve_status == 0
    D = plan.tffr_weights().cpu().numpy()
    assert np.all(np.abs(D).reshape(wl.n_pulses, -1).max(axis=1) > 0)  # every slice solved
    kx, ky, lam, X, Y = prob.geometry()
    print(f"  slice {n}: oracle pseudo-inverse of the 4096 x 4096 product", flush=True)
    ref = OW.ffr_weights(lam[n:n + 1], 0.01, 3.0, 2)[0]
    e = _max_rel(D[n], ref)
    print(f"  slice {n}: D max-rel {e:.2e} (max |D| {np.max(np.abs(ref)):.3e})", flush=True)
    assert e < tol


def test_ffr_singular_geometry_is_refused():
    """1024 x 2048 (samples 0.78-0.91 lattice units apart, as many samples as lattice points):
    the truncated frame product is singular to working precision (equilibrated cond(A) up
    to 6e10), so the plan refuses plain FFR with TFFR_ERR_SINGULAR instead of returning
    weights with no correct digit."""
    wl = scenes.WORKLOADS["autofocus_1k"]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov,
                           weighting=T.W_FFR)
    assert T.tffr_validate(prm, k, ku) == 0  # routed; the singularity shows in the solve
    with pytest.raises(RuntimeError, match="TFFR_ERR_SINGULAR"):
        T.Plan(prm, k, ku, DEV)


def test_ffr_full_swath_solves_every_slice():
    """4096 x 8192 (rank-deficient route, Gram systems of ~1850 lattice points per slice):
    every slice solves, and the weights are finite and nonzero in every slice.  (No slice
    is compared with the oracle here: one 8192 x 8192 SVD takes minutes; the 0.20-0.23
    spacing of this geometry is checked against the oracle on 512-sample slices above.)"""
    wl = scenes.WORKLOADS["full_swath_4k"]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    prm = T.default_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov,
                           weighting=T.W_FFR)
    plan = T.Plan(prm, k, ku, DEV)
    assert plan.ffr_route == 1 and plan.ffr_solve_status == 0
    D = plan.tffr_weights()
    assert bool(torch.isfinite(D).all())
    assert bool((D.abs().reshape(wl.n_pulses, -1).amax(dim=1) > 0).all())
