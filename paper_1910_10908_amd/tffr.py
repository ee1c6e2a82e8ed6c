"""Python binding of libtffr with the same names as the C ABI, plus torch.autograd wrappers.

PyTorch only supplies device memory and the current stream; every step of the path
runs in libtffr's HIP kernels.  Tensors must be contiguous and on the plan's device.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (C64, C64_FP16IN, C128, GRID_ES, GRID_LITERAL, THRESH_CORRELATION, THRESH_LITERAL,  # noqa: F401
                   W_FFR, W_NONE, W_QUAD, W_TFFR, W_USER, Params)

_DT = {C64: (torch.complex64, torch.float32), C128: (torch.complex128, torch.float64),
       C64_FP16IN: (torch.complex64, torch.float32)}


def default_params(**kw):
    p = Params()
    _lib.load().tffr_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tffr_validate(params, k, ku):
    k = np.ascontiguousarray(k, dtype=np.float64)
    ku = np.ascontiguousarray(ku, dtype=np.float64)
    return _lib.load().tffr_validate(ctypes.byref(params), _dptr(k), _dptr(ku))


def tffr_validate_xy(params, kx, ky):
    kx = np.ascontiguousarray(kx, dtype=np.float64)
    ky = np.ascontiguousarray(ky, dtype=np.float64)
    if kx.shape != (params.n_pulses, params.n_freq) or ky.shape != kx.shape:
        raise ValueError("kx / ky must be [n_pulses][n_freq]")
    return _lib.load().tffr_validate_xy(ctypes.byref(params), _dptr(kx), _dptr(ky))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """tffr_plan_create / tffr_plan_destroy, and the calls that take a plan."""

    def __init__(self, params, k, ku, device="cuda:0", kx=None, ky=None):
        """Plan from radar wavenumbers k [n_freq], ku [n_pulses] (Stolt map), or, with k and
        ku None, from explicit coordinates kx, ky [n_pulses][n_freq] (tffr_plan_create_xy)."""
        self.lib = _lib.load()
        self.params = params
        self.device = torch.device(device)
        self.ctype, self.rtype = _DT[params.dtype]
        h = ctypes.c_void_p()
        if kx is not None:
            self.kx = np.ascontiguousarray(kx, dtype=np.float64)
            kyv = np.ascontiguousarray(ky, dtype=np.float64)
            if self.kx.shape != (params.n_pulses, params.n_freq) or kyv.shape != self.kx.shape:
                raise ValueError("kx / ky must be [n_pulses][n_freq]")
            self.k, self.ku = None, kyv[:, 0].copy()
            with torch.cuda.device(self.device):
                _lib.check(self.lib.tffr_plan_create_xy(ctypes.byref(params), _dptr(self.kx), _dptr(kyv),
                                                        ctypes.byref(h)), "tffr_plan_create_xy")
        else:
            self.kx = None
            self.k = np.ascontiguousarray(k, dtype=np.float64)
            self.ku = np.ascontiguousarray(ku, dtype=np.float64)
            if self.k.size != params.n_freq or self.ku.size != params.n_pulses:
                raise ValueError("k / ku sizes do not match params")
            with torch.cuda.device(self.device):
                _lib.check(self.lib.tffr_plan_create(ctypes.byref(params), _dptr(self.k), _dptr(self.ku),
                                                     ctypes.byref(h)), "tffr_plan_create")
        self.handle = h
        nfx, nfy, hb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        beta = ctypes.c_double()
        _lib.check(self.lib.tffr_plan_info(h, ctypes.byref(nfx), ctypes.byref(nfy), ctypes.byref(beta),
                                           ctypes.byref(hb)))
        self.nfine = (nfx.value, nfy.value)
        self.beta = beta.value
        self.ffr_halfband = hb.value
        self.work = torch.empty(int(self.lib.tffr_workspace_bytes(h)), dtype=torch.uint8, device=self.device)
        rm, cb, fu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self.lib.tffr_debug_plan_config(h, ctypes.byref(rm), ctypes.byref(cb), ctypes.byref(fu)))
        self.range_mode, self.az_cols, self.ent_fused = rm.value, cb.value, bool(fu.value)
        self.ffr_route, self.ffr_lattice_max, self.ffr_solve_status = None, None, None
        if params.weighting == W_FFR:
            ro, lm, fs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _lib.check(self.lib.tffr_debug_ffr_route(h, ctypes.byref(ro), ctypes.byref(lm), ctypes.byref(fs)))
            self.ffr_route, self.ffr_lattice_max, self.ffr_solve_status = ro.value, lm.value, fs.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.tffr_plan_destroy(h)
            self.handle = None

    # ---------------------------------------------------------------- checks
    @property
    def shape_samples(self):
        return (self.params.n_pulses, self.params.n_freq)

    @property
    def shape_image(self):
        return (self.params.mx, self.params.my)

    def _chk(self, t, shape, dtype, name):
        if t is None:
            return None
        if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {self.device}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def _chk_samples(self, s):
        if self.params.dtype == C64_FP16IN:
            return self._chk(s, self.shape_samples + (2,), torch.float16, "samples")
        return self._chk(s, self.shape_samples, self.ctype, "samples")

    def _chk_weights(self, w):
        if w is None:
            return None
        shape = self.shape_samples
        if self.params.weighting == W_FFR:
            shape = shape + (2 * self.params.band_r + 1,)
        return self._chk(w, shape, self.rtype, "weights")

    # ---------------------------------------------------------------- calls
    def tffr_forward(self, samples, phase=None, dalong=None, user_w=None, out=None):
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        self._chk_weights(user_w)
        if out is None:
            out = torch.empty(self.shape_image, dtype=self.ctype, device=self.device)
        self._chk(out, self.shape_image, self.ctype, "image")
        _lib.check(self.lib.tffr_forward(self.handle, _ptr(samples), _ptr(phase), _ptr(dalong), _ptr(user_w),
                                         _ptr(out), _ptr(self.work), _stream()), "tffr_forward")
        return out

    def tffr_rma_range_fft(self, pulses, ref=None, out=None):
        """Time-domain pulses [n_positions][n_freq] -> their centred frequency bins times the
        matched filter's reference spectrum ref [n_freq] (None: ones)."""
        J = int(pulses.shape[0]) if pulses.dim() >= 1 else 0
        ct = torch.complex128 if self.params.dtype == C128 else torch.complex64
        self._chk(pulses, (J, self.params.n_freq), ct, "pulses")
        self._chk(ref, (self.params.n_freq,), ct, "ref")
        if out is None:
            out = torch.empty_like(pulses)
        self._chk(out, (J, self.params.n_freq), ct, "echoes")
        _lib.check(self.lib.tffr_rma_range_fft(self.handle, _ptr(pulses), J, _ptr(ref), _ptr(out), _stream()),
                   "tffr_rma_range_fft")
        return out

    def tffr_rma_front_end(self, echoes, du, xc, out=None, dpos=None):
        """Raw echoes [n_positions][n_freq] (complex compute type) -> samples of this plan.
        dpos: host sequence of per-position along-track errors (m), or None for the
        nominal positions."""
        J = int(echoes.shape[0]) if echoes.dim() >= 1 else 0
        ct = torch.complex128 if self.params.dtype == C128 else torch.complex64
        self._chk(echoes, (J, self.params.n_freq), ct, "echoes")
        if out is None:
            if self.params.dtype == C64_FP16IN:
                out = torch.empty(self.shape_samples + (2,), dtype=torch.float16, device=self.device)
            else:
                out = torch.empty(self.shape_samples, dtype=self.ctype, device=self.device)
        self._chk_samples(out)
        if dpos is None:
            _lib.check(self.lib.tffr_rma_front_end(self.handle, _ptr(echoes), J, float(du), float(xc), _ptr(out),
                                                   _stream()), "tffr_rma_front_end")
            return out
        d = np.ascontiguousarray(np.asarray(dpos, dtype=np.float64))
        if d.shape != (J,):
            raise ValueError(f"dpos must have shape ({J},), got {d.shape}")
        _lib.check(self.lib.tffr_rma_front_end_pos(self.handle, _ptr(echoes), J, float(du),
                                                   d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(xc),
                                                   _ptr(out), _stream()), "tffr_rma_front_end_pos")
        return out

    def tffr_stolt_image(self, samples, phase=None, dalong=None, out=None):
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        if out is None:
            out = torch.empty(self.shape_image, dtype=self.ctype, device=self.device)
        self._chk(out, self.shape_image, self.ctype, "image")
        _lib.check(self.lib.tffr_stolt_image(self.handle, _ptr(samples), _ptr(phase), _ptr(dalong), _ptr(out),
                                             _ptr(self.work), _stream()), "tffr_stolt_image")
        return out

    def tffr_adjoint(self, grad_image, samples=None, phase=None, dalong=None, user_w=None,
                     want_phase=False, want_dalong=False, out=None):
        self._chk(grad_image, self.shape_image, self.ctype, "grad_image")
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        self._chk_weights(user_w)
        if out is None:
            out = torch.empty(self.shape_samples, dtype=self.ctype, device=self.device)
        self._chk(out, self.shape_samples, self.ctype, "grad_samples")
        gph = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device) if want_phase else None
        gda = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device) if want_dalong else None
        _lib.check(self.lib.tffr_adjoint(self.handle, _ptr(grad_image), _ptr(samples), _ptr(phase), _ptr(dalong),
                                         _ptr(user_w), _ptr(out), _ptr(gph), _ptr(gda), _ptr(self.work),
                                         _stream()), "tffr_adjoint")
        return out, gph, gda

    def tffr_coord_grad(self, grad_image, samples, phase=None, dalong=None, user_w=None):
        """(dL/dkx [n_pulses][n_freq], dL/dky [n_pulses]) for a cotangent of the image."""
        self._chk(grad_image, self.shape_image, self.ctype, "grad_image")
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        self._chk_weights(user_w)
        gkx = torch.empty(self.shape_samples, dtype=self.rtype, device=self.device)
        gky = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device)
        _lib.check(self.lib.tffr_coord_grad(self.handle, _ptr(grad_image), _ptr(samples), _ptr(phase), _ptr(dalong),
                                            _ptr(user_w), _ptr(gkx), _ptr(gky), _ptr(self.work), _stream()),
                   "tffr_coord_grad")
        return gkx, gky

    def tffr_row_phase_grad(self, samples, grad_samples, want_dalong=True):
        """Per-slice (dL/dphi, dL/d du) from a sample cotangent computed elsewhere."""
        self._chk_samples(samples)
        self._chk(grad_samples, self.shape_samples, self.ctype, "grad_samples")
        gph = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device)
        gda = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device) if want_dalong else None
        _lib.check(self.lib.tffr_row_phase_grad(self.handle, _ptr(samples), _ptr(grad_samples), _ptr(gph),
                                                _ptr(gda), _stream()), "tffr_row_phase_grad")
        return gph, gda

    def tffr_entropy(self, image, want_grad=True):
        self._chk(image, self.shape_image, self.ctype, "image")
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        grad = torch.empty_like(image) if want_grad else None
        _lib.check(self.lib.tffr_entropy(self.handle, _ptr(image), _ptr(loss), _ptr(grad), _ptr(self.work),
                                         _stream()), "tffr_entropy")
        return loss, grad

    def tffr_entropy_step(self, samples, phase=None, dalong=None, user_w=None, want_phase=True,
                          want_dalong=True, out=None):
        """Fused forward + entropy + adjoint of dE/dI.  Returns (image, loss, grad_samples,
        grad_phase, grad_dalong)."""
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        self._chk_weights(user_w)
        img, loss, gs, gph, gda = out if out is not None else (None,) * 5
        if img is None:
            img = torch.empty(self.shape_image, dtype=self.ctype, device=self.device)
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=self.device)
        if gs is None:
            gs = torch.empty(self.shape_samples, dtype=self.ctype, device=self.device)
        if gph is None and want_phase:
            gph = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device)
        if gda is None and want_dalong:
            gda = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device)
        _lib.check(self.lib.tffr_entropy_step(self.handle, _ptr(samples), _ptr(phase), _ptr(dalong), _ptr(user_w),
                                              _ptr(img), _ptr(loss), _ptr(gs), _ptr(gph), _ptr(gda),
                                              _ptr(self.work), _stream()), "tffr_entropy_step")
        return img, loss, gs, gph, gda

    def tffr_entropy_step_noalloc(self, samples, phase=None, dalong=None, user_w=None, out=None):
        """tffr_entropy_step_noalloc: the fused step in the library's static scratch array
        (no workspace).  `out` = (image, loss, grad_samples, grad_phase, grad_dalong), each
        may be None to allocate it here; returns the five."""
        self._chk_samples(samples)
        self._chk(phase, (self.params.n_pulses,), self.rtype, "phase")
        self._chk(dalong, (self.params.n_pulses,), self.rtype, "dalong")
        self._chk_weights(user_w)
        img, loss, gs, gph, gda = out if out is not None else (None,) * 5
        img = torch.empty(self.shape_image, dtype=self.ctype, device=self.device) if img is None else img
        loss = torch.empty((), dtype=torch.float64, device=self.device) if loss is None else loss
        gs = torch.empty(self.shape_samples, dtype=self.ctype, device=self.device) if gs is None else gs
        gph = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device) if gph is None else gph
        gda = torch.empty(self.params.n_pulses, dtype=self.rtype, device=self.device) if gda is None else gda
        _lib.check(self.lib.tffr_entropy_step_noalloc(self.handle, _ptr(samples), _ptr(phase), _ptr(dalong),
                                                      _ptr(user_w), _ptr(img), _ptr(loss), _ptr(gs), _ptr(gph),
                                                      _ptr(gda), _stream()), "tffr_entropy_step_noalloc")
        return img, loss, gs, gph, gda

    def tffr_debug_step_kernel_times(self, samples, phase=None, dalong=None, user_w=None, out=None, nsteps=100):
        """Average time of each launch of the entropy step, in the step's own order (HIP
        events between its launches): {kernel name: microseconds}."""
        img, loss, gs, gph, gda = out
        ms = (ctypes.c_float * 7)()
        nk = ctypes.c_int32()
        names = (ctypes.c_char_p * 7)()
        _lib.check(self.lib.tffr_debug_step_kernel_times(self.handle, _ptr(samples), _ptr(phase), _ptr(dalong),
                                                         _ptr(user_w), _ptr(img), _ptr(loss), _ptr(gs), _ptr(gph),
                                                         _ptr(gda), _ptr(self.work), _stream(), nsteps, ms,
                                                         ctypes.byref(nk), names), "tffr_debug_step_kernel_times")
        return {names[i].decode(): ms[i] * 1e3 for i in range(nk.value)}

    def tffr_debug_step_kernel_marginal_times(self, samples, phase=None, dalong=None, user_w=None, out=None,
                                              nsteps=100):
        """What one more launch of each kernel adds to the entropy step (plain steps against
        steps with that launch issued twice; events around the loops only): {kernel name:
        microseconds}, in the step's order."""
        img, loss, gs, gph, gda = out
        ms = (ctypes.c_float * 7)()
        nk = ctypes.c_int32()
        names = (ctypes.c_char_p * 7)()
        _lib.check(self.lib.tffr_debug_step_kernel_marginal_times(
            self.handle, _ptr(samples), _ptr(phase), _ptr(dalong), _ptr(user_w), _ptr(img), _ptr(loss), _ptr(gs),
            _ptr(gph), _ptr(gda), _ptr(self.work), _stream(), nsteps, ms, ctypes.byref(nk), names),
            "tffr_debug_step_kernel_marginal_times")
        return {names[i].decode(): ms[i] * 1e3 for i in range(nk.value)}

    def tffr_weights(self, out=None):
        shape = self.shape_samples
        if self.params.weighting == W_FFR:
            shape = shape + (2 * self.params.band_r + 1,)
        if out is None:
            out = torch.empty(shape, dtype=self.rtype, device=self.device)
        self._chk(out, shape, self.rtype, "weights")
        _lib.check(self.lib.tffr_weights(self.handle, _ptr(out), _ptr(self.work), _stream()), "tffr_weights")
        return out

    def tffr_kept_count(self):
        c = ctypes.c_int64()
        _lib.check(self.lib.tffr_kept_count(self.handle, _ptr(self.work), ctypes.byref(c), _stream()),
                   "tffr_kept_count")
        return c.value

    def tffr_debug_rows(self, samples, stage=1, phase=None, dalong=None, user_w=None):
        self._chk_samples(samples)
        n = self.nfine[0] if stage == 0 else self.params.mx
        out = torch.empty((self.params.n_pulses, n), dtype=self.ctype, device=self.device)
        _lib.check(self.lib.tffr_debug_rows(self.handle, stage, _ptr(samples), _ptr(phase), _ptr(dalong),
                                            _ptr(user_w), _ptr(out), _stream()), "tffr_debug_rows")
        return out


def tffr_debug_cols(plan, hx, out=None):
    """Azimuth stage of the forward path alone: range spectra [n_pulses][mx] -> image."""
    plan._chk(hx, (plan.params.n_pulses, plan.params.mx), plan.ctype, "hx")
    if out is None:
        out = torch.empty(plan.shape_image, dtype=plan.ctype, device=plan.device)
    _lib.check(plan.lib.tffr_debug_cols(plan.handle, _ptr(hx), _ptr(out), _stream()), "tffr_debug_cols")
    return out


def tffr_debug_ent_cols(plan, hx):
    """Fused entropy-step azimuth stage alone: range spectra -> (image, h1, h2), where h1
    and h2 are the adjoint azimuth transforms of I (ln|I|^2 - c_b) and of I."""
    plan._chk(hx, (plan.params.n_pulses, plan.params.mx), plan.ctype, "hx")
    img = torch.empty(plan.shape_image, dtype=plan.ctype, device=plan.device)
    h12 = torch.empty((plan.params.n_pulses, plan.params.mx, 2), dtype=plan.ctype, device=plan.device)
    _lib.check(plan.lib.tffr_debug_ent_cols(plan.handle, _ptr(hx), _ptr(img), _ptr(h12), _ptr(plan.work),
                                            _stream()), "tffr_debug_ent_cols")
    return img, h12[..., 0], h12[..., 1]


def tffr_debug_fft(x, sign, max_radix=8):
    """Batched LDS FFT of the rows of x (complex64/complex128, power-of-two length)."""
    lib = _lib.load()
    x = x.contiguous()
    n = x.shape[-1]
    log2n = int(round(np.log2(n)))
    dtype = C128 if x.dtype == torch.complex128 else C64
    out = torch.empty_like(x)
    _lib.check(lib.tffr_debug_fft(log2n, x.numel() // n, sign, max_radix, dtype, _ptr(x), _ptr(out), _stream()),
               "tffr_debug_fft")
    return out


# -------------------------------------------------------------------- autograd
class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, samples, phase, dalong, user_w):
        ctx.plan = plan
        ctx.save_for_backward(samples, phase, dalong, user_w)
        return plan.tffr_forward(samples, phase, dalong, user_w)

    @staticmethod
    def backward(ctx, grad_image):
        plan = ctx.plan
        samples, phase, dalong, user_w = ctx.saved_tensors
        want_ph = phase is not None and ctx.needs_input_grad[2]
        want_da = dalong is not None and ctx.needs_input_grad[3]
        gs, gph, gda = plan.tffr_adjoint(grad_image.contiguous(), samples if (want_ph or want_da) else None,
                                         phase, dalong, user_w, want_phase=want_ph, want_dalong=want_da)
        return None, (gs if ctx.needs_input_grad[1] else None), gph, gda, None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, image, user_w):
        ctx.plan = plan
        ctx.save_for_backward(user_w)
        gs, _, _ = plan.tffr_adjoint(image, None, None, None, user_w)
        return gs

    @staticmethod
    def backward(ctx, grad_samples):
        (user_w,) = ctx.saved_tensors
        return None, ctx.plan.tffr_forward(grad_samples.contiguous(), None, None, user_w), None


class _Entropy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, image):
        loss, grad = plan.tffr_entropy(image, want_grad=True)
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return None, grad * g.to(grad.real.dtype)


class TFFR:
    """The plan's forward map as a differentiable operator:
    TFFR(plan).apply(samples, phase, dalong) -> image; backward is the adjoint (sample,
    per-pulse phase and along-track position gradients), and TFFRAdjoint(plan) is its
    transpose.  Tensors must be contiguous on the plan's device (phase / dalong may be
    None)."""

    def __init__(self, plan, user_w=None):
        self.plan, self.user_w = plan, user_w

    def apply(self, samples, phase=None, dalong=None):
        return _Forward.apply(self.plan, samples, phase, dalong, self.user_w)


class TFFRAdjoint:
    """TFFRAdjoint(plan).apply(image) -> samples: the adjoint operator, differentiable (its
    backward is the forward map)."""

    def __init__(self, plan, user_w=None):
        self.plan, self.user_w = plan, user_w

    def apply(self, image):
        return _Adjoint.apply(self.plan, image, self.user_w)


def tffr_image(plan, samples, phase=None, dalong=None, user_w=None):
    """Differentiable image formation: samples, phase, dalong -> image (range-major)."""
    return _Forward.apply(plan, samples, phase, dalong, user_w)


def tffr_adjoint_op(plan, image, user_w=None):
    """Differentiable adjoint operator A^H (its backward is the forward operator)."""
    return _Adjoint.apply(plan, image, user_w)


def image_entropy(plan, image):
    """Differentiable image entropy (FP64 scalar)."""
    return _Entropy.apply(plan, image)
