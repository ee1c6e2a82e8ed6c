"""Oracle end-to-end path (FP64): phasing, weighting, imaging, adjoint and gradients.

Test infrastructure only (see the package docstring).

Forward, for one batch of phase-history samples s[n, p] (n: pulse / azimuth slice,
p: fast-time frequency):

    s'[n,p] = s[n,p] exp(i (phi[n] + ky[n] du[n]))      per-pulse phase and along-track
                                                          position errors (autofocus model)
    c[n,.]  = D^(n) s'[n,.]                              weights of the chosen method
    I       = sum_{n,p} c[n,p] exp(i (kx X + ky Y))      Eq. (1) / Eq. (8), see nudft

The gradient of a real loss L(I) follows the PyTorch convention for complex tensors
(dL/dRe + i dL/dIm):

    grad_c  = A^H grad_I,  grad_s' = D^T grad_c,  grad_s = exp(-i psi) grad_s'
    dL/dphi[n] = sum_p Re(conj(grad_s'[n,p]) i s'[n,p]),   dL/ddu[n] = ky[n] dL/dphi[n].
"""

from dataclasses import dataclass

import numpy as np

from . import geometry, nudft, weights

WEIGHT_NONE = 0
WEIGHT_QUAD = 1
WEIGHT_FFR = 2
WEIGHT_TFFR = 3
WEIGHT_USER = 4


@dataclass
class Problem:
    """Geometry and method parameters of one reconstruction (Algorithm 1's inputs)."""

    k: np.ndarray  # [n_freq] fast-time wavenumbers, rad/m, strictly increasing
    ku: np.ndarray  # [n_pulses] azimuth wavenumbers, rad/m
    mx: int  # image size in range
    my: int  # image size in azimuth
    fov_x: float  # range field of view, m
    fov_y: float  # azimuth field of view, m
    weighting: int = WEIGHT_TFFR
    a: float = 0.01  # window w(x) = exp(-a|x - 1/2|)
    q: float = 3.0  # truncation of W and Psi, lattice units
    r: int = 2  # FFR band
    tau: float = 0.97  # tFFR threshold
    thresh_mode: int = weights.THRESH_LITERAL
    # explicit sample coordinates instead of the Stolt map of (k, ku): kx [n_pulses][n_freq],
    # ky [n_pulses] (each slice keeps one ky, as the slice structure of Algorithm 1 needs)
    kx_explicit: np.ndarray = None
    ky_explicit: np.ndarray = None

    def geometry(self):
        if self.kx_explicit is not None:
            kx = np.asarray(self.kx_explicit, dtype=np.float64)
            ky = np.asarray(self.ky_explicit, dtype=np.float64)
        else:
            kx, ky = geometry.stolt(self.k, self.ku)
        lam = geometry.lattice_coordinate(kx, self.fov_x)
        X = geometry.pixel_coordinates(self.mx, self.fov_x)
        Y = geometry.pixel_coordinates(self.my, self.fov_y)
        return kx, ky, lam, X, Y


def sample_weights(prob, user_w=None):
    """Weights of the chosen method: [n_pulses][n_freq] (diagonal) or [..][2r+1] (FFR)."""
    kx, ky, lam, X, Y = prob.geometry()
    if prob.weighting == WEIGHT_NONE:
        return np.ones_like(lam)
    if prob.weighting == WEIGHT_QUAD:
        return weights.quad_weights(lam)
    if prob.weighting == WEIGHT_TFFR:
        d, _ = weights.tffr_weights(lam, prob.a, prob.q, prob.tau, prob.thresh_mode)
        return d
    if prob.weighting == WEIGHT_FFR:
        return weights.ffr_weights(lam, prob.a, prob.q, prob.r)
    if prob.weighting == WEIGHT_USER:
        return np.asarray(user_w, dtype=np.float64)
    raise ValueError("unknown weighting")


def row_phase(ky, phase=None, dalong=None):
    """psi[n] = phi[n] + ky[n] du[n]; zero where the inputs are absent."""
    psi = np.zeros_like(np.asarray(ky, dtype=np.float64))
    if phase is not None:
        psi = psi + np.asarray(phase, dtype=np.float64)
    if dalong is not None:
        psi = psi + np.asarray(ky, dtype=np.float64) * np.asarray(dalong, dtype=np.float64)
    return psi


def apply_weights(w, x, transpose=False):
    """c = D x per row (diagonal or banded); with transpose=True, D^T x."""
    x = np.asarray(x, dtype=np.complex128)
    if w.ndim == 2:
        return w * x
    out = np.empty_like(x)
    for n in range(x.shape[0]):
        D = weights.band_to_dense(w[n])
        out[n] = (D.T if transpose else D) @ x[n]
    return out


def weighted_samples(prob, s, phase=None, dalong=None, user_w=None):
    kx, ky, lam, X, Y = prob.geometry()
    psi = row_phase(ky, phase, dalong)
    sp = np.asarray(s, dtype=np.complex128) * np.exp(1j * psi)[:, None]
    return apply_weights(sample_weights(prob, user_w), sp)


def image(prob, s, phase=None, dalong=None, user_w=None, form="separable", workers=1):
    """The reconstructed image I[jx, jy] (range-major)."""
    kx, ky, lam, X, Y = prob.geometry()
    c = weighted_samples(prob, s, phase, dalong, user_w)
    if form == "direct":
        return nudft.forward_direct(c, kx, ky, X, Y)
    return nudft.forward_separable(c, kx, ky, X, Y, workers)


def image_columns(prob, s, cols, phase=None, dalong=None, user_w=None, workers=1):
    kx, ky, lam, X, Y = prob.geometry()
    c = weighted_samples(prob, s, phase, dalong, user_w)
    return nudft.forward_columns(c, kx, ky, X, Y, cols, workers)


def backward(prob, grad_image, s, phase=None, dalong=None, user_w=None, workers=1):
    """Gradients of a real loss given grad_image = dL/dRe I + i dL/dIm I.

    Returns (grad_s, grad_phase, grad_dalong).
    """
    kx, ky, lam, X, Y = prob.geometry()
    psi = row_phase(ky, phase, dalong)
    rot = np.exp(1j * psi)[:, None]
    sp = np.asarray(s, dtype=np.complex128) * rot
    grad_c = nudft.adjoint(grad_image, kx, ky, X, Y, workers)
    grad_sp = apply_weights(sample_weights(prob, user_w), grad_c, transpose=True)
    grad_s = grad_sp * np.conj(rot)
    dpsi = np.sum(np.real(np.conj(grad_sp) * 1j * sp), axis=1)
    return grad_s, dpsi, ky * dpsi


def coordinate_gradients(prob, grad_image, s, phase=None, dalong=None, user_w=None):
    """Gradients of a real loss with respect to the sample coordinates, the method's
    weights held fixed (they are constants of the geometry in the forward map):

        dI_j / dkx[n,p] = i X_jx c[n,p] exp(i(kx X_jx + ky Y_jy)),  and likewise with Y for ky[n]

    so with dL = Re(sum_j conj(G_j) dI_j), G = grad_image:

        dL/dkx[n,p] = Re(i c[n,p] conj((A^H (X G))[n,p]))
        dL/dky[n]   = sum_p Re(i c[n,p] conj((A^H (Y G))[n,p]))

    A^H the plain adjoint sum (nudft.adjoint).  Returns (grad_kx [n][p], grad_ky [n]).
    """
    kx, ky, lam, X, Y = prob.geometry()
    c = weighted_samples(prob, s, phase, dalong, user_w)
    G = np.asarray(grad_image, dtype=np.complex128)
    aX = nudft.adjoint(X[:, None] * G, kx, ky, X, Y)
    aY = nudft.adjoint(Y[None, :] * G, kx, ky, X, Y)
    gkx = np.real(1j * c * np.conj(aX))
    gky = np.sum(np.real(1j * c * np.conj(aY)), axis=1)
    return gkx, gky

