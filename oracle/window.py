"""Oracle window transforms (FP64): the entries of W and Psi.

Test infrastructure only (see the package docstring).

The window of the NUFFT, FFR and tFFR is w(x) = exp(-a |x - 1/2|) on the unit image
interval, with a = 0.01 (Sec. IV, Baselines).  W collects its Fourier transform at
grid-minus-sample offsets (the matrix after Eq. (7)), and Psi collects inner products of
a Fourier mode with a grid mode divided by w (Eq. (6)), which the paper evaluates in
closed form (end of Sec. III-C).

Reading taken: both transforms are over the finite image interval (the frame's domain),
not over the real line.  On the interval centred at the window's peak the transforms of
w and of 1/w are real and even:

    R_W(d)   = integral_{-1/2}^{1/2} exp(-a|t|) cos(2 pi d t) dt
    R_Psi(d) = integral_{-1/2}^{1/2} exp(+a|t|) cos(2 pi d t) dt

The un-centred [0, 1] transforms differ from these by unimodular phases
exp(-+ i pi d), which cancel in every product the weights use (the diagonal of the
frame product) and amount to a diagonal unitary similarity for the band (plain FFR).
"""

import numpy as np


def r_w(d, a):
    """R_W(d): finite-interval cosine transform of exp(-a|t|), closed form.

    Integrating exp(-a t) cos(b t) over [0, 1/2] with b = 2 pi d gives
    2 [a + exp(-a/2) (b sin(b/2) - a cos(b/2))] / (a^2 + b^2).
    """
    d = np.asarray(d, dtype=np.float64)
    a = float(a)
    b = 2.0 * np.pi * d
    num = a + np.exp(-a / 2.0) * (b * np.sin(b / 2.0) - a * np.cos(b / 2.0))
    den = a * a + b * b
    with np.errstate(invalid="ignore", divide="ignore"):
        out = 2.0 * num / den
    if a == 0.0:
        out = np.where(d == 0.0, 1.0, out)
    return out


def r_psi(d, a):
    """R_Psi(d): finite-interval cosine transform of 1/w = exp(+a|t|), closed form.

    Integrating exp(+a t) cos(b t) over [0, 1/2] with b = 2 pi d gives
    2 [exp(a/2) (b sin(b/2) + a cos(b/2)) - a] / (a^2 + b^2).
    """
    d = np.asarray(d, dtype=np.float64)
    a = float(a)
    b = 2.0 * np.pi * d
    num = np.exp(a / 2.0) * (b * np.sin(b / 2.0) + a * np.cos(b / 2.0)) - a
    den = a * a + b * b
    with np.errstate(invalid="ignore", divide="ignore"):
        out = 2.0 * num / den
    if a == 0.0:
        out = np.where(d == 0.0, 1.0, out)
    return out
