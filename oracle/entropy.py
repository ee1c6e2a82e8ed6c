"""Oracle image-entropy loss (FP64), used to drive autofocus-style gradients.

Test infrastructure only (see the package docstring).

E(I) = -sum_j p_j ln p_j with p_j = |I_j|^2 / S and S = sum_j |I_j|^2 (0 ln 0 = 0).
The paper measures entropy of image regions (TBED, Eq. (10)); here the entropy of the
whole magnitude image is the differentiable focus criterion.
"""

import numpy as np


def entropy(image):
    a = np.abs(np.asarray(image, dtype=np.complex128)) ** 2
    S = a.sum()
    p = a / S
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(p > 0, p * np.log(p), 0.0)
    return -t.sum()


def entropy_grad(image):
    """dE/dRe I + i dE/dIm I = -(2/S) (ln p_j + E) I_j, and 0 where I_j = 0."""
    I = np.asarray(image, dtype=np.complex128)
    a = np.abs(I) ** 2
    S = a.sum()
    E = entropy(I)
    with np.errstate(divide="ignore", invalid="ignore"):
        lp = np.where(a > 0, np.log(a / S), 0.0)
    return np.where(a > 0, -(2.0 / S) * (lp + E) * I, 0.0)
