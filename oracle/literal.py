"""Oracle of the literal Algorithm-1 range gridding (FP64).

Test infrastructure only (see the package docstring).

Eq. (8) and Algorithm 1 as printed: per azimuth slice, the weighted samples are spread
onto the integer lattice l_m (cycles per range field of view) with the window transform
truncated to |l_m - lambda| < q, the lattice is inverse-transformed, and the result is
divided by the window w in the image domain.  In the centred pixel convention of this
package (range pixel X_j = (j - M/2) L / M, so u_j = X_j / L = (j - M/2) / M lies in
[-1/2, 1/2) and w(u) = exp(-a |u|)):

    G_n[m]   = sum_{p : |m - lam_np| < q} c_np R_W(m - lam_np)         (spread)
    H_n[j]   = exp(a |u_j|) sum_m G_n[m] exp(2 pi i m u_j)              (inverse DFT, / w)
    I[j, k]  = sum_n H_n[j] exp(i ky_n Y_k)                             (azimuth: exact)

R_W is the centred finite-interval transform of w (oracle.window.r_w), i.e. the Fourier
coefficients of w on the interval: sum over all integers m of R_W(m - lam) exp(2 pi i m u)
is w(u) exp(2 pi i lam u) for |u| < 1/2.  With the m-sum untruncated H_n is therefore the
exact range sum sum_p c_np exp(2 pi i lam_np u_j); the truncation |m - lam| < q is the
method's approximation, and this module computes it exactly as defined (explicit DFT over
the lattice points the samples reach, no FFT, no folding).
"""

import numpy as np

from . import window


def lattice_spread(c_row, lam_row, a, q):
    """G[m] for one slice: (m_lo, G) with G[i] the value at lattice point m_lo + i."""
    lam_row = np.asarray(lam_row, dtype=np.float64)
    c_row = np.asarray(c_row, dtype=np.complex128)
    K = int(np.ceil(q)) + 1
    m_lo = int(np.floor(lam_row.min())) - K
    m_hi = int(np.ceil(lam_row.max())) + K
    G = np.zeros(m_hi - m_lo + 1, dtype=np.complex128)
    for cp, lp in zip(c_row, lam_row):
        base = int(np.floor(lp))
        for m in range(base - K, base + K + 1):
            d = m - lp
            if abs(d) < q:
                G[m - m_lo] += cp * window.r_w(d, a)
    return m_lo, G


def range_spectra(c, lam, mx, a, q):
    """H[n][j] of the literal range stage for all slices ([n_pulses][mx])."""
    c = np.asarray(c, dtype=np.complex128)
    lam = np.asarray(lam, dtype=np.float64)
    u = (np.arange(mx) - mx / 2) / mx
    inv_w = np.exp(float(a) * np.abs(u))
    out = np.empty((c.shape[0], mx), dtype=np.complex128)
    for n in range(c.shape[0]):
        m_lo, G = lattice_spread(c[n], lam[n], a, q)
        m = m_lo + np.arange(G.size)
        out[n] = inv_w * (np.exp(2j * np.pi * np.outer(u, m)) @ G)
    return out


def image(prob, s, phase=None, dalong=None, user_w=None):
    """The image of the literal range gridding with the exact azimuth sum ([mx][my])."""
    from . import pipeline

    kx, ky, lam, X, Y = prob.geometry()
    c = pipeline.weighted_samples(prob, s, phase, dalong, user_w)
    H = range_spectra(c, lam, prob.mx, prob.a, prob.q)
    return H.T @ np.exp(1j * np.outer(ky, Y))
