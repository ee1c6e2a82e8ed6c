"""Oracle range-migration front end and Stolt-interpolation baseline (FP64).

Test infrastructure only (see the package docstring).

Front end (Sec. II-A: the data are mapped to the frequency domain and matched filtered
before the Stolt change of variables).  Raw echoes e[j, p] are recorded at J uniform
along-track positions u_j = (j - J/2) du for fast-time wavenumbers k_p; a point
scatterer at range X_c + x and along-track position y contributes
a exp(-2 i k_p R(u_j)), R(u) = sqrt((X_c + x)^2 + (y - u)^2).  The front end

    s[n, p] = exp(+i kx[n, p] X_c) * sum_j e[j, p] exp(-i ku_n u_j)

with ku_n = (n - N_u/2) dku, dku = 2 pi / (J du), n = 0..N_u-1 (the N_u azimuth
wavenumbers nearest zero of the J-point transform) and kx = sqrt(4 k^2 - ku^2).  By
stationary phase the azimuth transform of one scatterer's echo carries the phase
-(sqrt(4 k^2 - ku^2) (X_c + x) + ku y); the reference function exp(+i kx X_c) removes
the scene-centre range and leaves a exp(-i (kx x + ky y)), ky = ku: the samples the
image formation of Eq. (1) sums, on the Stolt coordinates of the geometry module.

Per-pulse position errors: when the platform recorded echo j at u_j + du_j instead of its
nominal position, the same sum taken at the true positions is the exact azimuth transform
(it is no longer a DFT); the scatterer's phase model above then holds unchanged.

Stolt baseline (Sec. II-A; Sec. IV, Baselines): along every azimuth slice the samples,
non-uniform in kx, are interpolated linearly onto the uniform range grid
kx = 2 pi l / fov_x (integer l, the lattice of Algorithm 1), zero outside the slice's
kx extent, and the image is the inverse Fourier sum over that grid,

    I[jx, jy] = sum_n sum_l S_n(l) exp(+i (2 pi l X[jx] / fov_x + ky_n Y[jy])).

Readings: the paper names only the interpolation routine of its numerical environment,
not the method; the reading is 1-D linear interpolation per slice, that environment's
default 1-D method.  Points outside a slice's sample range are zero.  The azimuth sum
is taken at the image's own pixels (the same sum an inverse FFT evaluates when the
pixels coincide with its grid).
"""

import numpy as np

from . import geometry


def azimuth_wavenumbers(n_pulses, n_positions, du):
    """ku_n = (n - N_u/2) * 2 pi / (J du), n = 0..N_u-1."""
    return (np.arange(n_pulses, dtype=np.float64) - n_pulses / 2.0) * (2.0 * np.pi / (n_positions * du))


def range_fft(pulses, ref=None):
    """Range FFT and matched filter of time-domain pulses (Sec. II-A: the data are taken to
    the frequency domain and matched filtered).

    pulses: [J, P] complex baseband samples of each pulse at the rate of the bandwidth (P
    samples), ref: [P] reference spectrum of the matched filter (None: ones, for data that
    are already dechirped).  Returns E[j, p] = ref[p] sum_t pulses[j, t] exp(-2 pi i (p - P/2)
    t / P): the centred frequency bins, p <-> f_p = fc + (p - P/2) bw / P, the fast-time
    samples the front end takes.
    """
    r = np.asarray(pulses, dtype=np.complex128)
    P = r.shape[1]
    m = np.arange(P, dtype=np.float64) - P // 2
    t = np.arange(P, dtype=np.float64)
    E = r @ np.exp(-2j * np.pi * np.outer(t, m) / P)
    if ref is not None:
        E = E * np.asarray(ref, dtype=np.complex128)[None, :]
    return E


def front_end(echoes, k, du, xc, n_pulses, dpos=None):
    """Azimuth transform of raw echoes and reference-function multiply (see module doc).

    echoes: [J, n_freq] complex, k: [n_freq] rad/m, du: position step (m), xc: reference
    range (m), dpos: [J] along-track position errors (m) or None.  With dpos the echo of
    position j was recorded at u_j + dpos[j], and the azimuth sum is taken at those true
    positions (a non-uniform transform; the wavenumbers ku_n stay those of the nominal
    grid).  Returns (s [n_pulses, n_freq] complex128, ku [n_pulses]).
    """
    e = np.asarray(echoes, dtype=np.complex128)
    J = e.shape[0]
    u = (np.arange(J, dtype=np.float64) - J / 2.0) * du
    if dpos is not None:
        u = u + np.asarray(dpos, dtype=np.float64)
    ku = azimuth_wavenumbers(n_pulses, J, du)
    F = np.exp(-1j * np.outer(ku, u))  # [n, j]
    kx, _ = geometry.stolt(k, ku)
    return np.exp(1j * kx * xc) * (F @ e), ku


def stolt_interpolate(s_row, lam_row):
    """Linear interpolation of one slice onto the integers within its sample range.

    s_row: [P] complex samples at increasing lattice coordinates lam_row [P].  Returns
    (l [L] int64, S [L] complex128) for every integer l in [lam_row[0], lam_row[-1]];
    at l with lam_p <= l < lam_{p+1}, S = s_p + (l - lam_p) (s_{p+1} - s_p) /
    (lam_{p+1} - lam_p), and S = s_{P-1} at l = lam_{P-1}.
    """
    lam_row = np.asarray(lam_row, dtype=np.float64)
    s_row = np.asarray(s_row, dtype=np.complex128)
    l = np.arange(int(np.ceil(lam_row[0])), int(np.floor(lam_row[-1])) + 1, dtype=np.int64)
    out = np.empty(l.size, dtype=np.complex128)
    for i, li in enumerate(l):
        p = int(np.searchsorted(lam_row, li, side="right")) - 1  # lam_p <= l < lam_{p+1}
        if p >= lam_row.size - 1:
            out[i] = s_row[-1]
        else:
            t = (li - lam_row[p]) / (lam_row[p + 1] - lam_row[p])
            out[i] = s_row[p] + t * (s_row[p + 1] - s_row[p])
    return l, out


def stolt_image(prob, s, phase=None, dalong=None, cols=None):
    """Stolt baseline image (see module doc) of the samples s [n_pulses, n_freq] of
    `prob`'s geometry, after the per-pulse phasing of the pipeline (phase, along-track
    errors; None for none).  Range-major [mx, my] complex128, or only the range columns
    `cols` [len(cols), my]."""
    kx, ky, lam, X, Y = prob.geometry()
    if cols is not None:
        X = X[np.asarray(cols)]
    s = np.asarray(s, dtype=np.complex128)
    psi = np.zeros(s.shape[0])
    if phase is not None:
        psi = psi + np.asarray(phase, dtype=np.float64)
    if dalong is not None:
        psi = psi + ky * np.asarray(dalong, dtype=np.float64)
    out = np.zeros((X.size, Y.size), dtype=np.complex128)
    for n in range(s.shape[0]):
        l, S = stolt_interpolate(np.exp(1j * psi[n]) * s[n], lam[n])
        T = np.exp(2j * np.pi * np.outer(X, l) / prob.fov_x) @ S  # [jx]
        out += np.outer(T, np.exp(1j * ky[n] * Y))
    return out
