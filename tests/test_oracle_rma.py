"""Pins of the oracle's range-migration front end and Stolt baseline (CPU only).

Each pin rests on something other than the oracle's own formulas: the physics of a
point scatterer (its image peaks at its position), a library FFT, exactness of linear
interpolation on linear data, and the direct Fourier sum of the nudft module.
"""

import numpy as np
import pytest

from oracle import geometry, nudft, pipeline as OP, rma
from paper_1910_10908_amd import scenes


def _small_rma(n_pulses=64, n_freq=64, fc=10e9, bw=600e6):
    k, ku_r = scenes.radar_sampling(n_pulses, n_freq, fc, bw)
    J, du = scenes.rma_positions(n_pulses, fc)
    return k, ku_r, J, du


def test_azimuth_wavenumbers_match_radar_sampling():
    """The front end's J = 2 N_u positions du = c / (4 fc) apart give exactly the azimuth
    wavenumbers the workloads are sampled on."""
    for n_pulses in (64, 512, 4096):
        k, ku_r, J, du = _small_rma(n_pulses, 16)
        np.testing.assert_allclose(rma.azimuth_wavenumbers(n_pulses, J, du), ku_r, rtol=0, atol=1e-12)


def test_front_end_transform_is_the_centred_fft():
    """Without the reference function the front end is the J-point DFT along azimuth with
    its centred bins: s[n] = (-1)^(n - N_u/2) FFT_J(e)[(n - N_u/2) mod J] (library FFT)."""
    k, _, J, du = _small_rma(32, 24)
    rng = np.random.default_rng(3)
    e = rng.standard_normal((J, 24)) + 1j * rng.standard_normal((J, 24))
    s, ku = rma.front_end(e, k, du, 0.0, 32)
    F = np.fft.fft(e, axis=0)
    nn = np.arange(32) - 16
    ref = ((-1.0) ** nn)[:, None] * F[nn % J]
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    # and the reference function is the unimodular exp(+i kx X_c)
    s2, _ = rma.front_end(e, k, du, 37.5, 32)
    kx, _ = geometry.stolt(k, ku)
    np.testing.assert_allclose(s2, np.exp(1j * kx * 37.5) * s, rtol=1e-12, atol=1e-12 * np.abs(s).max())


def _point_target_image(method, conj_reference=False):
    """Raw echoes of one scatterer through the front end, then the image: its peak."""
    n_pulses, n_freq = 64, 64
    k, _, J, du = _small_rma(n_pulses, n_freq)
    xc, xt, yt = 20.0, 0.75, 0.12
    e = scenes.raw_echoes(k, J, du, xc, [xt], [yt], [1.0 + 0.0j])
    s, ku = rma.front_end(e, k, du, xc, n_pulses)
    if conj_reference:  # planted mistake: the reference function with the wrong sign
        kx, _ = geometry.stolt(k, ku)
        s = s * np.exp(-2j * kx * xc)
    mx, my, fov_x, fov_y = 32, 16, 4.0, J * du  # fov_y: one period of the azimuth samples
    prob = OP.Problem(k=k, ku=ku, mx=mx, my=my, fov_x=fov_x, fov_y=fov_y, weighting=OP.WEIGHT_QUAD)
    img = rma.stolt_image(prob, s) if method == "stolt" else OP.image(prob, s)
    jx, jy = np.unravel_index(np.argmax(np.abs(img)), img.shape)
    X = geometry.pixel_coordinates(mx, fov_x)
    Y = geometry.pixel_coordinates(my, fov_y)
    return X[jx], Y[jy], fov_x / mx, fov_y / my, xt, yt


@pytest.mark.parametrize("method", ["stolt", "quadrature"])
def test_front_end_focuses_a_point_scatterer(method):
    """Physics pin of the whole front end: raw echoes of a scatterer at (0.75 m, 0.12 m)
    off the 20 m reference range, transformed and matched-filtered, form an image (Stolt
    baseline, or the trapezoid-weighted sum of Eq. (1)) that peaks within one pixel of
    the scatterer.  A reference function of the wrong sign does not."""
    x, y, px, py, xt, yt = _point_target_image(method)
    assert abs(x - xt) <= px and abs(y - yt) <= py, (x, y)
    x, y, px, py, xt, yt = _point_target_image(method, conj_reference=True)
    assert not (abs(x - xt) <= px and abs(y - yt) <= py)


def test_range_fft_is_the_centred_library_fft():
    """The range FFT is numpy's forward FFT of each pulse read at the centred bins
    (p - P/2) mod P, times the reference spectrum."""
    rng = np.random.default_rng(31)
    r = rng.standard_normal((5, 64)) + 1j * rng.standard_normal((5, 64))
    ref = np.exp(1j * rng.uniform(0, 2 * np.pi, 64))
    E = rma.range_fft(r, ref)
    F = np.fft.fft(r, axis=1)
    m = np.arange(64) - 32
    np.testing.assert_allclose(E, F[:, m % 64] * ref, rtol=0, atol=1e-10 * np.abs(F).max())


def test_range_fft_delay_and_matched_filter():
    """Closed forms: a pulse delayed by t0 samples becomes exp(-2 pi i (p - P/2) t0 / P); a
    phase-coded pulse whose spectrum is the code C times X comes out as X through the
    reference conj(C) (|C| = 1), the matched filter."""
    P, t0 = 128, 37
    r = np.zeros((1, P), complex)
    r[0, t0] = 1.0
    m = np.arange(P) - P // 2
    np.testing.assert_allclose(rma.range_fft(r)[0], np.exp(-2j * np.pi * m * t0 / P), rtol=0, atol=1e-12)
    rng = np.random.default_rng(32)
    X = rng.standard_normal((3, P)) + 1j * rng.standard_normal((3, P))
    C = np.exp(1j * np.pi * (m / P) ** 2 * P / 4)  # a linear-FM (chirp) code, unit modulus
    spec = C * X  # the coded pulse's centred spectrum
    pulses = np.fft.ifft(np.roll(spec, -P // 2, axis=1), axis=1)  # back to time samples
    np.testing.assert_allclose(rma.range_fft(pulses, np.conj(C)), X, rtol=0, atol=1e-10 * np.abs(X).max())


def test_front_end_position_errors_tone():
    """Per-pulse position errors: an azimuth tone exp(+i ku_m u) recorded at the true
    positions u_j + d_j transforms to exactly J at bin m (every term of the sum is 1) when
    the front end is given d; taken at the nominal positions instead, bin m is off by the
    unmodelled phases."""
    n_pulses, n_freq = 32, 4
    k, _, J, du = _small_rma(n_pulses, n_freq)
    rng = np.random.default_rng(21)
    d = rng.uniform(-0.4, 0.4, J) * du
    ku = rma.azimuth_wavenumbers(n_pulses, J, du)
    m = 30  # near the band edge, where ku d is largest
    u = (np.arange(J) - J / 2.0) * du + d
    e = np.repeat(np.exp(1j * ku[m] * u)[:, None], n_freq, axis=1)
    s, _ = rma.front_end(e, k, du, 0.0, n_pulses, dpos=d)
    np.testing.assert_allclose(s[m], J, rtol=0, atol=1e-9 * J)
    s0, _ = rma.front_end(e, k, du, 0.0, n_pulses)
    assert np.abs(s0[m] - J).min() > 0.02 * J


def test_front_end_uniform_position_shift():
    """A uniform error d at every position multiplies bin n by exp(-i ku_n d): the sign
    and the scale with which the errors enter the azimuth phase."""
    k, _, J, du = _small_rma(32, 12)
    rng = np.random.default_rng(22)
    e = rng.standard_normal((J, 12)) + 1j * rng.standard_normal((J, 12))
    d = 0.37 * du
    s0, ku = rma.front_end(e, k, du, 5.0, 32)
    s1, _ = rma.front_end(e, k, du, 5.0, 32, dpos=np.full(J, d))
    np.testing.assert_allclose(s1, np.exp(-1j * ku * d)[:, None] * s0, rtol=0, atol=1e-10 * np.abs(s0).max())


def test_stolt_interpolation_is_exact_on_linear_data():
    """Linear interpolation reproduces a linear function of lam exactly, and returns the
    samples themselves where they sit on integers."""
    rng = np.random.default_rng(5)
    lam = np.cumsum(rng.uniform(0.3, 1.9, 200)) + 10.25
    lam[37] = np.ceil(lam[36] + 1e-9)  # one sample exactly on an integer
    assert lam[36] < lam[37] < lam[38]
    alpha, beta = 0.7 - 0.2j, 0.013 + 0.031j
    l, S = rma.stolt_interpolate(alpha + beta * lam, lam)
    assert l[0] == int(np.ceil(lam[0])) and l[-1] == int(np.floor(lam[-1]))
    np.testing.assert_allclose(S, alpha + beta * l, rtol=0, atol=1e-12)
    on = np.nonzero(lam == np.round(lam))[0]
    assert on.size >= 1
    s = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    l, S = rma.stolt_interpolate(s, lam)
    for p in on:
        assert S[np.searchsorted(l, int(lam[p]))] == s[p]


def test_stolt_interpolation_is_not_nearest_neighbour():
    """A planted nearest-neighbour interpolation fails the linear-data pin (the pin has
    power against the plausible mistake)."""
    lam = np.array([0.2, 1.7, 2.4, 3.9])
    s = 2.0 * lam
    l, S = rma.stolt_interpolate(s, lam)
    nn = s[np.abs(lam[None, :] - l[:, None]).argmin(axis=1)]
    assert np.allclose(S, 2.0 * l) and not np.allclose(nn, 2.0 * l)


def test_stolt_image_of_lattice_samples_is_the_direct_sum():
    """Samples that sit on consecutive integers of the lattice need no interpolation:
    the Stolt image is then the plain sum of Eq. (1) with unit weights, evaluated by
    the nudft module's own direct double sum."""
    n_pulses, n_freq, fov = 6, 40, 30.0
    rng = np.random.default_rng(7)
    l0 = rng.integers(300, 320, n_pulses)
    lam = (l0[:, None] + np.arange(n_freq)[None, :]).astype(np.float64)
    # kx -> lam rounds in the last place; the end samples sit 1e-9 outside their integers
    # so that both ends stay inside the slice's range (their weights move by 1e-9)
    lam[:, 0] -= 1e-9
    lam[:, -1] += 1e-9
    kx = 2.0 * np.pi * lam / fov
    ky = np.linspace(-3.0, 2.5, n_pulses)
    prob = OP.Problem(k=np.linspace(1, 2, n_freq), ku=ky, mx=16, my=12, fov_x=fov, fov_y=fov,
                      kx_explicit=kx, ky_explicit=ky)
    s = rng.standard_normal((n_pulses, n_freq)) + 1j * rng.standard_normal((n_pulses, n_freq))
    got = rma.stolt_image(prob, s)
    X = geometry.pixel_coordinates(16, fov)
    Y = geometry.pixel_coordinates(12, fov)
    ref = nudft.forward_direct(s, 2.0 * np.pi * np.round(lam) / fov, ky, X, Y)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * np.abs(ref).max())
