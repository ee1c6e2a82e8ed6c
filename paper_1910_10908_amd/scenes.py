"""Seeded synthetic stripmap-SAR inputs (shared by the tests, the smoke check and the bench).

This module only draws inputs: radar sampling vectors, scene content, phase-history
samples and injected per-pulse errors.  It holds none of the reconstruction's arithmetic
(no weights, no gridding, no transforms); the phase history of a point target is the
forward signal model that the reconstruction inverts.

Acquisition model (Sec. II-A; the workloads stand in for the paper's rail-SAR data,
which are not available):

* fast-time frequencies f_p = fc - B/2 + p B / n_freq, wavenumbers k_p = 2 pi f_p / c;
* aperture positions spaced du = lambda_c / 4; the azimuth wavenumbers are the central
  n_pulses bins of a 2 n_pulses-point azimuth FFT, ku_n = (n - n_pulses/2) * 2 pi / (2 n_pulses du),
  so |ku| <= k_c < 2 k_min and no sample is evanescent;
* a point scatterer of complex reflectivity a at (x, y) (range, azimuth, metres from the
  scene centre) contributes a exp(-i (sqrt(4 k^2 - ku^2) x + ku y)) after matched
  filtering;
* per-pulse phase errors phi and along-track position errors du multiply pulse n by
  exp(i (phi_n + ku_n du_n)).
"""

from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0
SEED_BASE = 20191024


@dataclass(frozen=True)
class Workload:
    name: str
    n_pulses: int
    n_freq: int
    m: int  # image is m x m
    fov: float  # scene extent, m (square)
    n_scatterers: int
    clutter: bool
    snr_db: float = None
    phase_sigma: float = 0.0  # rad
    dalong_sigma: float = 0.0  # m
    fc: float = 10e9
    bw: float = 600e6
    dtype: str = "c64"
    kernel_width: int = 7
    extra: dict = field(default_factory=dict)

    @property
    def n_samples(self):
        return self.n_pulses * self.n_freq


WORKLOADS = {
    # Tiny plain-FFR problem in complex128; the direct NUDFT finishes in seconds.
    "tiny_ffr_c128": Workload("tiny_ffr_c128", 64, 128, 128, 40.0, 5, False, snr_db=30.0,
                              dtype="c128", kernel_width=14),
    # Plain FFR vs tFFR in complex64: 512 x 1024 samples, 1024^2 image.
    "ffr_vs_tffr_c64": Workload("ffr_vs_tffr_c64", 512, 1024, 1024, 400.0, 200, True,
                                kernel_width=7, extra={"config_width": 6}),
    # Precision study: 2048 x 4096 samples, 2048^2 image, FP32 and FP16-stored samples.
    "precision_2k": Workload("precision_2k", 2048, 4096, 2048, 400.0, 1000, True),
    # Differentiation: 1024 x 2048 samples, 1024^2 image, per-pulse phase errors.
    "autofocus_1k": Workload("autofocus_1k", 1024, 2048, 1024, 400.0, 300, False,
                             phase_sigma=0.5),
    # Full swath: 4096 x 8192 samples, 4096^2 image, phase and along-track errors.
    "full_swath_4k": Workload("full_swath_4k", 4096, 8192, 4096, 400.0, 5000, True,
                              phase_sigma=0.5, dalong_sigma=(C_LIGHT / 10e9) / 8.0),
}
WORKLOAD_ORDER = ["tiny_ffr_c128", "ffr_vs_tffr_c64", "precision_2k", "autofocus_1k",
                  "full_swath_4k"]


def radar_sampling(n_pulses, n_freq, fc=10e9, bw=600e6):
    """Fast-time wavenumbers k [n_freq] and azimuth wavenumbers ku [n_pulses] (FP64, host)."""
    f = fc - bw / 2.0 + np.arange(n_freq, dtype=np.float64) * (bw / n_freq)
    k = 2.0 * np.pi * f / C_LIGHT
    du = C_LIGHT / (4.0 * fc)
    dku = 2.0 * np.pi / (2.0 * n_pulses * du)
    ku = (np.arange(n_pulses, dtype=np.float64) - n_pulses / 2.0) * dku
    return k, ku


def rma_positions(n_pulses, fc=10e9):
    """Along-track sampling of the raw echoes behind radar_sampling's ku: J = 2 n_pulses
    positions du = c / (4 fc) apart, so the J-point azimuth transform has the bin width
    2 pi / (J du) of radar_sampling.  Returns (J, du)."""
    return 2 * n_pulses, C_LIGHT / (4.0 * fc)


def raw_echoes(k, n_positions, du, xc, x, y, a, chunk=16, dpos=None):
    """Point-scatterer raw echoes e[j, p] = sum_t a_t exp(-2 i k_p R_t(u_j)) (FP64 numpy),
    R_t(u) = sqrt((xc + x_t)^2 + (y_t - u)^2), u_j = (j - J/2) du (+ dpos[j]: the
    platform's along-track position error at position j, when given)."""
    k = np.asarray(k, dtype=np.float64)
    u = (np.arange(n_positions, dtype=np.float64) - n_positions / 2.0) * du
    if dpos is not None:
        u = u + np.asarray(dpos, dtype=np.float64)
    out = np.zeros((n_positions, k.size), dtype=np.complex128)
    for t0 in range(0, len(x), chunk):
        for t in range(t0, min(t0 + chunk, len(x))):
            R = np.sqrt((xc + x[t]) ** 2 + (y[t] - u) ** 2)
            out += a[t] * np.exp(-2j * np.outer(R, k))
    return out


def rng_for(workload_name, offset=0):
    return np.random.default_rng(SEED_BASE + WORKLOAD_ORDER.index(workload_name) + offset)


def random_samples(n_pulses, n_freq, seed):
    """CN(0, 1) samples, complex128 numpy [n_pulses][n_freq]."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n_pulses, n_freq))
    im = rng.standard_normal((n_pulses, n_freq))
    return (re + 1j * im) / np.sqrt(2.0)


def point_scene(wl, rng):
    """Scatterer positions (uniform over the scene) and amplitudes.

    Tiny workload: a ~ CN(0, 1).  Others: |a| log-normal (sigma 1), uniform phase.
    """
    J = wl.n_scatterers
    x = rng.uniform(-wl.fov / 2, wl.fov / 2, J)
    y = rng.uniform(-wl.fov / 2, wl.fov / 2, J)
    if wl.snr_db is not None:
        a = (rng.standard_normal(J) + 1j * rng.standard_normal(J)) / np.sqrt(2.0)
    else:
        a = np.exp(rng.standard_normal(J)) * np.exp(2j * np.pi * rng.uniform(size=J))
    return x, y, a


def _phase_history_points(k, ku, x, y, a, device, chunk=64):
    import torch

    kt = torch.as_tensor(k, dtype=torch.float64, device=device)
    kut = torch.as_tensor(ku, dtype=torch.float64, device=device)
    kxx = torch.sqrt(4.0 * kt[None, :] ** 2 - kut[:, None] ** 2)  # two-way range wavenumber
    out = torch.zeros(kxx.shape, dtype=torch.complex128, device=device)
    xs = torch.as_tensor(x, dtype=torch.float64, device=device)
    ys = torch.as_tensor(y, dtype=torch.float64, device=device)
    am = torch.as_tensor(a, dtype=torch.complex128, device=device)
    for j0 in range(0, xs.numel(), chunk):
        for j in range(j0, min(j0 + chunk, xs.numel())):
            ph = kxx * xs[j] + kut[:, None] * ys[j]
            out += am[j] * torch.polar(torch.ones_like(ph), -ph)
    return out, kxx, kut


def _phase_history_clutter(kxx, kut, fov, rng, device, sigma2=0.01, spacing=1.0):
    """Speckle clutter CN(0, sigma2) on a regular grid, synthesised row by row.

    V[n, gx] = sum_gy c[gx, gy] exp(-i ku_n y_gy);  s[n, p] += sum_gx V[n, gx] exp(-i kx[n,p] x_gx).
    """
    import torch

    g = int(round(fov / spacing))
    pos = (np.arange(g) + 0.5) * spacing - fov / 2.0
    cl = (rng.standard_normal((g, g)) + 1j * rng.standard_normal((g, g))) * np.sqrt(sigma2 / 2.0)
    ct = torch.as_tensor(cl, dtype=torch.complex128, device=device)
    pt = torch.as_tensor(pos, dtype=torch.float64, device=device)
    Ey = torch.polar(torch.ones(kut.numel(), g, dtype=torch.float64, device=device),
                     -kut[:, None] * pt[None, :])  # [n, gy]
    V = Ey @ ct.T.contiguous()  # [n, gx]
    out = torch.zeros(kxx.shape, dtype=torch.complex128, device=device)
    rows = max(1, (1 << 22) // max(1, kxx.shape[1] * g))
    for n0 in range(0, kxx.shape[0], rows):
        n1 = min(n0 + rows, kxx.shape[0])
        ph = kxx[n0:n1, :, None] * pt[None, None, :]  # [rows, p, gx]
        E = torch.polar(torch.ones_like(ph), -ph)
        out[n0:n1] = torch.matmul(E, V[n0:n1].unsqueeze(-1).contiguous()).squeeze(-1)
    return out


def make_inputs(wl, device="cpu", scene=True):
    """Draw one seeded batch for workload `wl`.

    Returns dict with k, ku (numpy FP64, host), samples (torch complex128 on `device`),
    phase_true and dalong_true (numpy FP64 [n_pulses], zeros when absent).
    With scene=False the samples are CN(0,1) noise of the same shape (parity inputs).
    """
    import torch

    rng = rng_for(wl.name)
    k, ku = radar_sampling(wl.n_pulses, wl.n_freq, wl.fc, wl.bw)
    if scene:
        x, y, a = point_scene(wl, rng)
        s, kxx, kut = _phase_history_points(k, ku, x, y, a, device)
        if wl.clutter:
            s += _phase_history_clutter(kxx, kut, wl.fov, rng, device)
        if wl.snr_db is not None:
            p_sig = float(torch.mean(torch.abs(s) ** 2))
            sig = np.sqrt(p_sig / 10 ** (wl.snr_db / 10.0) / 2.0)
            nz = rng.standard_normal(s.shape) + 1j * rng.standard_normal(s.shape)
            s += torch.as_tensor(nz * sig, dtype=torch.complex128, device=device)
    else:
        s = torch.as_tensor(random_samples(wl.n_pulses, wl.n_freq, SEED_BASE + 1000
                                           + WORKLOAD_ORDER.index(wl.name)),
                            dtype=torch.complex128, device=device)
    phase = rng.normal(0.0, wl.phase_sigma, wl.n_pulses) if wl.phase_sigma else np.zeros(wl.n_pulses)
    dalong = rng.normal(0.0, wl.dalong_sigma, wl.n_pulses) if wl.dalong_sigma else np.zeros(wl.n_pulses)
    if wl.phase_sigma or wl.dalong_sigma:
        rot = torch.polar(torch.ones(wl.n_pulses, dtype=torch.float64, device=device),
                          torch.as_tensor(phase + ku * dalong, dtype=torch.float64, device=device))
        s = s * rot[:, None]
    return {"k": k, "ku": ku, "samples": s, "phase_true": phase, "dalong_true": dalong}
