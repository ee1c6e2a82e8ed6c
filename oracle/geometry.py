"""Oracle geometry: Stolt map, weight-lattice and pixel coordinates (FP64).

Test infrastructure only (see the package docstring).
"""

import numpy as np


class GeometryError(ValueError):
    pass


def stolt(k, ku):
    """Stolt map of the range-migration spectrum (Sec. II-A).

    After matched filtering the data sit on a grid that is uniform in the azimuth
    wavenumber ku and in the fast-time wavenumber k; the Stolt change of variables
    puts sample (n, p) at range wavenumber kx = sqrt(4 k_p^2 - ku_n^2) and azimuth
    wavenumber ky = ku_n.  Rows n keep a constant ky (azimuth slices of Algorithm 1),
    and kx is non-uniform along each row.

    Returns kx with shape [n_pulses, n_freq] and ky with shape [n_pulses].
    Raises GeometryError for evanescent samples (4 k^2 <= ku^2) and when k is not
    strictly increasing.
    """
    k = np.asarray(k, dtype=np.float64)
    ku = np.asarray(ku, dtype=np.float64)
    if k.ndim != 1 or ku.ndim != 1:
        raise GeometryError("k and ku must be 1-D")
    if k.size > 1 and not np.all(np.diff(k) > 0):
        raise GeometryError("k must be strictly increasing")
    arg = 4.0 * k[None, :] ** 2 - ku[:, None] ** 2
    if np.any(arg <= 0):
        raise GeometryError("evanescent sample: 4 k^2 <= ku^2")
    return np.sqrt(arg), ku.copy()


def lattice_coordinate(kx, fov):
    """Range frequency in cycles per image field of view.

    The frame of Sec. III lives on a unit image interval; with the range field of view
    of length `fov` mapped onto it, exp(i kx X) = exp(2 pi i lam (X / fov)), so the
    sample sits at lam = kx * fov / (2 pi) on the frequency axis whose integer points
    are the uniform grid {l_m} of Eq. (3) and Algorithm 1.  The value is not wrapped.
    """
    return np.asarray(kx, dtype=np.float64) * fov / (2.0 * np.pi)


def pixel_coordinates(m, fov):
    """Centred pixel positions X_j = (j - m/2) * fov / m, j = 0..m-1.

    Algorithm 1 writes the image abscissae as (1/M)[1..M]; here the scene centre sits
    at pixel m/2 so the image is centred on the scene (a translation of the paper's
    convention, which only changes a unimodular phase per sample).
    """
    j = np.arange(m, dtype=np.float64)
    return (j - m / 2.0) * (fov / m)
