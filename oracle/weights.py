"""Oracle sample weights (FP64): tFFR, plain FFR and trapezoid quadrature.

Test infrastructure only (see the package docstring).

Readings taken where the paper's matrices do not conform or are under-specified:

* The product that is inverted is the sample-indexed one, G = Psi W (P x P per azimuth
  slice), so that W D f_hat in Algorithm 1 conforms and "diagonal" / "band" refer to
  the sample index within the slice.  The inner-product order is the one under which
  the untruncated product is the frame Gram matrix (unit diagonal).
* W and Psi are both truncated to grid points m with |m - lam| < q (the bound of
  Eq. (4)); q is not given for the frame methods, the default is q = 3.
* The weight lattice is the image's own DFT lattice: the integers in cycles per field of
  view, infinite and periodic.
* tFFR keeps only the diagonal of G (Sec. III-C isolates it before inverting):
  D = diag(pinv(diag(G))), i.e. 1/g elementwise with 1/0 -> 0, then R_tau.
* R_tau(x) = x if x >= tau else 0 (Sec. III-B), inclusive, compared on |x| (x is real
  and positive here).  Mode 0 thresholds the entries of the pseudo-inverse as written;
  mode 1 thresholds the correlation g itself (Sec. III-B's interpretation of R_tau as
  keeping the most strongly correlated frame coefficients).
* Plain FFR: D = B_r(pinv(G)) with r = 2 (Eq. (8) and Sec. IV, Baselines); B_r keeps
  entries with |p - p'| <= r.
* Quadrature: trapezoid rule per azimuth slice in lam (Sec. II-B and Sec. IV), half
  intervals at both ends; azimuth is uniform so it carries no factor.
"""

import numpy as np

from .window import r_psi, r_w

THRESH_LITERAL = 0  # keep iff |1/g| >= tau
THRESH_CORRELATION = 1  # keep iff g >= tau


def grid_points(lam, q):
    """Integers m with |m - lam| < q, as an array [..., K] plus a validity mask.

    This is the truncation of Eq. (4): each grid point l_m takes only the samples within a
    chosen distance q of it.
    """
    lam = np.asarray(lam, dtype=np.float64)
    kmax = int(np.ceil(q)) + 1
    base = np.floor(lam)[..., None]
    offs = np.arange(-kmax, kmax + 1, dtype=np.float64)
    m = base + offs
    mask = np.abs(m - lam[..., None]) < q
    return m, mask


def frame_diagonal(lam, a=0.01, q=3.0):
    """g = (Psi W)_{pp} = sum_{|m - lam| < q} R_Psi(m - lam) R_W(m - lam).

    The diagonal of the (truncated) frame product for every sample (Sec. III-C, end:
    only the diagonal of W Psi is needed for stripmap tFFR).
    """
    m, mask = grid_points(lam, q)
    d = m - np.asarray(lam, dtype=np.float64)[..., None]
    terms = r_psi(d, a) * r_w(d, a)
    return np.sum(np.where(mask, terms, 0.0), axis=-1)


def threshold_diagonal(g, tau=0.97, mode=THRESH_LITERAL):
    """R_tau applied to the pseudo-inverse of a diagonal with entries g (Sec. III-B).

    pinv(diag(g)) = diag(1/g) with 1/0 -> 0.  R_tau keeps an entry x iff x >= tau
    (inclusive); on real entries of either sign it is read as |x| >= tau.  Mode 0 applies
    it to the entries 1/g of the pseudo-inverse; mode 1 to the correlation g itself
    (keep iff g >= tau, so a negative g is never kept).  Returns (d, kept).
    """
    g = np.asarray(g, dtype=np.float64)
    with np.errstate(divide="ignore"):
        inv = np.where(g != 0.0, 1.0 / np.where(g != 0.0, g, 1.0), 0.0)
    if mode == THRESH_LITERAL:
        kept = np.abs(inv) >= tau
    elif mode == THRESH_CORRELATION:
        kept = g >= tau
    else:
        raise ValueError("unknown threshold mode")
    return np.where(kept, inv, 0.0), kept


def tffr_weights(lam, a=0.01, q=3.0, tau=0.97, mode=THRESH_LITERAL):
    """tFFR weights D = R_tau(pinv(diag(Psi W))) for every sample (Sec. III-B/III-C).

    Returns (d, kept) with d the weight (0 where thresholded) and kept the boolean mask
    of surviving samples; kept.sum() is the count c of Sec. III-C.
    """
    return threshold_diagonal(frame_diagonal(lam, a, q), tau, mode)


def quad_weights(lam):
    """Trapezoid quadrature weights along each azimuth slice (Sec. II-B, Sec. IV).

    alpha_p = (lam_{p+1} - lam_{p-1}) / 2 inside, (lam_1 - lam_0)/2 and
    (lam_{P-1} - lam_{P-2})/2 at the ends; a single sample gets weight 1.
    """
    lam = np.atleast_2d(np.asarray(lam, dtype=np.float64))
    n_rows, n_p = lam.shape
    out = np.empty_like(lam)
    if n_p == 1:
        out[:] = 1.0
        return out
    for p in range(n_p):
        lo = lam[:, max(p - 1, 0)]
        hi = lam[:, min(p + 1, n_p - 1)]
        out[:, p] = (hi - lo) / 2.0
    return out


def frame_product_row(lam_row, a=0.01, q=3.0):
    """Truncated frame product G~ (P x P) for one azimuth slice.

    G~_{pp'} = sum over integers m with |m - lam_p| < q and |m - lam_p'| < q of
    R_Psi(m - lam_p) R_W(m - lam_p')  (Psi truncated around lam_p, W around lam_p').
    The samples of a slice are sorted by lam (kx rises along the slice); a grid point
    within q of both samples needs |lam_p - lam_p'| < 2q, so each row sample p only meets
    the column samples in that window, found by binary search.
    """
    lam = np.asarray(lam_row, dtype=np.float64)
    n_p = lam.size
    if n_p > 1 and not np.all(np.diff(lam) > 0):
        raise ValueError("frame_product_row: lam must increase along the slice")
    m, mask = grid_points(lam, q)  # [p, j]: the grid points Psi reaches from sample p
    lo = np.searchsorted(lam, lam - 2.0 * q, side="right")  # first p' with lam_p' > lam_p - 2q
    hi = np.searchsorted(lam, lam + 2.0 * q, side="left")  # one past the last p' < lam_p + 2q
    width = int(np.max(hi - lo))
    idx = lo[:, None] + np.arange(width)[None, :]  # [p, o]: candidate column samples
    valid = idx < hi[:, None]
    idx = np.minimum(idx, n_p - 1)
    d_w = m[:, None, :] - lam[idx][:, :, None]  # [p, o, j]: offsets of p's points from p'
    ok = mask[:, None, :] & valid[:, :, None] & (np.abs(d_w) < q)  # ... which W reaches from p'
    terms = np.where(ok, r_psi(m - lam[:, None], a)[:, None, :] * r_w(d_w, a), 0.0)
    G = np.zeros((n_p, n_p))
    rows = np.broadcast_to(np.arange(n_p)[:, None], idx.shape)
    G[rows[valid], idx[valid]] = np.sum(terms, axis=2)[valid]
    return G


def pinv(G, band=None):
    """Moore-Penrose pseudo-inverse of a square real matrix.

    A nonsingular G's pseudo-inverse is its inverse.  It is formed from an LU
    factorisation with partial pivoting (LAPACK's banded one when G vanishes beyond `band`
    diagonals, the frame products being banded) and used when the 1-norm condition number
    ||G|| ||G^-1|| stays below 1e12 (the products of slices whose samples are more than a
    lattice unit apart have 2-3).  Otherwise the SVD pseudo-inverse, keeping the singular
    values above max(M, N) eps sigma_max (the usual numerical-rank cut-off): a product of
    rank L < P computed in FP64 carries P - L singular values of rounding size (~1e-15
    sigma_max), which the exact pseudo-inverse does not have and which numpy's fixed
    1e-15 default would invert.
    """
    from scipy.linalg import lapack

    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    Z = None
    if band is not None and 0 <= band < n - 1:
        kl = ku = int(band)
        ab = np.zeros((2 * kl + ku + 1, n))
        for d in range(-kl, ku + 1):  # LAPACK band storage: ab[kl + ku + i - j, j] = G[i, j]
            j = np.arange(max(0, d), min(n, n + d))
            ab[kl + ku - d, j] = G[j - d, j]
        lu, ipiv, info = lapack.dgbtrf(ab, kl, ku)
        if info == 0:
            Z, info = lapack.dgbtrs(lu, kl, ku, np.eye(n), ipiv)
            Z = Z if info == 0 else None
    else:
        lu, ipiv, info = lapack.dgetrf(G)
        if info == 0:
            Z, info = lapack.dgetri(lu, ipiv)
            Z = Z if info == 0 else None
    if Z is not None and np.all(np.isfinite(Z)) and np.linalg.norm(G, 1) * np.linalg.norm(Z, 1) < 1e12:
        return Z
    return np.linalg.pinv(G, rtol=max(G.shape) * np.finfo(np.float64).eps)


def ffr_weights_row(lam_row, a=0.01, q=3.0, r=2):
    """Plain FFR weights for one slice: D = B_r(pinv(G~)) (Eq. (8))."""
    G = frame_product_row(lam_row, a, q)
    nz = np.nonzero(G)
    band = int(np.max(np.abs(nz[0] - nz[1]))) if nz[0].size else 0
    Z = pinv(G, band)
    n_p = np.asarray(lam_row).size
    idx = np.arange(n_p)
    keep = np.abs(idx[:, None] - idx[None, :]) <= r
    return np.where(keep, Z, 0.0)


def ffr_weights(lam, a=0.01, q=3.0, r=2, workers=1):
    """Plain FFR banded weights for every slice, stored as [n_pulses][n_freq][2r+1].

    Entry [n, p, r + o] is D^{(n)}_{p, p+o} for o in [-r, r] (0 outside the row).
    Slices are independent; workers > 1 solves them on threads.
    """
    lam = np.atleast_2d(np.asarray(lam, dtype=np.float64))
    n_rows, n_p = lam.shape
    out = np.zeros((n_rows, n_p, 2 * r + 1))

    def one(n):
        D = ffr_weights_row(lam[n], a, q, r)
        for o in range(-r, r + 1):  # diagonal o: D[p, p + o]
            if o >= 0:
                out[n, : max(n_p - o, 0), r + o] = np.diagonal(D, o)
            else:
                out[n, -o:, r + o] = np.diagonal(D, o)

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor

        from threadpoolctl import threadpool_limits

        # one BLAS thread per worker: the slices are the parallelism
        with threadpool_limits(limits=1), ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, range(n_rows)))
    else:
        for n in range(n_rows):
            one(n)
    return out


def band_to_dense(band_row):
    """[P][2r+1] band storage of one slice -> dense P x P matrix."""
    n_p, width = band_row.shape
    r = (width - 1) // 2
    D = np.zeros((n_p, n_p))
    for p in range(n_p):
        for o in range(-r, r + 1):
            if 0 <= p + o < n_p:
                D[p, p + o] = band_row[p, r + o]
    return D
