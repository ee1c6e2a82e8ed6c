"""Oracle image formation (FP64): the weighted 2-D non-uniform DFT and its adjoint.

Test infrastructure only (see the package docstring).

Eq. (1) approximates the image by sum_n alpha_n f_hat(lambda_n) exp(2 pi i lambda_n x).
The windowed NUFFT of Eqs. (3)-(4) and the frame reconstruction of Eq. (8) (with a
diagonal D and the grid sum taken over all integers) reach exactly that weighted sum,
because sum_l w_hat(l - lam) exp(2 pi i l x) = w(x) exp(2 pi i lam x) on the unit
interval; the truncation |l - lam| < q is the approximation.  The oracle therefore
evaluates the weighted sum itself:

    I[jx, jy] = sum_{n,p} c[n,p] exp(+i (kx[n,p] X[jx] + ky[n] Y[jy]))

with no global normalisation (the 1/N of Eq. (1) is absorbed).  Images are stored
range-major: index [jx, jy].
"""

from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _row_chunks(n_rows, workers):
    step = max(1, -(-n_rows // max(1, workers)))
    return [(a, min(a + step, n_rows)) for a in range(0, n_rows, step)]


def _map_rows(fn, n_rows, workers):
    """fn(a, b) on consecutive row ranges, on `workers` threads (NumPy's exponentials and
    products release the GIL); the results in row order."""
    chunks = _row_chunks(n_rows, workers)
    if len(chunks) <= 1:
        return [fn(a, b) for a, b in chunks]
    with ThreadPoolExecutor(len(chunks)) as ex:
        return list(ex.map(lambda ab: fn(*ab), chunks))


def forward_direct(c, kx, ky, X, Y):
    """Direct evaluation of the double sum, one azimuth slice at a time."""
    c = np.asarray(c, dtype=np.complex128)
    out = np.zeros((X.size, Y.size), dtype=np.complex128)
    for n in range(c.shape[0]):
        ex = np.exp(1j * np.outer(X, kx[n]))  # [jx, p]
        ey = np.exp(1j * ky[n] * Y)  # [jy]
        out += np.outer(ex @ c[n], ey)
    return out


def forward_separable(c, kx, ky, X, Y, workers=1):
    """Same sum, factored through the slice structure (ky constant along a row).

    T[n, jx] = sum_p c[n,p] exp(i kx[n,p] X[jx]);  I[jx, jy] = sum_n T[n, jx] exp(i ky[n] Y[jy]).
    With workers > 1 the rows are split into that many ranges whose partial images are
    formed on threads and added.
    """
    c = np.asarray(c, dtype=np.complex128)

    def rows(a, b):
        T = np.empty((b - a, X.size), dtype=np.complex128)
        for n in range(a, b):
            T[n - a] = np.exp(1j * np.outer(X, kx[n])) @ c[n]
        Ey = np.exp(1j * np.outer(ky[a:b], Y))  # [n, jy]
        return T.T @ Ey

    return sum(_map_rows(rows, c.shape[0], workers))


def forward_columns(c, kx, ky, X, Y, cols, workers=1):
    """The separable sum restricted to the range columns `cols` -> [len(cols), len(Y)]."""
    Xs = np.asarray(X)[np.asarray(cols)]
    return forward_separable(c, kx, ky, Xs, Y, workers)


def forward_pixels(c, kx, ky, X, Y, pix):
    """Individual pixels (jx, jy) of the image, each summed over all samples."""
    c = np.asarray(c, dtype=np.complex128)
    out = np.empty(len(pix), dtype=np.complex128)
    for i, (jx, jy) in enumerate(pix):
        out[i] = np.sum(c * np.exp(1j * (kx * X[jx] + ky[:, None] * Y[jy])))
    return out


def adjoint(y, kx, ky, X, Y, workers=1):
    """Adjoint of the forward sum: out[n,p] = sum_{jx,jy} y[jx,jy] exp(-i(kx X + ky Y)).
    Rows are independent; workers > 1 forms row ranges on threads."""
    y = np.asarray(y, dtype=np.complex128)

    def rows(a, b):
        Ey = np.exp(-1j * np.outer(ky[a:b], Y))  # [n, jy]
        Z = Ey @ y.T  # [n, jx]
        out = np.empty((b - a,) + kx.shape[1:], dtype=np.complex128)
        for n in range(a, b):
            out[n - a] = np.exp(-1j * np.outer(kx[n], X)) @ Z[n - a]
        return out

    return np.concatenate(_map_rows(rows, kx.shape[0], workers), axis=0)


def adjoint_samples(y, kx, ky, X, Y, samples):
    """Adjoint at selected samples [(n, p), ...], each summed over all pixels."""
    y = np.asarray(y, dtype=np.complex128)
    out = np.empty(len(samples), dtype=np.complex128)
    for i, (n, p) in enumerate(samples):
        out[i] = np.sum(y * np.exp(-1j * (kx[n, p] * X[:, None] + ky[n] * Y[None, :])))
    return out
