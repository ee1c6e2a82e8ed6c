"""FP64 CPU oracle for thresholded non-uniform Fourier frame reconstruction (tFFR).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct NumPy
implementation of what the GPU path computes.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does, and the two share no code.

What it computes (McKay, Gelb, Jayasuriya, Monga, "Thresholded Non-Uniform Fourier
Frame-Based Reconstruction for Stripmap SAR"):

* geometry   -- the Stolt map of Sec. II-A (range non-uniform, azimuth uniform) and the
                lattice / pixel coordinates of Algorithm 1.
* window     -- the finite-interval transforms of the window w(x) = exp(-a|x-1/2|)
                (Sec. IV, Baselines) and of 1/w that make up W and Psi (Eqs. (5)-(8)).
* weights    -- tFFR (Sec. III-B and III-C: the diagonal of the frame product, inverted
                and thresholded by R_tau), plain FFR (Eq. (8): band B_r of the
                pseudo-inverse) and trapezoid quadrature (Sec. II-B).
* nudft      -- the weighted discrete inverse Fourier sum of Eq. (1) evaluated directly
                (the exact result the windowed NUFFT of Eqs. (3)-(4) approximates), and
                its adjoint.
* pipeline   -- sample phasing by per-pulse phase / along-track errors, weighting,
                imaging, and the gradients of an image loss through the adjoint.
* entropy    -- image entropy loss and its gradient.
* literal    -- the range gridding of Algorithm 1 / Eq. (8) taken literally: the window's
                own truncated transform on the image lattice, inverse DFT, division by w.
* rma        -- the range-migration front end (azimuth transform of raw echoes and the
                reference-function multiply, Sec. II-A) and the Stolt-interpolation
                baseline image (Sec. II-A; Sec. IV, Baselines).

Where the paper is ambiguous or garbled, the reading taken is stated in the docstring of
the function that takes it.
"""

from . import geometry, window, weights, nudft, pipeline, entropy, literal, rma  # noqa: F401
