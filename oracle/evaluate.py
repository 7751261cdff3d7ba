"""FP64 CPU oracle of the evaluation step after a reconstruction.

TEST INFRASTRUCTURE ONLY (see ``oracle/shlr_oracle.py``): only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP path.

What the paper fixes and what it leaves open:

* SSOS (Results, opening paragraph): multi-coil images are combined by the square root of the sum
  of squares; the coil images are the centred unitary inverse 2D DFT of each coil's k-space.
* RLNE (Eq. S10): ||x - x_hat||_2 / ||x||_2 on the vectorised SSOS images (x the fully sampled
  reference).  For T2 maps the same ratio is taken over the map (pixels outside the ROI are 0 in
  both, so they add nothing).
* MSSIM (Eq. S11): the mean over R local windows of
  (2 mu_a mu_b + C1)(2 sigma_ab + C2) / ((mu_a^2 + mu_b^2 + C1)(sigma_a^2 + sigma_b^2 + C2)).
  The paper cites the SSIM paper for it but states neither the window nor C1, C2.  Reading taken
  (that paper's defaults): an 11 x 11 circular Gaussian window with sigma 1.5 normalised to unit
  sum, weighted local means, variances and covariance, every window position that fits inside the
  image (R = (M - 10)(N - 10)), C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L the dynamic range, taken
  as the maximum of the reference image unless given.
* T2 fit (Section IV-B, the T2 mapping experiment): a standard nonlinear least-squares fit per
  pixel inside a region of interest, with T2 values outside a reasonable range excluded.
  Readings taken: the model S(TE) = rho exp(-TE / T2) fitted to the SSOS magnitudes of the
  echoes; the ROI is every pixel whose first-echo SSOS value is at least roi_frac times that
  image's maximum; the fit starts from the log-linear least-squares line and is solved by
  MINPACK's Levenberg-Marquardt (scipy's least_squares, method 'lm'); a T2 outside
  [t2_min, t2_max] (or a failed fit) is excluded; excluded and non-ROI pixels hold 0.
"""

from __future__ import annotations

import numpy as np


def ifft2c(k):
    """Centred unitary inverse 2D DFT over the last two axes."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(k, axes=ax), axes=ax, norm="ortho"), axes=ax)


def ssos(k):
    """SSOS image of multi-coil k-space (..., J, M, N) -> (..., M, N)."""
    x = ifft2c(np.asarray(k, dtype=np.complex128))
    return np.sqrt(np.sum(np.abs(x) ** 2, axis=-3))


def rlne(x, x_hat):
    """Eq. S10 on vectorised images."""
    x = np.asarray(x, dtype=np.float64).ravel()
    x_hat = np.asarray(x_hat, dtype=np.float64).ravel()
    return float(np.linalg.norm(x - x_hat) / np.linalg.norm(x))


def gaussian_window(size: int = 11, sigma: float = 1.5):
    """Circular Gaussian window of unit sum."""
    h = size // 2
    t = np.arange(-h, h + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2.0 * sigma ** 2))
    return g / g.sum()


def mssim(a, b, L=None, size: int = 11, sigma: float = 1.5, k1: float = 0.01, k2: float = 0.03):
    """Eq. S11: the mean SSIM over every window position inside the image."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if L is None:
        L = float(a.max())
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    w = gaussian_window(size, sigma)
    wa = np.lib.stride_tricks.sliding_window_view(a, (size, size))      # (M-10, N-10, 11, 11)
    wb = np.lib.stride_tricks.sliding_window_view(b, (size, size))
    mu_a = np.einsum("ijkl,kl->ij", wa, w)
    mu_b = np.einsum("ijkl,kl->ij", wb, w)
    var_a = np.einsum("ijkl,kl->ij", (wa - mu_a[..., None, None]) ** 2, w)
    var_b = np.einsum("ijkl,kl->ij", (wb - mu_b[..., None, None]) ** 2, w)
    cov = np.einsum("ijkl,kl->ij", (wa - mu_a[..., None, None]) * (wb - mu_b[..., None, None]), w)
    ssim = ((2 * mu_a * mu_b + c1) * (2 * cov + c2)) / ((mu_a ** 2 + mu_b ** 2 + c1) * (var_a + var_b + c2))
    return float(ssim.mean())


def t2_fit(img, te, roi_frac=0.1, t2_min=5.0, t2_max=500.0, pixels=None):
    """Pixel-wise T2 of echo images img (L, M, N) at echo times te (L,), ms.

    Returns (t2, rho, roi): t2 and rho maps (0 outside the ROI and where excluded) and the mask of
    kept pixels.  pixels: optional list of flat indices to fit (others are left 0), for sampled
    checks of large maps.
    """
    from scipy.optimize import least_squares

    img = np.asarray(img, dtype=np.float64)
    te = np.asarray(te, dtype=np.float64)
    Lh = img.shape[0]
    flat = img.reshape(Lh, -1)
    thr = roi_frac * flat[0].max()
    t2 = np.zeros(flat.shape[1])
    rho = np.zeros(flat.shape[1])
    keep = np.zeros(flat.shape[1], dtype=bool)
    todo = range(flat.shape[1]) if pixels is None else pixels
    for p in todo:
        s = flat[:, p]
        if not s[0] >= thr:
            continue
        pos = s > 0
        if pos.sum() < 2:
            continue
        # log-linear start: ln s = ln rho - r TE
        A = np.stack([np.ones(pos.sum()), -te[pos]], axis=1)
        coef = np.linalg.lstsq(A, np.log(s[pos]), rcond=None)[0]
        x0 = np.array([np.exp(coef[0]), max(coef[1], 1e-6)])

        def res(x, s=s):
            return x[0] * np.exp(-x[1] * te) - s

        def jac(x):
            e = np.exp(-x[1] * te)
            return np.stack([e, -x[0] * te * e], axis=1)

        sol = least_squares(res, x0, jac=jac, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
        r = sol.x[1]
        if not (np.all(np.isfinite(sol.x)) and r > 0):
            continue
        T = 1.0 / r
        if t2_min <= T <= t2_max:
            t2[p], rho[p], keep[p] = T, sol.x[0], True
    shp = img.shape[1:]
    return t2.reshape(shp), rho.reshape(shp), keep.reshape(shp)
