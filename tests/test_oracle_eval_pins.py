"""Pins of the evaluation oracle (oracle/evaluate.py): SSOS, RLNE (Eq. S10), MSSIM (Eq. S11) and the
pixel-wise T2 fit, against closed forms, special cases, brute force and an independent fit route."""

import numpy as np
import pytest

from oracle import brute
from oracle import evaluate as E
from paper_2107_11650_amd import inputs


def test_ssos_of_coil_images_is_magnitude_times_coil_energy():
    # K_j = F2(s_j x): the SSOS image is |x| sqrt(sum_j |s_j|^2), with F2 built from explicit DFT matrices
    J, M, N = 3, 9, 8
    x = inputs.random_complex((M, N), seed=1)
    s = inputs.random_complex((J, M, N), seed=2)
    FM, FN = brute.dft_matrix(M), brute.dft_matrix(N)
    K = np.stack([FM @ (s[j] * x) @ FN.T for j in range(J)])
    want = np.abs(x) * np.sqrt(np.sum(np.abs(s) ** 2, axis=0))
    assert np.abs(E.ssos(K) - want).max() < 1e-13 * want.max()


def test_rlne_special_cases():
    x = np.abs(inputs.random_complex((16, 16), seed=3))
    assert E.rlne(x, x) == 0.0
    assert abs(E.rlne(x, 1.25 * x) - 0.25) < 1e-15
    assert abs(E.rlne(np.array([3.0, 4.0]), np.array([3.0, 0.0])) - 0.8) < 1e-15


def test_gaussian_window():
    w = E.gaussian_window(11, 1.5)
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1]) and w.argmax() == 60
    # separable (rank one) with the Gaussian fall-off of sigma = 1.5 between taps
    assert np.linalg.svd(w, compute_uv=False)[1] < 1e-15
    assert abs(w[5, 6] / w[5, 5] - np.exp(-1.0 / 4.5)) < 1e-15
    assert abs(w[7, 8] / w[5, 5] - np.exp(-13.0 / 4.5)) < 1e-15


def _mssim_loops(a, b, L, size=11, sigma=1.5):
    """Eq. S11 with explicit loops over windows and window pixels."""
    h = size // 2
    g = [[np.exp(-((i - h) ** 2 + (j - h) ** 2) / (2 * sigma ** 2)) for j in range(size)] for i in range(size)]
    tot = sum(sum(r) for r in g)
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    vals = []
    for i0 in range(a.shape[0] - size + 1):
        for j0 in range(a.shape[1] - size + 1):
            ma = mb = 0.0
            for i in range(size):
                for j in range(size):
                    ma += g[i][j] / tot * a[i0 + i, j0 + j]
                    mb += g[i][j] / tot * b[i0 + i, j0 + j]
            va = vb = cab = 0.0
            for i in range(size):
                for j in range(size):
                    da, db = a[i0 + i, j0 + j] - ma, b[i0 + i, j0 + j] - mb
                    va += g[i][j] / tot * da * da
                    vb += g[i][j] / tot * db * db
                    cab += g[i][j] / tot * da * db
            vals.append((2 * ma * mb + c1) * (2 * cab + c2) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    return sum(vals) / len(vals)


def test_mssim_against_window_loops_and_limits():
    a = np.abs(inputs.random_complex((15, 14), seed=4))
    b = a + 0.2 * np.abs(inputs.random_complex((15, 14), seed=5))
    L = float(a.max())
    assert abs(E.mssim(a, b) - _mssim_loops(a, b, L)) < 1e-14
    assert abs(E.mssim(a, a) - 1.0) < 1e-15
    # constant images: only the luminance term differs from 1
    al, be, Lc = 2.0, 3.0, 5.0
    c1 = (0.01 * Lc) ** 2
    want = (2 * al * be + c1) / (al * al + be * be + c1)
    assert abs(E.mssim(np.full((12, 12), al), np.full((12, 12), be), L=Lc) - want) < 1e-15
    # invariant to a common scale of both images and the dynamic range
    assert abs(E.mssim(7.0 * a, 7.0 * b, L=7.0 * L) - E.mssim(a, b, L=L)) < 1e-13


def _vp_fit(s, te):
    """Variable projection: for a rate r the best rho is <s, e> / <e, e>; minimise the reduced cost
    over r by a dense scan and a bounded refinement (a route independent of the LM solver)."""
    from scipy.optimize import minimize_scalar

    def cost(r):
        e = np.exp(-r * te)
        return float(np.sum(s * s) - np.dot(s, e) ** 2 / np.dot(e, e))
    grid = np.linspace(1e-4, 0.5, 20001)
    i = int(np.argmin([cost(r) for r in grid]))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    r = minimize_scalar(cost, bounds=(lo, hi), method="bounded", options={"xatol": 1e-15}).x
    e = np.exp(-r * te)
    return 1.0 / r, np.dot(s, e) / np.dot(e, e)


def test_t2_fit_exact_noisy_roi_and_range():
    te = 10.0 * (np.arange(8) + 1)
    t2_true = np.array([[40.0, 80.0, 120.0], [60.0, 2000.0, 90.0]])      # 2000 ms: outside the range
    rho = np.array([[1.0, 0.8, 0.5], [0.03, 0.9, 0.7]])                  # 0.03: below the ROI threshold
    img = rho[None] * np.exp(-te[:, None, None] / t2_true[None])
    t2, r, keep = E.t2_fit(img, te, roi_frac=0.1, t2_min=5.0, t2_max=500.0)
    assert keep.tolist() == [[True, True, True], [False, False, True]]
    sel = keep
    assert np.abs(t2[sel] / t2_true[sel] - 1).max() < 1e-10
    assert np.abs(r[sel] / rho[sel] - 1).max() < 1e-10
    assert t2[~keep].tolist() == [0.0, 0.0]
    # noisy curves: the LM minimiser equals the variable-projection minimiser
    rng = np.random.default_rng(6)
    for T in (35.0, 70.0, 140.0):
        s = np.exp(-te / T) + 0.01 * rng.standard_normal(te.size)
        t2n, rn, kn = E.t2_fit(s[:, None, None], te)
        tv, rv = _vp_fit(s, te)
        assert kn[0, 0] and abs(t2n[0, 0] / tv - 1) < 1e-7 and abs(rn[0, 0] / rv - 1) < 1e-7
