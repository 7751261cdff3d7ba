"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's in-vivo data (4- and 8-coil 256x256 brains, Section IV-A; a
12-coil 192x192 T2 series with 15 echoes, Section IV-B) are not available, so
every test and benchmark draws its inputs from here instead.  This module
holds no arithmetic of the reconstruction method: it only synthesises images,
coil maps, k-space and sampling masks, and it is the one module that both the
CPU oracle's tests and the HIP path's tests use.

Recipe (stated once, used everywhere):

* image: an outer ellipse (semi-axes 0.9, 0.7, intensity 1) plus ten random
  ellipses (centres U[-0.6, 0.6]^2, semi-axes U[0.05, 0.5], angles U[0, pi),
  additive intensities U[-0.3, 0.6]) on the grid [-1, 1]^2, seed 1000+slice;
* smooth phase pi*(a x^2 + b y^2 + c x y + d x + e y), a..e ~ U[-0.5, 0.5];
* Gaussian coil maps exp(-|r - c_j|^2 / (2 * 0.6^2)) * exp(2 pi i j / J),
  centres c_j = 1.2 (cos 2 pi j / J, sin 2 pi j / J);
* k-space = centred unitary 2D DFT of coil image (DC at index n // 2);
* T2 series: each ellipse gets T2 ~ U[30, 150] ms, echo l has TE = 10 (l+1) ms;
* masks: 1D variable-density Cartesian rows, 2D Poisson-disc with a fully
  sampled centre, and per-echo shifted uniform Cartesian PE lines.
"""

from __future__ import annotations

import functools

import numpy as np


# ---------------------------------------------------------------------------
# images, phases, coils
# ---------------------------------------------------------------------------

def _grid(M: int, N: int):
    y = np.linspace(-1.0, 1.0, M)[:, None] * np.ones((1, N))
    x = np.ones((M, 1)) * np.linspace(-1.0, 1.0, N)[None, :]
    return x, y


def _ellipses(rng: np.random.Generator, n_random: int = 10):
    """Return a list of (cx, cy, ax, ay, angle, intensity)."""
    ells = [(0.0, 0.0, 0.7, 0.9, 0.0, 1.0)]
    for _ in range(n_random):
        cx, cy = rng.uniform(-0.6, 0.6, size=2)
        ax, ay = rng.uniform(0.05, 0.5, size=2)
        ang = rng.uniform(0.0, np.pi)
        inten = rng.uniform(-0.3, 0.6)
        ells.append((cx, cy, ax, ay, ang, inten))
    return ells


def _inside(x, y, e):
    cx, cy, ax, ay, ang, _ = e
    ca, sa = np.cos(ang), np.sin(ang)
    xr = (x - cx) * ca + (y - cy) * sa
    yr = -(x - cx) * sa + (y - cy) * ca
    return (xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0


def phantom_image(M: int, N: int, seed: int = 1000, t2_echo_times=None):
    """Complex image(s) with smooth phase.

    Returns (M, N) complex128, or (L, M, N) when ``t2_echo_times`` (ms) is given.
    """
    rng = np.random.default_rng(seed)
    x, y = _grid(M, N)
    ells = _ellipses(rng)
    a, b, c, d, e = rng.uniform(-0.5, 0.5, size=5)
    phase = np.exp(1j * np.pi * (a * x * x + b * y * y + c * x * y + d * x + e * y))
    if t2_echo_times is None:
        img = np.zeros((M, N))
        for el in ells:
            img += el[5] * _inside(x, y, el)
        return img * phase
    t2 = rng.uniform(30.0, 150.0, size=len(ells))
    te = np.asarray(t2_echo_times, dtype=np.float64)
    out = np.zeros((len(te), M, N))
    for el, t2e in zip(ells, t2):
        ins = _inside(x, y, el)
        out += el[5] * ins[None] * np.exp(-te / t2e)[:, None, None]
    return out * phase[None]


def coil_maps(J: int, M: int, N: int):
    x, y = _grid(M, N)
    maps = np.empty((J, M, N), dtype=np.complex128)
    for j in range(J):
        ang = 2.0 * np.pi * j / J
        cxj, cyj = 1.2 * np.cos(ang), 1.2 * np.sin(ang)
        r2 = (x - cxj) ** 2 + (y - cyj) ** 2
        maps[j] = np.exp(-r2 / (2.0 * 0.6 ** 2)) * np.exp(1j * ang)
    return maps


def _dft2c(img):
    """Centred unitary 2D DFT over the last two axes (synthesis of k-space)."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img, axes=ax), axes=ax, norm="ortho"), axes=ax)


def phantom_kspace(J: int, M: int, N: int, seed: int = 1000, noise: float = 0.0):
    """Fully sampled multi-coil k-space, (J, M, N) complex128."""
    img = phantom_image(M, N, seed)
    k = _dft2c(coil_maps(J, M, N) * img[None])
    if noise > 0:
        rng = np.random.default_rng(seed + 77)
        s = noise * np.abs(k).max()
        k = k + s * (rng.standard_normal(k.shape) + 1j * rng.standard_normal(k.shape)) / np.sqrt(2)
    return k


def t2_kspace(J: int, M: int, N: int, L: int = 8, seed: int = 1000):
    """Fully sampled multi-echo multi-coil k-space, (L, J, M, N) complex128."""
    te = 10.0 * (np.arange(L) + 1)
    img = phantom_image(M, N, seed, t2_echo_times=te)          # (L, M, N)
    return _dft2c(coil_maps(J, M, N)[None] * img[:, None])


# ---------------------------------------------------------------------------
# sampling masks
# ---------------------------------------------------------------------------

def mask_cartesian_vd(M: int, N: int, R: float = 3.0, n_center: int = 8, seed: int = 2000):
    """1D variable-density Cartesian mask: whole k-space rows (index along M).

    round(M/R) rows, the n_center central rows always included, the others drawn
    without replacement with density exp(-(k/(0.3 M))^2) in the centred index k.
    """
    rng = np.random.default_rng(seed)
    c = M // 2
    n_total = int(round(M / R))
    chosen = set(range(c - n_center // 2, c - n_center // 2 + n_center))
    rest = np.array([i for i in range(M) if i not in chosen])
    kc = (rest - c).astype(np.float64)
    p = np.exp(-(kc / (0.3 * M)) ** 2)
    p /= p.sum()
    extra = rng.choice(rest, size=max(0, n_total - len(chosen)), replace=False, p=p)
    rows = np.zeros(M, dtype=bool)
    rows[list(chosen)] = True
    rows[extra] = True
    return np.repeat(rows[:, None], N, axis=1)


def _poisson_disc_count(M, N, r0, growth, rng_seed, acs):
    """Dart throwing in a seeded random order: a pixel is kept when no kept pixel lies
    closer than its radius r0 (1 + growth rho), rho the normalised distance to the centre.
    The distance from every pixel to the nearest kept one is updated as pixels are kept."""
    rng = np.random.default_rng(rng_seed)
    cm, cn = M // 2, N // 2
    order = rng.permutation(M * N)
    taken = np.zeros((M, N), dtype=bool)
    # fully sampled centre
    taken[cm - acs // 2: cm - acs // 2 + acs, cn - acs // 2: cn - acs // 2 + acs] = True
    occ = np.zeros((M, N), dtype=bool)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    rho = np.hypot((ii - cm) / (M / 2), (jj - cn) / (N / 2)) / np.sqrt(2.0)
    rad = r0 * (1.0 + growth * rho)
    w = int(np.ceil(rad.max()))
    off = np.arange(-w, w + 1)
    hyp = np.hypot(off[:, None], off[None, :])
    near = np.full((M, N), np.inf)
    taken_f, near_f, rad_f = taken.ravel(), near.ravel(), rad.ravel()
    for idx in order:
        idx = int(idx)
        if taken_f[idx] or near_f[idx] < rad_f[idx]:
            continue
        i, j = divmod(idx, N)
        occ[i, j] = True
        i0, i1 = max(0, i - w), min(M, i + w + 1)
        j0, j1 = max(0, j - w), min(N, j + w + 1)
        np.minimum(near[i0:i1, j0:j1], hyp[i0 - i + w:i1 - i + w, j0 - j + w:j1 - j + w], out=near[i0:i1, j0:j1])
    return taken | occ


@functools.lru_cache(maxsize=64)
def _poisson_cached(M, N, R, acs, seed, growth):
    target = M * N / R
    lo, hi = 0.3, 6.0
    best = None
    for _ in range(18):
        r0 = 0.5 * (lo + hi)
        m = _poisson_disc_count(M, N, r0, growth, seed, acs)
        cnt = int(m.sum())
        best = m
        if abs(cnt - target) <= 0.02 * target:
            break
        if cnt > target:
            lo = r0
        else:
            hi = r0
    return best


def mask_poisson_disc(M: int, N: int, R: float = 4.0, acs: int = 24, seed: int = 2000, growth: float = 1.0):
    """2D Poisson-disc mask with radially growing radius and a fully sampled acs x acs centre.

    The base radius is tuned by bisection so that about M*N/R points are kept.
    """
    return _poisson_cached(int(M), int(N), float(R), int(acs), int(seed), float(growth)).copy()


def mask_t2_cartesian(L: int, N: int, R: int = 6, n_center: int = 16):
    """Per-echo shifted uniform Cartesian PE lines, (L, N) bool.

    Echo l keeps PE indices i with i % R == l % R, plus n_center central lines.
    The FE direction is fully sampled, so the mask does not depend on the FE index.
    """
    m = np.zeros((L, N), dtype=bool)
    c = N // 2
    for l in range(L):
        m[l, (np.arange(N) % R) == (l % R)] = True
        m[l, c - n_center // 2: c - n_center // 2 + n_center] = True
    return m


# ---------------------------------------------------------------------------
# the paper's other sampling patterns (parallel imaging, Section IV-A and Supplement S3)
# ---------------------------------------------------------------------------

def _acs_rows(M: int, n_acs: int):
    c = M // 2
    return set(range(c - n_acs // 2, c - n_acs // 2 + n_acs))


def _pf_rows(M: int, pf: float):
    """Rows a partial-Fourier acquisition keeps: the first round(pf M) phase-encode rows, which hold
    the k-space centre and one side of it."""
    return np.arange(M) < int(round(pf * M))


def mask_uniform_cartesian(M: int, N: int, R: int = 6, n_acs: int = 20, pf: float = 1.0):
    """Uniform Cartesian undersampling: every R-th phase-encode row (the centre row among them),
    plus n_acs central ACS rows, optionally cut to partial Fourier pf (e.g. 3/4)."""
    c = M // 2
    rows = ((np.arange(M) - c) % R) == 0
    rows[list(_acs_rows(M, n_acs))] = True
    rows &= _pf_rows(M, pf)
    return np.repeat(rows[:, None], N, axis=1)


def mask_gaussian_cartesian(M: int, N: int, rate: float = 0.34, n_acs: int = 22, seed: int = 2000,
                            pf: float = 1.0, width: float = 0.3):
    """Gaussian variable-density Cartesian undersampling at a total sampling rate: round(rate M)
    phase-encode rows, n_acs central ACS rows among them, the others drawn without replacement
    with density exp(-(k / (width M))^2) in the centred row index k, only from the rows a partial-
    Fourier acquisition pf keeps."""
    rng = np.random.default_rng(seed)
    c = M // 2
    keep = _pf_rows(M, pf)
    acs = sorted(i for i in _acs_rows(M, n_acs) if keep[i])
    rest = np.array([i for i in range(M) if keep[i] and i not in set(acs)])
    kc = (rest - c).astype(np.float64)
    p = np.exp(-(kc / (width * M)) ** 2)
    p /= p.sum()
    n_extra = max(0, min(len(rest), int(round(rate * M)) - len(acs)))
    extra = rng.choice(rest, size=n_extra, replace=False, p=p)
    rows = np.zeros(M, dtype=bool)
    rows[acs] = True
    rows[extra] = True
    return np.repeat(rows[:, None], N, axis=1)


def mask_random_2d(M: int, N: int, rate: float = 0.18, acs: int = 16, seed: int = 2000, pf: float = 1.0):
    """2D random undersampling at a sampling rate: the Poisson-disc pattern (radially growing radius,
    fully sampled acs x acs centre) tuned to rate / pf of the points, then cut to partial Fourier pf
    along the first axis (so the kept part carries about the requested total rate)."""
    m = mask_poisson_disc(M, N, R=pf / rate, acs=acs, seed=seed)
    m &= _pf_rows(M, pf)[:, None]
    return m


def sampling_rate(mask) -> float:
    return float(np.mean(mask))


# ---------------------------------------------------------------------------
# random states for step-level tests
# ---------------------------------------------------------------------------

def ragged_sizes(n_slices: int = 32, lo: int = 192, hi: int = 320, seed: int = 3000, rates=(4, 5, 6)):
    """Seeded slice shapes and acceleration rates of a ragged batch: [(M, N, R)], M, N ~ U{lo..hi}."""
    rng = np.random.default_rng(seed)
    M = rng.integers(lo, hi + 1, size=n_slices)
    N = rng.integers(lo, hi + 1, size=n_slices)
    R = rng.choice(np.asarray(rates), size=n_slices)
    return [(int(m), int(n), float(r)) for m, n, r in zip(M, N, R)]


def random_complex(shape, seed: int, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def undersample(k, mask):
    """Zero-fill k-space outside the mask (mask broadcast over leading axes)."""
    return np.where(mask, k, 0)
