"""The paper's sampling patterns as seeded generators (no method arithmetic): structure and rates."""

import numpy as np
import pytest

from paper_2107_11650_amd import inputs as I


def test_uniform_cartesian_with_acs_and_partial_fourier():
    M, N = 256, 200
    m = I.mask_uniform_cartesian(M, N, R=6, n_acs=20)
    rows = m[:, 0]
    assert np.all(m == rows[:, None])                       # whole phase-encode rows
    c = M // 2
    assert rows[c - 10:c + 10].all()                        # 20 ACS rows
    outer = np.nonzero(rows & ((np.arange(M) < c - 10) | (np.arange(M) >= c + 10)))[0]
    assert np.all((outer - c) % 6 == 0)                     # every 6th row elsewhere
    pf = I.mask_uniform_cartesian(M, N, R=6, n_acs=20, pf=0.75)
    assert not pf[192:].any() and np.array_equal(pf[:192], m[:192])
    assert abs(I.sampling_rate(pf) - 0.20) < 0.015          # "uniform + 3/4 PF, 0.20"


@pytest.mark.parametrize("n_acs", [8, 14, 22])
def test_gaussian_cartesian_rate_and_acs(n_acs):
    M, N = 256, 256
    m = I.mask_gaussian_cartesian(M, N, rate=0.34, n_acs=n_acs, seed=2000)
    rows = m[:, 0]
    assert rows.sum() == round(0.34 * M)
    assert rows[M // 2 - n_acs // 2: M // 2 - n_acs // 2 + n_acs].all()
    # variable density: more rows near the centre than at the edge
    k = np.abs(np.arange(M) - M // 2)
    assert rows[k < M // 8].mean() > rows[k > 3 * M // 8].mean()
    pf = I.mask_gaussian_cartesian(M, N, rate=0.30, n_acs=22, pf=0.75)
    assert not pf[192:].any() and pf[:, 0].sum() == round(0.30 * M)    # "3/4 PF, total 0.30"
    assert np.array_equal(I.mask_gaussian_cartesian(M, N, 0.34, n_acs, seed=5),
                          I.mask_gaussian_cartesian(M, N, 0.34, n_acs, seed=5))


def test_random_2d_rate_centre_and_partial_fourier():
    M, N = 256, 256
    m = I.mask_random_2d(M, N, rate=0.18, acs=16, seed=2000)
    assert abs(I.sampling_rate(m) - 0.18) < 0.01
    assert m[120:136, 120:136].all()
    pf = I.mask_random_2d(M, N, rate=0.17, acs=16, seed=2000, pf=0.8)
    assert not pf[int(round(0.8 * M)):].any() and abs(I.sampling_rate(pf) - 0.17) < 0.01
