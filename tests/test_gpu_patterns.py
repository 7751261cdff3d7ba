"""GPU parity of SHLR-SV (virtual coils + SPIRiT) under the paper's other sampling patterns
(uniform R = 6 with ACS lines, Gaussian Cartesian at 0.34 with few and many ACS lines, 3/4 partial
Fourier at 0.30, 2D random at 0.18, 4/5 partial Fourier 2D random at 0.17, uniform with 3/4 partial
Fourier), 4 coils, 64 x 64, 5 iterations, against the FP64 oracle with the same SPIRiT kernel
(calibrated on the centre 6 x 6 or 8 x 8 block; with 2 ACS lines that block is partly zero-filled,
as a calibration on such data is, and the Tikhonov term carries the underdetermined fit)."""

import numpy as np
import pytest

from oracle import shlr_oracle as O
from paper_2107_11650_amd import inputs as I
from parity_util import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M = N = 64
# ACS line counts scaled from the paper's 256-row patterns (20 and 8..22 lines) to 64 rows
PATTERNS = {
    "uniform_R6_acs6": (lambda: I.mask_uniform_cartesian(M, N, R=6, n_acs=6), 6),
    "gauss_0.34_acs6": (lambda: I.mask_gaussian_cartesian(M, N, rate=0.34, n_acs=6, seed=2002), 6),
    "gauss_0.34_acs2": (lambda: I.mask_gaussian_cartesian(M, N, rate=0.34, n_acs=2, seed=2003), 6),
    "gauss_pf3/4_0.30": (lambda: I.mask_gaussian_cartesian(M, N, rate=0.30, n_acs=6, seed=2004, pf=0.75), 6),
    "random2d_0.18": (lambda: I.mask_random_2d(M, N, rate=0.18, acs=8, seed=2005), 8),
    "random2d_pf4/5_0.17": (lambda: I.mask_random_2d(M, N, rate=0.17, acs=8, seed=2006, pf=0.8), 8),
    "uniform_R6_pf3/4": (lambda: I.mask_uniform_cartesian(M, N, R=6, n_acs=6, pf=0.75), 6),
}
BARS = {"fp64": (1e-18, 1e-11), "mixed": (1e-12, 2e-4)}


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(PATTERNS))
def test_shlr_sv_under_pattern(name, prec):
    from paper_2107_11650_amd import shlr
    make, acs = PATTERNS[name]
    mask = make()
    k = I.phantom_kspace(4, M, N, seed=1010)
    Y = I.undersample(k, mask)
    g = O.spirit_calibrate(Y / np.abs(Y).max(), acs=acs, ks=5)
    prm = O.PIParams(k_row=8, k_col=8, lam=1e4, lam1=10.0, beta=10.0, vc=True, n_cg=6, iters=5)
    ref = O.shlr_pi(Y, mask, prm, g=g)
    p = shlr.Params(M=(M,), N=(N,), J=4, k_row=8, k_col=8, use_vc=True, lam=1e4, lambda1=10.0, beta=10.0, tau=10.0,
                    n_cg=6, spirit_ksize=5, max_iter=5,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.init(torch.from_numpy(Y).to(plan.cdtype).cuda(), torch.from_numpy(mask.astype(np.uint8)).cuda())
    plan.set_spirit_kernel(g)
    plan.iterate(5)
    out = plan.kspace().cpu().numpy().astype(np.complex128)
    plan.close()
    check(out, ref, *BARS[prec], label=f"SHLR-SV {name} (rate {I.sampling_rate(mask):.3f}) {prec}")
