"""The allocation-free low-rank entry point (shlr_lowrank_lines_noalloc) against shlr_lowrank_lines.

Two calls in a row through the C ABI, the second with a smaller input: a 40-line batch of
8-coil 256-point lines (232 x 200 lifts, more than the fixed scratch holds at once, so it runs in
chunks), then 6 lines of 4-coil 64-point lines in FP64.  Outputs (D, the adjoint lines, the ranks)
must equal the workspace entry point's bit for bit (each matrix is computed by the same kernels
in both), and both stay at the mixed/FP64 bars against the oracle.
"""

import numpy as np
import pytest

from oracle import shlr_oracle as O
from paper_2107_11650_amd import inputs
from parity_util import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(B, J, n, k, seed):
    lift = O.LineLift(n, k, True, False)
    h = inputs.random_complex((B, J, n), seed=seed)
    D = inputs.random_complex((B, lift.p, lift.q(J)), seed=seed + 1, scale=0.5)
    T = lift.forward(h) + D / 3.0
    srt = np.sort(np.linalg.svd(T, compute_uv=False).ravel())
    thr = 0.5 * (srt[len(srt) // 2] + srt[len(srt) // 2 + 1])
    return lift, h, D, thr


def test_noalloc_matches_workspace_entry_point_twice():
    from paper_2107_11650_amd import shlr
    for (B, J, n, k, dt, bars) in ((40, 8, 256, 25, torch.complex64, (1e-11, 2e-4)),
                                   (6, 4, 64, 8, torch.complex128, (1e-20, 1e-11))):
        lift, h, D, thr = _case(B, J, n, k, seed=300 + n)
        print(f"no-alloc case: {B} lines, J={J}, n={n}, k={k}, {dt}", flush=True)
        hd = torch.from_numpy(h).to(dt).cuda()
        d1 = torch.from_numpy(D).to(dt).cuda()
        d2 = d1.clone()
        b1, r1 = shlr.lowrank_lines(hd, d1, k, 3.0, 2.0, thr, ranks=True)
        b2, r2 = shlr.lowrank_lines_noalloc(hd, d2, k, 3.0, 2.0, thr, ranks=True)
        torch.cuda.synchronize()
        assert torch.equal(r1, r2)
        assert torch.equal(b1, b2) and torch.equal(d1, d2)
        Dn_ref, b_ref = O.lowrank_step(lift, h, D, 3.0, 2.0, thr)
        check(d2.cpu().numpy().astype(np.complex128), Dn_ref, *bars, label=f"no-alloc D n={n}")
        check(b2.cpu().numpy().astype(np.complex128), b_ref, *bars, label=f"no-alloc b n={n}")
