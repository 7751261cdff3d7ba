"""Pins of the derivative oracle (unrolled SHLR, reverse mode) on the CPU.

The gradient oracle is tied to the NumPy forward oracle iterate by iterate and
to central finite differences of its own forward in FP64; the SVT derivative is
checked at the thresholds where it reduces to a closed form.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import shlr_grad as G   # noqa: E402
from oracle import shlr_oracle as O  # noqa: E402
from paper_2107_11650_amd import inputs  # noqa: E402


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def small_problem(J=2, M=12, N=10, seed=3):
    k = inputs.phantom_kspace(J, M, N, seed=1000 + seed)
    mask = inputs.mask_cartesian_vd(M, N, R=2.0, n_center=4, seed=2000 + seed)
    Y = inputs.undersample(k, mask)
    return Y / np.abs(Y).max(), mask


def loss(Y, mask, prm, n, gK):
    K = G.unrolled_pi(torch.from_numpy(Y), torch.tensor(prm.lam, dtype=torch.float64), mask, prm, n)
    return float((np.conj(gK) * K.numpy()).real.sum())


@pytest.mark.parametrize("vc", [False, True])
def test_torch_forward_matches_numpy_oracle(vc):
    Y, mask = small_problem()
    prm = O.PIParams(k_row=4, k_col=3, lam=50.0, beta=4.0, tau=2.0, vc=vc, iters=4, normalize=False)
    ref = O.shlr_pi(Y, mask, prm)
    out = G.unrolled_pi(torch.from_numpy(Y), torch.tensor(50.0, dtype=torch.float64), mask, prm, 4).numpy()
    assert O.nmse(out, ref) < 1e-26


@pytest.mark.parametrize("vc", [False, True])
def test_torch_adjoint_lift_is_the_adjoint(vc):
    lift = O.LineLift(11, 4, True, vc)
    tl = G.TorchLift(lift)
    h = inputs.random_complex((3, 2, 11), seed=5)
    R = inputs.random_complex((3, lift.p, lift.q(2)), seed=6)
    lhs = np.vdot(tl.forward(torch.from_numpy(h)).numpy(), R).real
    rhs = np.vdot(h, tl.adjoint(torch.from_numpy(R), 2).numpy()).real
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert rel(tl.adjoint(torch.from_numpy(R), 2).numpy(), lift.adjoint(R, 2)) < 1e-14


def _singular_gap(Y, mask, prm, n):
    """Smallest |sigma - t| met by any SVT of the run (finite differences must not cross it)."""
    st = O.pi_init(Y, mask, prm)
    J, M, N = Y.shape
    Lr, Lc = O.pi_lifts(M, N, prm)
    gap = np.inf
    for _ in range(n - 1):
        st.K = O.pi_x_update(Y, mask, st, prm)
        Hr = np.transpose(O.ifftc(st.K, axis=1), (1, 0, 2))
        Hc = np.transpose(O.ifftc(st.K, axis=2), (2, 0, 1))
        for Lf, H, D in ((Lr, Hr, st.Dr), (Lc, Hc, st.Dc)):
            s = np.linalg.svd(Lf.forward(H) + D / prm.beta, compute_uv=False)
            gap = min(gap, np.abs(s - 1.0 / prm.beta).min())
        O.pi_zd_update(st, prm)
    return gap


@pytest.mark.parametrize("vc,n", [(False, 3), (True, 3), (False, 5)])
def test_gradient_matches_central_differences(vc, n):
    Y, mask = small_problem(seed=4)
    prm = O.PIParams(k_row=4, k_col=3, lam=50.0, beta=4.0, tau=2.0, vc=vc, normalize=False)
    gap = _singular_gap(Y, mask, prm, n)
    assert gap > 1e-4, "pick a problem away from sigma = t"
    gK = inputs.random_complex(Y.shape, seed=11)
    K, gY, gl = G.unrolled_pi_vjp(Y, mask, prm, n, gK)
    rng = np.random.default_rng(12)
    for trial in range(3):
        d = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
        eps = 1e-6
        fd = (loss(Y + eps * d, mask, prm, n, gK) - loss(Y - eps * d, mask, prm, n, gK)) / (2 * eps)
        an = np.vdot(gY, d).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.linalg.norm(gY) * np.linalg.norm(d))
    # the data-consistency weight
    eps = 1e-5 * prm.lam
    hi = loss(Y, mask, _with_lam(prm, prm.lam + eps), n, gK)
    lo = loss(Y, mask, _with_lam(prm, prm.lam - eps), n, gK)
    fd = (hi - lo) / (2 * eps)
    assert abs(fd - gl) <= 1e-6 * max(abs(gl), 1e-12)


def _with_lam(prm, lam):
    p = O.PIParams(k_row=prm.k_row, k_col=prm.k_col, lam=lam, beta=prm.beta, tau=prm.tau, vc=prm.vc,
                   use_w=prm.use_w, d0=prm.d0, normalize=False)
    return p


def test_single_iteration_gradient_is_the_data_term():
    # With one iteration K_1 = (lambda U Y + beta F(B_0)) / den and B_0 does not depend on Y:
    # the gradient is lambda * mask * gK / den, exactly.
    Y, mask = small_problem(seed=5)
    prm = O.PIParams(k_row=4, k_col=3, lam=30.0, beta=4.0, normalize=False)
    gK = inputs.random_complex(Y.shape, seed=13)
    K, gY, gl = G.unrolled_pi_vjp(Y, mask, prm, 1, gK)
    den = O.pi_den(mask, prm)
    assert rel(gY, prm.lam * mask * gK / den) < 1e-14
    # d K / d lambda = mask (Y - K) / den
    assert abs(gl - np.vdot(gK, mask * (Y - K) / den).real) < 1e-12 * abs(gl)


def test_svt_derivative_closed_forms():
    T = torch.from_numpy(inputs.random_complex((7, 5), seed=21))
    gZ = inputs.random_complex((7, 5), seed=22)
    s = np.linalg.svd(T.numpy(), compute_uv=False)
    for t, expect in ((0.0, gZ), (1.01 * s[0], np.zeros_like(gZ))):
        Tl = T.clone().requires_grad_(True)
        Z = G.svt_t(Tl, t)
        (g,) = torch.autograd.grad((torch.conj(torch.from_numpy(gZ)) * Z).real.sum(), Tl)
        assert rel(g.numpy(), expect) < 1e-12 if t == 0 else np.abs(g.numpy()).max() < 1e-14
