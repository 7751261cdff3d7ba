"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: explicit
formulas, brute force, closed forms, invariants and special cases that reduce
to textbook routines.  None of these needs a GPU.
"""

import numpy as np
import pytest

from oracle import brute
from oracle import shlr_oracle as O
from paper_2107_11650_amd import inputs


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# --------------------------------------------------------------------------
# F^1D: centred unitary DFT (DC at n // 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 8, 64, 193])
def test_fftc_matches_explicit_dft_matrix(n):
    x = inputs.random_complex((3, n), seed=n)
    F = brute.dft_matrix(n)
    assert rel(O.fftc(x, -1), x @ F.T) < 1e-13
    assert rel(O.ifftc(O.fftc(x, -1), -1), x) < 1e-13
    assert abs(np.linalg.norm(O.fftc(x, -1)) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("n", [8, 9, 64, 65])
def test_dagger_of_real_row_is_itself(n):
    # Eq. 4: a real image row has a conjugate-symmetric spectrum, so the virtual
    # coil (conjugate, flipped about the centre) equals the original line.
    x = np.random.default_rng(n).standard_normal((2, n))
    h = O.fftc(x, -1)
    assert rel(O.dagger(h), h) < 1e-14
    # and the dagger is an involution for any line
    z = inputs.random_complex((2, n), seed=1)
    assert rel(O.dagger(O.dagger(z)), z) == 0


def test_weights_are_dft_of_first_difference():
    # W of Eq. 2: multiplying the spectrum by w equals taking the circular first
    # difference x[t] - x[t-1] in the image domain.
    for n in (8, 9, 64):
        x = inputs.random_complex(n, seed=n)
        lhs = O.weights(n) * O.fftc(x)
        rhs = O.fftc(x - np.roll(x, 1))
        assert rel(lhs, rhs) < 1e-13
        assert O.weights(n)[n // 2] == 0


# --------------------------------------------------------------------------
# H and the lift
# --------------------------------------------------------------------------

def test_hankel_counts_and_left_inverse():
    for n, k in ((16, 1), (16, 5), (16, 16), (57, 8), (256, 25)):
        c = O.hankel_counts(n, k)
        # H* H is diagonal with the anti-diagonal counts
        HtH = np.zeros((n, n))
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1
            HtH[:, i] = O.hankel_adj(O.hankel(e, k), n).real
        assert np.allclose(HtH, np.diag(c), atol=0)
        # anti-diagonal averaging is a left inverse of H
        v = inputs.random_complex(n, seed=n + k)
        assert rel(O.hankel_adj(O.hankel(v, k), n) / c, v) < 1e-14


@pytest.mark.parametrize("vc", [False, True])
@pytest.mark.parametrize("use_w", [False, True])
def test_lift_adjoint_identity(vc, use_w):
    # <L h, R> = <h, L* R>; real part for the antilinear virtual-coil blocks (Eq. 4).
    n, k, J = 23, 6, 3
    lift = O.LineLift(n, k, use_w, vc)
    h = inputs.random_complex((4, J, n), seed=3)
    R = inputs.random_complex((4, lift.p, lift.q(J)), seed=4)
    lhs = np.vdot(lift.forward(h), R)
    rhs = np.vdot(h, lift.adjoint(R, J))
    if vc:
        assert abs(lhs.real - rhs.real) < 1e-12 * abs(lhs)
    else:
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("vc", [False, True])
def test_lift_matches_entrywise_definition(vc):
    n, k, J = 11, 4, 2
    h = inputs.random_complex((J, n), seed=5)
    assert rel(O.LineLift(n, k, True, vc).forward(h), brute.lift_line(h, k, True, vc)) < 1e-14


@pytest.mark.parametrize("vc", [False, True])
def test_lift_gram_is_diagonal(vc):
    # The Eq. 15 Hankel term is diagonal per line with gram_diag().
    n, k, J = 13, 4, 2
    lift = O.LineLift(n, k, True, vc)
    A = brute.real_matrix(lambda h: lift.forward(h), (J, n))
    G = A.T @ A
    d = np.tile(lift.gram_diag(), J)
    assert np.abs(G - np.diag(np.concatenate([d, d]))).max() < 1e-12


# --------------------------------------------------------------------------
# low-rank premises (Section I, Section III-A)
# --------------------------------------------------------------------------

def test_damped_exponentials_give_rank_r():
    n, k, r = 64, 10, 3
    rng = np.random.default_rng(0)
    z = np.exp(-rng.uniform(0.01, 0.1, r) + 2j * np.pi * rng.uniform(0, 1, r))
    a = inputs.random_complex(r, seed=9)
    v = (a[None, :] * z[None, :] ** np.arange(n)[:, None]).sum(1)
    s = np.linalg.svd(O.hankel(v, k), compute_uv=False)
    assert s[r - 1] / s[0] > 1e-6
    assert s[r] / s[0] < 1e-12


def test_piecewise_constant_row_gives_rank_equal_to_jumps():
    # W F of a piecewise-constant row with s circular jumps is a sum of s
    # exponentials, so its Hankel matrix has rank s.
    n, k = 64, 12
    x = np.zeros(n)
    x[10:20] = 1.0
    x[30:45] = -0.5
    jumps = np.count_nonzero(x - np.roll(x, 1))
    lift = O.LineLift(n, k, True, False)
    s = np.linalg.svd(lift.forward(O.fftc(x)[None]), compute_uv=False)
    assert jumps == 4
    assert s[jumps - 1] / s[0] > 1e-6
    assert s[jumps] / s[0] < 1e-12


def test_echo_decay_gives_rank_one_across_coils():
    # A mono-exponential decay along echoes times coil weights: the echo-direction
    # lift (no W, no F) of Eq. 7 has rank 1.
    L, J, k = 8, 5, 4
    te = 10.0 * (np.arange(L) + 1)
    sens = inputs.random_complex(J, seed=2)
    lines = sens[:, None] * 0.8 * np.exp(-te / 70.0)[None, :]
    s = np.linalg.svd(O.LineLift(L, k, False, False).forward(lines), compute_uv=False)
    assert s[1] / s[0] < 1e-12


# --------------------------------------------------------------------------
# SVT (Eq. 16)
# --------------------------------------------------------------------------

def test_svt_limits_and_prox_optimality():
    T = inputs.random_complex((20, 12), seed=11)
    s = np.linalg.svd(T, compute_uv=False)
    assert rel(O.svt(T, 0.0), T) < 1e-13
    assert np.abs(O.svt(T, s[0] * 1.0001)).max() == 0
    t = np.median(s)
    Z = O.svt(T, t)
    # prox of t ||.||_*: (T - Z)/t = U_r V_r^H + W with ||W||_2 <= 1, W orthogonal to U_r, V_r
    U, sz, Vh = np.linalg.svd(Z)
    r = int((sz > 1e-10).sum())
    assert r == int((s > t).sum())
    Ur, Vr = U[:, :r], Vh[:r].conj().T
    W = (T - Z) / t - Ur @ Vr.conj().T
    assert np.linalg.norm(W, 2) <= 1 + 1e-10
    assert np.abs(Ur.conj().T @ W).max() < 1e-10
    assert np.abs(W @ Vr).max() < 1e-10


def test_svt_window_one_is_coil_svt():
    # k = 1: the lift of a line is the n x J coil matrix (times W).
    n, J = 16, 4
    h = inputs.random_complex((J, n), seed=12)
    lift = O.LineLift(n, 1, False, False)
    assert rel(lift.forward(h), h.T) == 0
    Z = O.svt(lift.forward(h), 0.3)
    U, s, Vh = np.linalg.svd(h.T, full_matrices=False)
    assert rel(Z, U @ np.diag(np.maximum(s - 0.3, 0)) @ Vh) < 1e-13


def test_svt_single_row_is_vector_soft_threshold():
    # p = 1 (k = n), J = 1: the lift is a row vector, SVT = v max(1 - t/||v||, 0).
    n = 9
    v = inputs.random_complex((1, n), seed=13)
    T = O.LineLift(n, n, False, False).forward(v)
    assert T.shape == (1, n)
    t = 0.4 * np.linalg.norm(v)
    assert rel(O.svt(T, t), v * (1 - t / np.linalg.norm(v))) < 1e-14


def test_low_rank_step_fixed_point_leaves_row_unchanged():
    # A row whose lift L has rank r, with multiplier D = U_r V_r^H, is a fixed
    # point of the Z/D step (Eqs. 16, 13): Z = L and D is unchanged.
    n, k, r, J, beta = 48, 8, 3, 2, 2.0
    rng = np.random.default_rng(1)
    z = np.exp(-rng.uniform(0.01, 0.1, r) + 2j * np.pi * rng.uniform(0, 1, r))
    amp = inputs.random_complex((J, r), seed=14)
    lines = (amp[:, None, :] * z[None, None, :] ** np.arange(n)[None, :, None]).sum(-1)
    lift = O.LineLift(n, k, False, False)
    Lx = lift.forward(lines)
    U, s, Vh = np.linalg.svd(Lx, full_matrices=False)
    D = U[:, :r] @ Vh[:r]
    Z = O.svt(Lx + D / beta, 1.0 / beta)
    assert rel(Z, Lx) < 1e-12
    Dn = D + beta * (Lx - Z)
    assert rel(Dn, D) < 1e-12


# --------------------------------------------------------------------------
# Eq. 15 closed form against a dense solve (brute force)
# --------------------------------------------------------------------------

def _tiny_pi(J=2, M=8, N=8, seed=0):
    k = inputs.phantom_kspace(J, M, N, seed=1000 + seed)
    mask = inputs.mask_cartesian_vd(M, N, R=2.0, n_center=2, seed=2000 + seed)
    mask[M // 2, :] = True
    Y = inputs.undersample(k, mask)
    return Y / np.abs(Y).max(), mask


@pytest.mark.parametrize("vc", [False, True])
@pytest.mark.parametrize("hard", [False, True])
def test_x_update_closed_form_equals_dense_solve(vc, hard):
    Y, mask = _tiny_pi()
    prm = O.PIParams(k_row=3, k_col=3, lam=50.0, beta=0.7, tau=0.7, vc=vc, hard_dc=hard, normalize=False)
    st = O.pi_init(Y, mask, prm)
    st.Zr[...] = inputs.random_complex(st.Zr.shape, seed=21)
    st.Zc[...] = inputs.random_complex(st.Zc.shape, seed=22)
    st.Dr[...] = inputs.random_complex(st.Dr.shape, seed=23)
    st.Dc[...] = inputs.random_complex(st.Dc.shape, seed=24)
    K = O.pi_x_update(Y, mask, st, prm)
    b = brute.BrutePI(Y, mask, 3, 3, 50.0, 0.0, 0.7, 0.7, vc, hard_dc=hard)
    b.Zr, b.Zc = list(st.Zr), list(st.Zc)
    b.Dr, b.Dc = list(st.Dr), list(st.Dc)
    b.x_update()
    assert rel(K, b.f2(b.X)) < 1e-11
    if hard:
        assert np.array_equal(K[:, mask], Y[:, mask])


def test_soft_dc_tends_to_hard_dc():
    Y, mask = _tiny_pi()
    prm = O.PIParams(k_row=3, k_col=3, beta=0.7, iters=3, normalize=False)
    hard = O.shlr_pi(Y, mask, O.PIParams(**{**prm.__dict__, "hard_dc": True}))
    errs = [rel(O.shlr_pi(Y, mask, O.PIParams(**{**prm.__dict__, "lam": lam}))[:, mask], hard[:, mask])
            for lam in (1e2, 1e4, 1e6)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


# --------------------------------------------------------------------------
# whole iterations on 8x8 k-space against the dense brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("vc", [False, True])
def test_pi_iterations_match_brute_force(vc):
    Y, mask = _tiny_pi()
    prm = O.PIParams(k_row=3, k_col=3, lam=30.0, beta=2.0, tau=1.5, vc=vc, iters=10, normalize=False)
    K = O.shlr_pi(Y, mask, prm)
    b = brute.BrutePI(Y, mask, 3, 3, 30.0, 0.0, 2.0, 1.5, vc)
    Kb = b.run(10)
    assert O.nmse(K, Kb) < 1e-24


def test_pi_hard_dc_iterations_match_brute_force():
    Y, mask = _tiny_pi(seed=1)
    prm = O.PIParams(k_row=3, k_col=4, beta=2.0, vc=False, iters=6, hard_dc=True, normalize=False)
    K = O.shlr_pi(Y, mask, prm)
    b = brute.BrutePI(Y, mask, 3, 4, 0.0, 0.0, 2.0, 2.0, False, hard_dc=True)
    Kb = b.run(6)
    assert O.nmse(K, Kb) < 1e-22
    assert np.array_equal(K[:, mask], Y[:, mask])


def test_spirit_convolution_matches_dense_matrix():
    J, M, N = 2, 6, 7
    g = inputs.random_complex((J, J, 3, 3), seed=31)
    K = inputs.random_complex((J, M, N), seed=32)
    A = brute.spirit_kspace_matrix(g, M, N)
    assert rel(O.spirit_apply(K, g).ravel(), A @ K.ravel()) < 1e-13
    V = inputs.random_complex((J, M, N), seed=33)
    assert rel(O.spirit_adjoint(V, g).ravel(), A.conj().T @ V.ravel()) < 1e-13


def test_spirit_x_update_pcg_converges_to_dense_solve():
    Y, mask = _tiny_pi()
    g = inputs.random_complex((2, 2, 3, 3), seed=34) * 0.2
    for t in range(2):
        g[t, t, 1, 1] = 0
    prm = O.PIParams(k_row=3, k_col=3, lam=20.0, lam1=5.0, beta=1.0, n_cg=300, normalize=False)
    st = O.pi_init(Y, mask, prm)
    st.Zr[...] = inputs.random_complex(st.Zr.shape, seed=35)
    st.Zc[...] = inputs.random_complex(st.Zc.shape, seed=36)
    K = O.pi_x_update(Y, mask, st, prm, g)
    b = brute.BrutePI(Y, mask, 3, 3, 20.0, 5.0, 1.0, 1.0, False, g=g)
    b.Zr, b.Zc, b.Dr, b.Dc = list(st.Zr), list(st.Zc), list(st.Dr), list(st.Dc)
    b.x_update()
    assert rel(K, b.f2(b.X)) < 1e-10


def test_spirit_calibration_fits_fully_sampled_data():
    # Eq. 3 premise: each k-space point is a convolution of its multi-coil
    # neighbourhood.  A kernel calibrated on the centre reproduces the whole
    # smooth synthetic k-space closely.
    J, M, N = 4, 48, 48
    K = inputs.phantom_kspace(J, M, N, seed=1003)
    K = K / np.abs(K).max()
    g = O.spirit_calibrate(K, acs=20, ks=5)
    for t in range(J):
        assert g[t, t, 2, 2] == 0
    res = O.spirit_apply(K, g) - K
    assert np.linalg.norm(res) / np.linalg.norm(K) < 0.05


# --------------------------------------------------------------------------
# SHLR-P / SHLR-VP against the dense brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("vc", [False, True])
def test_param_iterations_match_brute_force(vc):
    L, J, M, N = 6, 2, 4, 8
    k = inputs.t2_kspace(J, M, N, L=L, seed=1001)
    mask = inputs.mask_t2_cartesian(L, N, R=3, n_center=2)
    Y = inputs.undersample(k, mask[:, None, None, :])
    Y = Y / np.abs(Y).max()
    prm = O.ParamParams(k_pe=3, k_l=3, lam=40.0, lam2=1.5, beta=2.0, tau=2.0, vc=vc, iters=8, normalize=False)
    Kout = O.shlr_param(Y, mask, prm)
    Yh = O.ifftc(Y, axis=2)
    Kh = O.ifftc(Kout, axis=2)
    for m in range(M):
        b = brute.BruteParam(Yh[:, :, m, :], mask, 3, 3, 40.0, 1.5, 2.0, 2.0, vc)
        Kb = b.run(8)
        assert O.nmse(Kh[:, :, m, :], Kb) < 1e-24


def test_param_den_has_no_zero():
    mask = np.zeros((8, 16), dtype=bool)
    den = O.param_den(mask, O.ParamParams(k_pe=5, k_l=4, beta=1.0))
    assert den.min() > 0


def test_param_oracle_fe_subset_matches_full_run():
    # the FE positions iterate independently: a subset run equals the same rows of the full run
    L, J, M, N = 4, 2, 6, 16
    k = inputs.t2_kspace(J, M, N, L=L, seed=1009)
    mask = inputs.mask_t2_cartesian(L, N, R=4, n_center=4)
    Y = inputs.undersample(k, mask[:, None, None, :])
    prm = O.ParamParams(k_pe=5, k_l=2, lam=1e3, lam2=1.0, beta=3.0, vc=True, iters=3)
    full = O.shlr_param(Y, mask, prm)
    hyb = np.transpose(O.ifftc(full, axis=2), (2, 0, 1, 3))          # (M, L, J, N)
    sub = O.shlr_param(Y, mask, prm, fe_positions=[1, 4])
    assert rel(sub, hyb[[1, 4]]) < 1e-13


# --------------------------------------------------------------------------
# SPIRiT over whole iterations, and the calibration (Eq. 3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("vc", [False, True])
def test_spirit_iterations_match_brute_force(vc):
    # SHLR-S / SHLR-SV: the oracle's PCG X-update (run to convergence) inside whole ADMM iterations
    # against the dense solve of the brute force, 6 iterations on 8 x 8 k-space
    Y, mask = _tiny_pi(seed=2)
    g = inputs.random_complex((2, 2, 3, 3), seed=41) * 0.2
    for t in range(2):
        g[t, t, 1, 1] = 0
    prm = O.PIParams(k_row=3, k_col=3, lam=20.0, lam1=5.0, beta=1.0, vc=vc, n_cg=100, iters=6, normalize=False)
    K = O.shlr_pi(Y, mask, prm, g=g)
    Kb = brute.BrutePI(Y, mask, 3, 3, 20.0, 5.0, 1.0, 1.0, vc, g=g).run(6)
    assert O.nmse(K, Kb) < 1e-20


def _shift_conv(K, a):
    """out(x) = sum_d a[d] K(x + d) with d = (dm - h, dn - h), circular (the relation Eq. 3 states)."""
    h = a.shape[-1] // 2
    out = np.zeros_like(K)
    for dm in range(a.shape[0]):
        for dn in range(a.shape[1]):
            out = out + a[dm, dn] * np.roll(K, shift=(-(dm - h), -(dn - h)), axis=(-2, -1))
    return out


def _planted(M, N, acs, ks, tgt):
    # two coils: the target coil is exactly a planted 5x5 convolution of the other coil inside the
    # centred acs x acs block (a window shifted by one sample sees the perturbed outside)
    base = inputs.random_complex((M, N), seed=51)
    a = inputs.random_complex((ks, ks), seed=52) * 0.3
    K = np.stack([_shift_conv(base, a), base]) if tgt == 0 else np.stack([base, _shift_conv(base, a)])
    cm, cn = M // 2, N // 2
    inside = np.zeros((M, N), dtype=bool)
    inside[cm - acs // 2: cm - acs // 2 + acs, cn - acs // 2: cn - acs // 2 + acs] = True
    K[1 - tgt][~inside] += inputs.random_complex(((~inside).sum(),), seed=54)
    gp = np.zeros((2, 2, ks, ks), dtype=np.complex128)
    gp[tgt, 1 - tgt] = a
    return K, gp


@pytest.mark.parametrize("shape", [(40, 36), (41, 37)])
@pytest.mark.parametrize("tgt", [0, 1])
def test_spirit_calibration_recovers_planted_kernel(shape, tgt):
    M, N = shape
    K, gp = _planted(M, N, 24, 5, tgt)
    g = O.spirit_calibrate(K, acs=24, ks=5, reg=0.0)
    assert np.abs(g[tgt] - gp[tgt]).max() < 1e-10
    # the same data one sample off the centred block no longer fit the planted kernel
    for sh in ((1, 0), (0, 1), (-1, 0), (0, -1)):
        g2 = O.spirit_calibrate(np.roll(K, shift=sh, axis=(1, 2)), acs=24, ks=5, reg=0.0)
        assert np.abs(g2[tgt] - gp[tgt]).max() > 1e-3


def test_spirit_calibration_is_the_tikhonov_minimiser():
    # with reg > 0 each target's kernel is a stationary point of
    # sum_x |K_t(x) - sum_{s,d} g K_s(x + d)|^2 + mu |g|^2 over the fit positions, mu = reg tr(A^H A) / n,
    # checked through the gradient formed with circular shifts (not the calibration's matrix)
    J, M, N, acs, ks, reg = 3, 32, 30, 20, 5, 1e-2
    K = inputs.phantom_kspace(J, M, N, seed=1005)
    K = K / np.abs(K).max()
    g = O.spirit_calibrate(K, acs=acs, ks=ks, reg=reg)
    h = ks // 2
    cm, cn = M // 2, N // 2
    fit = np.zeros((M, N), dtype=bool)
    fit[cm - acs // 2 + h: cm - acs // 2 + acs - h, cn - acs // 2 + h: cn - acs // 2 + acs - h] = True
    for t in range(J):
        r = K[t] - sum(_shift_conv(K[s], g[t, s]) for s in range(J))
        grad = np.zeros((J, ks, ks), dtype=np.complex128)
        energy = 0.0
        for s in range(J):
            for dm in range(ks):
                for dn in range(ks):
                    if s == t and dm == h and dn == h:
                        continue
                    src = np.roll(K[s], shift=(-(dm - h), -(dn - h)), axis=(0, 1))[fit]
                    grad[s, dm, dn] = np.vdot(src, r[fit])          # sum_x conj(K_s(x+d)) r(x)
                    energy += np.vdot(src, src).real
        n_unk = J * ks * ks - 1
        mu = reg * energy / n_unk
        keep = np.ones((J, ks, ks), dtype=bool)
        keep[t, h, h] = False
        assert rel(grad[keep], mu * g[t][keep]) < 1e-9
        assert g[t, t, h, h] == 0


# --------------------------------------------------------------------------
# the relative-change stop of Algorithms S1 / S2
# --------------------------------------------------------------------------

def _stop_rule(Ks, tol):
    """First k (1-based) with ||K^k - K^{k-1}||^2 / ||K^{k-1}||^2 < tol, from the list [K^0, K^1, ...]."""
    for k in range(1, len(Ks)):
        d = np.sum(np.abs(Ks[k] - Ks[k - 1]) ** 2)
        if d / np.sum(np.abs(Ks[k - 1]) ** 2) < tol:
            return k
    return None


def test_pi_tol_stop_follows_the_printed_rule():
    J, M, N = 2, 24, 20
    k = inputs.phantom_kspace(J, M, N, seed=1013)
    mask = inputs.mask_cartesian_vd(M, N, R=2.5, n_center=4, seed=2013)
    Y = inputs.undersample(k, mask)
    base = dict(k_row=4, k_col=4, lam=1e3, beta=6.0)
    Ks = [Y] + [O.shlr_pi(Y, mask, O.PIParams(**base, iters=n)) for n in range(1, 16)]
    rels = [np.sum(np.abs(Ks[i] - Ks[i - 1]) ** 2) / np.sum(np.abs(Ks[i - 1]) ** 2) for i in range(1, 16)]
    # a tolerance between the changes of iterations 9 and 10, at least 10% from both
    tol = np.sqrt(rels[8] * rels[9])
    assert rels[9] < rels[8] and min(rels[8] / tol, tol / rels[9]) > 1.1, rels
    want = _stop_rule(Ks, tol)
    got, st = O.shlr_pi(Y, mask, O.PIParams(**base, iters=40, tol=tol), return_state=True)
    assert st.it == want
    assert np.array_equal(got, Ks[want])


def test_param_tol_stop_is_per_fe_position():
    L, J, M, N = 5, 2, 4, 24
    k = inputs.t2_kspace(J, M, N, L=L, seed=1014)
    k = k + 0.02 * np.abs(k).max() * inputs.random_complex(k.shape, seed=1015)
    mask = inputs.mask_t2_cartesian(L, N, R=3, n_center=4)
    Y = inputs.undersample(k, mask[:, None, None, :])
    base = dict(k_pe=4, k_l=2, lam=1e3, lam2=1.5, beta=5.0)
    Yh = np.transpose(O.ifftc(Y, axis=2), (2, 0, 1, 3))
    tol = 1e-3   # every change within 6% of it stays on one side (FP64 rounding cannot move a stop)
    want = []
    for m in range(M):
        Ks = [Yh[m]] + [O.shlr_param(Y, mask, O.ParamParams(**base, iters=n), fe_positions=[m])[0]
                        for n in range(1, 20)]
        want.append(_stop_rule(Ks, tol))
    assert None not in want and len(set(want)) > 1, want
    _, st = O.shlr_param(Y, mask, O.ParamParams(**base, iters=60, tol=tol), return_state=True)
    assert st.it_fe.tolist() == want


# --------------------------------------------------------------------------
# values the paper prints (tests/golden/paper_constants.json)
# --------------------------------------------------------------------------

def _paper():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")) as f:
        return json.load(f)


def test_stdlr_block_hankel_size_fixes_the_lift_orientation():
    # the introduction's block Hankel of 4-coil 256 x 256 data with pencil 23 is 2116 x 54756: window
    # and coils on one axis, positions on the other.  The 1D lift of reading c-4 (positions x window*coils)
    # gives that size when taken in both directions: (k * q) x p^2.
    c = _paper()["stdlr_block_hankel_shape"]
    lift = O.LineLift(c["n"], c["window"], True, False)
    assert c["window"] * lift.q(c["coils"]) == c["rows"]
    assert lift.p ** 2 == c["cols"]
    # the rejected orientation (coils along the positions axis) would give another size
    assert (c["window"] ** 2, (lift.p * c["coils"]) ** 2) != (c["rows"], c["cols"])


def test_oracle_defaults_follow_the_algorithms():
    c = _paper()
    assert O.PIParams().d0 == c["alg_init"]["d0"] and O.ParamParams().d0 == c["alg_init"]["d0"]
    assert O.ParamParams().iters == c["alg_s2_caps"]["max_iter"]
    st = O.pi_init(np.ones((1, 8, 8), complex), np.ones((8, 8), bool), O.PIParams(k_row=3, k_col=3))
    assert np.all(st.Zr == c["alg_init"]["z0"]) and np.all(st.Dr == c["alg_init"]["d0"])


def test_caller_weights_enter_every_weighted_operator():
    # W given as an array equal to the first difference reproduces the default run exactly, and other
    # weights keep the lift's adjoint identity and the diagonal Gram of reading c-2
    Y, mask = _tiny_pi(seed=3)
    prm = O.PIParams(k_row=3, k_col=3, lam=30.0, beta=2.0, vc=True, iters=4, normalize=False)
    a = O.shlr_pi(Y, mask, prm)
    prm_w = O.PIParams(k_row=3, k_col=3, lam=30.0, beta=2.0, vc=True, iters=4, normalize=False,
                       w_row=O.weights(8), w_col=O.weights(8))
    assert np.array_equal(O.shlr_pi(Y, mask, prm_w), a)
    w = inputs.random_complex(8, seed=61)
    lift = O.LineLift(8, 3, True, True, w)
    h = inputs.random_complex((2, 8), seed=62)
    R = inputs.random_complex((6, 12), seed=63)
    assert abs(np.vdot(lift.forward(h), R).real - np.vdot(h, lift.adjoint(R, 2)).real) < 1e-12
    G = brute.real_matrix(lambda x: lift.forward(x), (2, 8))
    GtG = G.T @ G
    assert np.abs(GtG - np.diag(np.diag(GtG))).max() < 1e-12
    assert rel(np.diag(GtG)[:8], lift.gram_diag()) < 1e-13
    # and the whole iteration with those weights against the brute force's entry-wise lift
    prm_r = O.PIParams(k_row=3, k_col=3, lam=30.0, beta=2.0, iters=3, normalize=False, w_row=w, w_col=w)
    K = O.shlr_pi(Y, mask, prm_r)
    b = brute.BrutePI(Y, mask, 3, 3, 30.0, 0.0, 2.0, 2.0, False, wvec=w)
    assert O.nmse(K, b.run(3)) < 1e-24
