"""FP64 CPU oracle of the separable low-rank Hankel (SHLR) reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; both sides receive their inputs from ``paper_2107_11650_amd.inputs``.

It is a plain, slow NumPy (complex128) rendering of the paper's method, in the
paper's order and notation:

* operators of Section III-A (Eq. 2 and the text after it): F^1D, W, H, the
  coil-wise tilde lift, and the virtual-coil lift H_vc of Eq. 4;
* SHLR / SHLR-S / SHLR-V / SHLR-SV (Eqs. 2, 3, 5, 6) solved by the ADMM of
  Eqs. 9-17 in the order of Algorithm S1 (X-update, then Z, then D);
* SHLR-P / SHLR-VP (Eqs. 7, 8) solved by Eqs. S1-S9 in the order of
  Algorithm S2, every frequency-encode position independently.

The singular-value threshold is a direct LAPACK SVD of every lifted matrix
(no Gram matrix), so it is a different route from the GPU's Gram +
eigen-decomposition.

Readings of passages that the paper leaves open (all listed again in the
design notes with their justification):

* lifted domain: the 1D DFT of an image row/column (hybrid space), as the
  formula F^1D P_m X states (Eq. 2);
* DFTs are centred (DC at index n // 2) and unitary, so F* = F^-1 (Eq. 15);
* W is the DFT of the circular first difference, w(f) = 1 - exp(-2 pi i f / n)
  with the centred frequency f (Eq. 2 text);
* H(v) is (n-k+1) x k with H[a, b] = v[a+b]; coils (and virtual coils) are
  side by side along the window axis (Eq. 2 text and Eq. 4);
* the dagger of Eq. 4 is v_dag[i] = conj(v[(2 (n//2) - i) mod n]);
* Eq. 15 is applied exactly: every non-SPIRiT term of its normal matrix is
  diagonal in 2D k-space, so the inverse is an elementwise division; with
  SPIRiT the system is solved by a fixed number of preconditioned CG steps;
* the SPIRiT operator is a circular multi-coil convolution in k-space with a
  5x5 kernel that excludes each target's own centre sample (Eq. 3 text);
* initial values Z = 0, D = 1 (Algorithm S1 / S2), K^0 = Y;
* Y is divided by max |Y| before the iteration and the result is scaled back.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# 1D operators (Section III-A, Eq. 2 and the text after it; Eq. 4)
# ---------------------------------------------------------------------------

def fftc(x, axis=-1):
    """Centred unitary DFT along ``axis`` (F^1D; DC at index n // 2)."""
    return np.fft.fftshift(np.fft.fft(np.fft.ifftshift(x, axes=axis), axis=axis, norm="ortho"), axes=axis)


def ifftc(x, axis=-1):
    """Inverse of :func:`fftc` (its adjoint, since it is unitary)."""
    return np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(x, axes=axis), axis=axis, norm="ortho"), axes=axis)


def weights(n: int) -> np.ndarray:
    """W of Eq. 2: DFT of the circular first-difference filter, centred frequencies."""
    f = np.arange(n) - n // 2
    return 1.0 - np.exp(-2j * np.pi * f / n)


def flip_index(n: int) -> np.ndarray:
    """Index map of the dagger in Eq. 4: conjugate-symmetric partner about the centre."""
    return (2 * (n // 2) - np.arange(n)) % n


def dagger(v, axis=-1):
    """v_dag[i] = conj(v[flip(i)]) along ``axis`` (Eq. 4)."""
    return np.conj(np.take(v, flip_index(v.shape[axis]), axis=axis))


def hankel_index(n: int, k: int) -> np.ndarray:
    p = n - k + 1
    return np.arange(p)[:, None] + np.arange(k)[None, :]


def hankel(v, k: int):
    """H of Eq. 2: (..., n) -> (..., n-k+1, k), H[a, b] = v[a + b]."""
    return v[..., hankel_index(v.shape[-1], k)]


def hankel_adj(R, n: int):
    """Adjoint of H: anti-diagonal sums, (..., p, k) -> (..., n)."""
    p, k = R.shape[-2:]
    assert p == n - k + 1
    out = np.zeros(R.shape[:-2] + (n,), dtype=np.result_type(R, np.complex128))
    idx = hankel_index(n, k)
    for a in range(p):
        out[..., idx[a]] += R[..., a, :]
    return out


def hankel_counts(n: int, k: int) -> np.ndarray:
    """Diagonal of H* H: the number of entries on each anti-diagonal."""
    i = np.arange(n)
    return np.minimum.reduce([i + 1, np.full(n, k), np.full(n, n - k + 1), n - i]).astype(np.float64)


@dataclass(frozen=True)
class LineLift:
    """The lifted operator of one line direction: H~ W~ (Eq. 2) or H~_vc W~ (Eq. 4).

    n: line length; k: window; use_w: apply W; vc: append the virtual-coil blocks;
    wvec: caller weights in place of the first-difference W (the library's shlr_set_weights).
    """
    n: int
    k: int
    use_w: bool = True
    vc: bool = False
    wvec: np.ndarray | None = field(default=None, compare=False)

    @property
    def p(self):
        return self.n - self.k + 1

    def q(self, J):
        return self.k * J * (2 if self.vc else 1)

    def w(self):
        if not self.use_w:
            return np.ones(self.n, dtype=np.complex128)
        return weights(self.n) if self.wvec is None else np.asarray(self.wvec, dtype=np.complex128)

    def forward(self, h):
        """h: (..., J, n) lines of J coils -> (..., p, q) lifted matrices."""
        w = self.w()
        J = h.shape[-2]
        blocks = [hankel(w * h, self.k)]                      # (..., J, p, k)
        if self.vc:
            blocks.append(hankel(w * dagger(h), self.k))
        B = np.concatenate(blocks, axis=-3)                   # (..., V*J, p, k)
        B = np.moveaxis(B, -3, -2)                            # (..., p, V*J, k)
        return B.reshape(B.shape[:-2] + (B.shape[-2] * self.k,))

    def adjoint(self, R, J):
        """Adjoint (real-inner-product adjoint for the antilinear VC part): (..., p, q) -> (..., J, n)."""
        V = 2 if self.vc else 1
        Rb = R.reshape(R.shape[:-1] + (V * J, self.k))        # (..., p, V*J, k)
        Rb = np.moveaxis(Rb, -2, -3)                          # (..., V*J, p, k)
        g = np.conj(self.w()) * hankel_adj(Rb, self.n)        # (..., V*J, n)
        out = g[..., :J, :]
        if self.vc:
            out = out + dagger(g[..., J:, :])
        return out

    def gram_diag(self):
        """Diagonal of (lift)* (lift) acting on one coil line (Eq. 15 terms)."""
        c = hankel_counts(self.n, self.k)
        aw2 = np.abs(self.w()) ** 2
        r = c * aw2
        if self.vc:
            f = flip_index(self.n)
            r = r + c[f] * aw2[f]
        return r


def svt(T, t):
    """S_t of Eq. 16: U max(Sigma - t, 0) V^H, via a direct SVD (stacked)."""
    U, s, Vh = np.linalg.svd(T, full_matrices=False)
    return (U * np.maximum(s - t, 0.0)[..., None, :]) @ Vh


# ---------------------------------------------------------------------------
# SPIRiT (Eq. 3): circular multi-coil k-space convolution
# ---------------------------------------------------------------------------

def spirit_apply(K, g):
    """(G K)_j(x) = sum_{j', d} g[j, j', d] K_j'(x + d), circular; K: (J, M, N), g: (J, J, ks, ks)."""
    J, ks = g.shape[0], g.shape[-1]
    h = ks // 2
    out = np.zeros_like(K, dtype=np.complex128)
    for dm in range(ks):
        for dn in range(ks):
            sh = np.roll(K, shift=(-(dm - h), -(dn - h)), axis=(-2, -1))   # sh[x] = K[x + d]
            out += np.einsum("ab,bmn->amn", g[:, :, dm, dn], sh)
    return out


def spirit_adjoint(V, g):
    J, ks = g.shape[0], g.shape[-1]
    h = ks // 2
    out = np.zeros_like(V, dtype=np.complex128)
    for dm in range(ks):
        for dn in range(ks):
            t = np.einsum("ab,amn->bmn", np.conj(g[:, :, dm, dn]), V)
            out += np.roll(t, shift=(dm - h, dn - h), axis=(-2, -1))
    return out


def spirit_calibrate(Y, acs: int = 24, ks: int = 5, reg: float = 1e-3):
    """Least-squares SPIRiT kernel from the fully sampled acs x acs centre of Y (J, M, N).

    For each target coil j: Y_j(x) ~ sum_{j', d} g[j, j', d] Y_j'(x + d) over every
    position x whose ks x ks neighbourhood lies inside the centre block, without
    the target's own centre sample; Tikhonov weight reg * tr(A^H A) / n_unknowns.
    """
    J, M, N = Y.shape
    h = ks // 2
    cm, cn = M // 2, N // 2
    C = Y[:, cm - acs // 2: cm - acs // 2 + acs, cn - acs // 2: cn - acs // 2 + acs]
    pos = [(i, j) for i in range(h, acs - h) for j in range(h, acs - h)]
    cols = [(jj, dm, dn) for jj in range(J) for dm in range(ks) for dn in range(ks)]
    A = np.array([[C[jj, i + dm - h, j + dn - h] for (jj, dm, dn) in cols] for (i, j) in pos])
    g = np.zeros((J, J, ks, ks), dtype=np.complex128)
    for t in range(J):
        keep = [c for c, (jj, dm, dn) in enumerate(cols) if not (jj == t and dm == h and dn == h)]
        At = A[:, keep]
        b = np.array([C[t, i, j] for (i, j) in pos])
        AhA = At.conj().T @ At
        lam = reg * np.real(np.trace(AhA)) / AhA.shape[0]
        sol = np.linalg.solve(AhA + lam * np.eye(AhA.shape[0]), At.conj().T @ b)
        full = np.zeros(len(cols), dtype=np.complex128)
        full[keep] = sol
        g[t] = full.reshape(J, ks, ks)
    return g


# ---------------------------------------------------------------------------
# SHLR(-S/-V/-SV): Eqs. 2-6 by the ADMM of Eqs. 9-17, order of Algorithm S1
# ---------------------------------------------------------------------------

@dataclass
class PIParams:
    k_row: int = 8            # window of the row lifts (lines of length N)
    k_col: int = 8            # window of the column lifts (lines of length M)
    lam: float = 1e4          # data-consistency weight lambda (Eq. 2)
    lam1: float = 0.0         # SPIRiT weight lambda_1 (Eq. 3); 0 = off
    beta: float = 1.0         # ADMM penalty (Eq. 9)
    tau: float | None = None  # dual step (Eqs. 13-14); None = beta
    vc: bool = False          # virtual coils (Eq. 4)
    use_w: bool = True        # weighting W (Eq. 2)
    iters: int = 20
    tol: float = 0.0          # relative-change stop (Algorithm S1); <= 0: fixed count
    n_cg: int = 10            # PCG steps per X-update when lam1 > 0
    hard_dc: bool = False     # lambda = +inf: sampled entries kept exactly
    d0: float = 1.0           # initial multiplier value (Algorithm S1: D = 1)
    normalize: bool = True
    w_row: np.ndarray | None = None   # caller weights of the row lines (length N); None: first difference
    w_col: np.ndarray | None = None   # caller weights of the column lines (length M)

    def t(self):
        return self.tau if self.tau is not None else self.beta


@dataclass
class PIState:
    K: np.ndarray
    Zr: np.ndarray
    Dr: np.ndarray
    Zc: np.ndarray
    Dc: np.ndarray
    it: int = 0
    rel_change: list = field(default_factory=list)


def pi_lifts(M, N, prm: PIParams):
    return (LineLift(N, prm.k_row, prm.use_w, prm.vc, prm.w_row),   # rows: lines along n
            LineLift(M, prm.k_col, prm.use_w, prm.vc, prm.w_col))   # columns: lines along m


def pi_den(mask, prm: PIParams):
    """Diagonal of the Eq. 15 normal matrix in 2D k-space (without SPIRiT)."""
    M, N = mask.shape
    Lr, Lc = pi_lifts(M, N, prm)
    r = Lr.gram_diag()[None, :] + Lc.gram_diag()[:, None]
    if prm.hard_dc:
        return prm.beta * r
    return prm.lam * mask + prm.beta * r


def pi_init(Y, mask, prm: PIParams) -> PIState:
    J, M, N = Y.shape
    Lr, Lc = pi_lifts(M, N, prm)
    Zr = np.zeros((M, Lr.p, Lr.q(J)), dtype=np.complex128)
    Zc = np.zeros((N, Lc.p, Lc.q(J)), dtype=np.complex128)
    return PIState(K=Y.astype(np.complex128).copy(), Zr=Zr, Dr=np.full_like(Zr, prm.d0),
                   Zc=Zc, Dc=np.full_like(Zc, prm.d0))


def pi_rhs(Y, mask, st: PIState, prm: PIParams):
    """Right-hand side of Eq. 15 mapped to 2D k-space."""
    J, M, N = Y.shape
    Lr, Lc = pi_lifts(M, N, prm)
    Br = Lr.adjoint(st.Zr - st.Dr / prm.beta, J)           # (M, J, N): image m, k-space n
    Bc = Lc.adjoint(st.Zc - st.Dc / prm.beta, J)           # (N, J, M): k-space m, image n
    Br = np.transpose(Br, (1, 0, 2))
    Bc = np.transpose(Bc, (1, 2, 0))
    lr = 0.0 if prm.hard_dc else prm.lam
    return lr * mask * Y + prm.beta * fftc(Br, axis=1) + prm.beta * fftc(Bc, axis=2)


def pcg(apply_A, b, x0, precond, n_steps):
    """Preconditioned conjugate gradients, complex inner product, fixed step count."""
    x = x0.copy()
    r = b - apply_A(x)
    z = r / precond
    p = z.copy()
    rz = np.vdot(r, z).real
    for _ in range(n_steps):
        if rz == 0.0:
            break
        Ap = apply_A(p)
        alpha = rz / np.vdot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        z = r / precond
        rz_new = np.vdot(r, z).real
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def pi_x_update(Y, mask, st: PIState, prm: PIParams, g=None):
    """Eq. 15: exact elementwise inverse; PCG on the SPIRiT-augmented system."""
    rhs = pi_rhs(Y, mask, st, prm)
    den = pi_den(mask, prm)
    if prm.lam1 > 0:
        if prm.hard_dc:
            raise ValueError("SPIRiT needs a finite lambda")

        def A(x):
            e = spirit_apply(x, g) - x
            return den * x + prm.lam1 * (spirit_adjoint(e, g) - e)
        return pcg(A, rhs, st.K, den[None], prm.n_cg)
    free = ~mask if prm.hard_dc else np.ones_like(mask)
    if (den[free] <= 0).any():
        raise ValueError("Eq. 15 is singular: a k-space point has no data and no lifted term")
    K = np.divide(rhs, den, out=np.zeros_like(rhs), where=free[None])
    if prm.hard_dc:
        K = np.where(mask, Y, K)
    return K


def pi_zd_update(st: PIState, prm: PIParams):
    """Eqs. 16-17 (SVT of every row/column lift) then Eqs. 13-14 (multipliers)."""
    J, M, N = st.K.shape
    Lr, Lc = pi_lifts(M, N, prm)
    Hr = np.transpose(ifftc(st.K, axis=1), (1, 0, 2))       # rows m: (M, J, N)
    Hc = np.transpose(ifftc(st.K, axis=2), (2, 0, 1))       # columns n: (N, J, M)
    thr = 1.0 / prm.beta
    for Lf, H, Z, D in ((Lr, Hr, st.Zr, st.Dr), (Lc, Hc, st.Zc, st.Dc)):
        LX = Lf.forward(H)
        Z[...] = svt(LX + D / prm.beta, thr)
        D[...] = D + prm.t() * (LX - Z)


def shlr_pi(Y, mask, prm: PIParams, g=None, state: PIState | None = None, return_state=False):
    """SHLR / SHLR-S / SHLR-V / SHLR-SV (Algorithm S1). Y: (J, M, N) zero-filled centred k-space."""
    Y = np.asarray(Y, dtype=np.complex128)
    mask = np.asarray(mask, dtype=bool)
    scale = np.abs(Y).max() if prm.normalize else 1.0
    if scale == 0:
        scale = 1.0
    Yn = Y / scale
    st = state if state is not None else pi_init(Yn, mask, prm)
    for _ in range(prm.iters):
        K_prev = st.K
        st.K = pi_x_update(Yn, mask, st, prm, g)
        pi_zd_update(st, prm)
        st.it += 1
        nrm = np.vdot(K_prev, K_prev).real
        rel = np.vdot(st.K - K_prev, st.K - K_prev).real / nrm if nrm > 0 else np.inf
        st.rel_change.append(rel)
        if prm.tol > 0 and rel < prm.tol:
            break
    out = st.K * scale
    return (out, st) if return_state else out


# ---------------------------------------------------------------------------
# SHLR-P / SHLR-VP: Eqs. 7-8 by Eqs. S1-S9, order of Algorithm S2
# ---------------------------------------------------------------------------

@dataclass
class ParamParams:
    k_pe: int = 25            # window of the PE-direction lifts (per echo)
    k_l: int = 4              # window of the parameter-direction lifts (per PE position)
    lam: float = 1e4
    lam2: float = 2.0         # weight of the parameter-direction nuclear norms (Eq. 7)
    beta: float = 1.0
    tau: float | None = None
    vc: bool = False          # SHLR-VP (Eq. 8) when True
    use_w: bool = True
    iters: int = 100
    tol: float = 0.0
    hard_dc: bool = False
    d0: float = 1.0
    normalize: bool = True
    w_pe: np.ndarray | None = None   # caller weights of the PE lines (length N); None: first difference

    def t(self):
        return self.tau if self.tau is not None else self.beta


@dataclass
class ParamState:
    K: np.ndarray      # (M, L, J, N): PE k-space of every FE position m
    Zp: np.ndarray     # (M, L, p_pe, q_pe)
    Dp: np.ndarray
    Ze: np.ndarray     # (M, N, p_l, q_l)
    De: np.ndarray
    active: np.ndarray
    it: int = 0
    it_fe: np.ndarray | None = None      # iterations run by each FE position
    rel_change: list = field(default_factory=list)   # per iteration: relative change of each FE position


def param_lifts(L, N, prm: ParamParams):
    return (LineLift(N, prm.k_pe, prm.use_w, prm.vc, prm.w_pe),     # PE lines of each echo (Q_l)
            LineLift(L, prm.k_l, False, False))            # echo lines of each PE position (P_n)


def param_den(mask, prm: ParamParams):
    """den(l, k) = lam U_l(k) + beta r_PE(k) + beta c_L(l) (Eq. S7)."""
    L, N = mask.shape
    Lp, Le = param_lifts(L, N, prm)
    r = Lp.gram_diag()[None, :] + Le.gram_diag()[:, None]
    if prm.hard_dc:
        return prm.beta * r
    return prm.lam * mask + prm.beta * r


def shlr_param(Yk, mask, prm: ParamParams, return_state=False, fe_positions=None):
    """SHLR-P / SHLR-VP (Algorithm S2).

    Yk: (L, J, M, N) zero-filled centred k-space (M: frequency encode, fully
    sampled; N: phase encode).  mask: (L, N) PE lines acquired per echo.
    Returns the reconstructed k-space, (L, J, M, N).

    fe_positions: run only these frequency-encode positions (the iteration of
    each position is independent once the FE transform is applied) and return
    their hybrid-space result, (len(fe_positions), L, J, N), scaled back.
    """
    Yk = np.asarray(Yk, dtype=np.complex128)
    mask = np.asarray(mask, dtype=bool)
    L, J, M, N = Yk.shape
    scale = np.abs(Yk).max() if prm.normalize else 1.0
    if scale == 0:
        scale = 1.0
    Yh = ifftc(Yk / scale, axis=2)                          # 1D inverse DFT along FE
    Ym = np.transpose(Yh, (2, 0, 1, 3))                     # (M, L, J, N)
    if fe_positions is not None:
        Ym = Ym[np.asarray(fe_positions)]
        M = Ym.shape[0]
    Lp, Le = param_lifts(L, N, prm)
    den = param_den(mask, prm)                              # (L, N)
    Zp = np.zeros((M, L, Lp.p, Lp.q(J)), dtype=np.complex128)
    Ze = np.zeros((M, N, Le.p, Le.q(J)), dtype=np.complex128)
    st = ParamState(K=Ym.copy(), Zp=Zp, Dp=np.full_like(Zp, prm.d0), Ze=Ze,
                    De=np.full_like(Ze, prm.d0), active=np.ones(M, dtype=bool), it_fe=np.zeros(M, dtype=np.int64))
    lr = 0.0 if prm.hard_dc else prm.lam
    for _ in range(prm.iters):
        act = st.active
        if not act.any():
            break
        # X-update (Eq. S7)
        Bp = Lp.adjoint(st.Zp[act] - st.Dp[act] / prm.beta, J)             # (m, L, J, N) PE k-space
        Be = Le.adjoint(st.Ze[act] - st.De[act] / prm.beta, J)             # (m, N, J, L) PE image
        Be = np.transpose(Be, (0, 3, 2, 1))                                # (m, L, J, N)
        rhs = lr * mask[None, :, None, :] * Ym[act] + prm.beta * Bp + prm.beta * fftc(Be, axis=3)
        Kn = rhs / den[None, :, None, :]
        if prm.hard_dc:
            Kn = np.where(mask[None, :, None, :], Ym[act], Kn)
        K_prev = st.K[act]
        st.K[act] = Kn
        # Z-updates (Eqs. S8, S9) and multipliers (Eqs. S5, S6)
        xe = np.transpose(ifftc(Kn, axis=3), (0, 3, 2, 1))                # (m, N, J, L)
        LXp = Lp.forward(Kn)                                               # (m, L, p, q)
        LXe = Le.forward(xe)                                               # (m, N, p, q)
        Zp_ = svt(LXp + st.Dp[act] / prm.beta, 1.0 / prm.beta)
        Ze_ = svt(LXe + st.De[act] / prm.beta, prm.lam2 / prm.beta)
        st.Zp[act] = Zp_
        st.Ze[act] = Ze_
        st.Dp[act] = st.Dp[act] + prm.t() * (LXp - Zp_)
        st.De[act] = st.De[act] + prm.t() * (LXe - Ze_)
        st.it += 1
        st.it_fe[act] += 1
        # relative change of each FE position (Algorithm S2's test, evaluated after the update)
        num = np.sum(np.abs(Kn - K_prev) ** 2, axis=(1, 2, 3))
        dd = np.sum(np.abs(K_prev) ** 2, axis=(1, 2, 3))
        rel = np.full(M, np.nan)
        rel[act] = np.where(dd > 0, num / np.where(dd > 0, dd, 1.0), np.inf)
        st.rel_change.append(rel)
        if prm.tol > 0:
            idx = np.nonzero(act)[0]
            st.active[idx[num < prm.tol * dd]] = False
    if fe_positions is not None:
        out = st.K * scale
    else:
        out = fftc(np.transpose(st.K, (1, 2, 0, 3)), axis=2) * scale
    return (out, st) if return_state else out


# ---------------------------------------------------------------------------
# single steps used by the step-level parity tests
# ---------------------------------------------------------------------------

def lowrank_step(lift: LineLift, h, D, beta, tau, thr):
    """One Z/D step on a batch of lines, plus the next X-update's adjoint term.

    h: (B, J, n) lines; D: (B, p, q).  Returns (D_new, Badj) with
    Z = S_thr(lift(h) + D / beta)            (Eq. 16)
    D_new = D + tau (lift(h) - Z)            (Eq. 13)
    Badj = lift*(Z - D_new / beta)           (the Eq. 15 right-hand-side term)
    """
    J = h.shape[-2]
    LX = lift.forward(h)
    Z = svt(LX + D / beta, thr)
    Dn = D + tau * (LX - Z)
    return Dn, lift.adjoint(Z - Dn / beta, J)


def nmse(a, b):
    """||a - b||^2 / ||b||^2."""
    return float(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2))
