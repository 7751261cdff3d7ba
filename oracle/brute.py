"""Dense brute-force SHLR for tiny inputs (8x8 and the like).

TEST INFRASTRUCTURE ONLY (see ``oracle/shlr_oracle.py``).  This is a second,
independently written implementation used to pin the oracle.  It never calls
the oracle's operators.  Instead it works with the paper's variables directly:

* the unknown is the multi-coil IMAGE X, as in Eqs. 2-6 and Eq. 15;
* every DFT is an explicit matrix built from its formula (no np.fft);
* every lifted operator (P_m or Q_n, then F^1D, W, H or H_vc) is evaluated
  entry by entry with Python loops and turned into a real matrix by applying
  it to the real basis vectors; this also handles the antilinear dagger;
* the X-subproblem of Eq. 10 is solved as a dense real linear system
  (normal equations of the quadratic objective; a KKT system for hard data
  consistency);
* the singular-value thresholds use one np.linalg.svd per matrix.
"""

from __future__ import annotations

import numpy as np


def dft_matrix(n: int) -> np.ndarray:
    """Centred unitary DFT matrix: F[f, t] = exp(-2 pi i (f - n//2)(t - n//2) / n) / sqrt(n)."""
    c = n // 2
    f = np.arange(n)[:, None] - c
    t = np.arange(n)[None, :] - c
    return np.exp(-2j * np.pi * f * t / n) / np.sqrt(n)


def realify(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v).ravel()
    return np.concatenate([v.real, v.imag])


def complexify(x: np.ndarray, shape) -> np.ndarray:
    n = x.size // 2
    return (x[:n] + 1j * x[n:]).reshape(shape)


def real_matrix(func, in_shape) -> np.ndarray:
    """Real matrix of a real-linear map on complex arrays of ``in_shape``."""
    n = int(np.prod(in_shape))
    cols = []
    for unit in (1.0, 1j):
        for i in range(n):
            e = np.zeros(n, dtype=np.complex128)
            e[i] = unit
            cols.append(realify(func(e.reshape(in_shape))))
    return np.array(cols).T


def lift_line(v_lines: np.ndarray, k: int, use_w: bool, vc: bool, wvec=None) -> np.ndarray:
    """Lift J k-space lines (J, n) to the (n-k+1) x (k J [2]) matrix, entry by entry (wvec: given
    weights in place of the first difference)."""
    J, n = v_lines.shape
    p = n - k + 1
    c = n // 2
    nblk = J * (2 if vc else 1)
    T = np.zeros((p, k * nblk), dtype=np.complex128)
    for blk in range(nblk):
        j = blk % J
        for a in range(p):
            for b in range(k):
                i = a + b
                if not use_w:
                    wi = 1.0
                elif wvec is not None:
                    wi = wvec[i]
                else:
                    wi = 1.0 - np.exp(-2j * np.pi * (i - c) / n)
                if blk < J:
                    val = v_lines[j, i]
                else:
                    val = np.conj(v_lines[j, (2 * c - i) % n])
                T[a, blk * k + b] = wi * val
    return T


def svt_loop(T, t):
    U, s, Vh = np.linalg.svd(T, full_matrices=False)
    return U @ np.diag(np.maximum(s - t, 0.0)) @ Vh


def spirit_kspace_matrix(g: np.ndarray, M: int, N: int) -> np.ndarray:
    """Complex matrix of the circular k-space SPIRiT convolution on (J, M, N)."""
    J, ks = g.shape[0], g.shape[-1]
    h = ks // 2
    n = J * M * N
    A = np.zeros((n, n), dtype=np.complex128)
    idx = lambda j, m, q: (j * M + m) * N + q
    for j in range(J):
        for m in range(M):
            for q in range(N):
                for jj in range(J):
                    for dm in range(ks):
                        for dn in range(ks):
                            A[idx(j, m, q), idx(jj, (m + dm - h) % M, (q + dn - h) % N)] += g[j, jj, dm, dn]
    return A


class BrutePI:
    """SHLR(-S/-V/-SV) on an image X of shape (J, M, N) with dense linear algebra."""

    def __init__(self, Y, mask, k_row, k_col, lam, lam1, beta, tau, vc, use_w=True,
                 hard_dc=False, g=None, d0=1.0, wvec=None):
        self.Y = np.asarray(Y, dtype=np.complex128)
        self.mask = np.asarray(mask, dtype=bool)
        J, M, N = self.Y.shape
        self.J, self.M, self.N = J, M, N
        self.kr, self.kc = k_row, k_col
        self.lam, self.lam1, self.beta, self.tau = lam, lam1, beta, tau
        self.vc, self.use_w, self.hard_dc = vc, use_w, hard_dc
        FM, FN = dft_matrix(M), dft_matrix(N)
        self.FM, self.FN = FM, FN
        shape = (J, M, N)
        self.shape = shape

        def f2(X):
            return np.einsum("ab,jbc,dc->jad", FM, X, FN)
        self.f2 = f2
        # U F^2D as a real matrix restricted to sampled entries (Eq. 2 data term)
        UF = real_matrix(lambda X: f2(X)[:, self.mask], shape)
        self.UF = UF
        # lifted row operators: X -> lift(F_N x_row_m) for each m (Eq. 2, Eq. 4)
        self.row_ops = [real_matrix(lambda X, m=m: lift_line((X[:, m, :] @ FN.T), k_row, use_w, vc, wvec), shape)
                        for m in range(M)]
        self.col_ops = [real_matrix(lambda X, q=q: lift_line((X[:, :, q] @ FM.T), k_col, use_w, vc, wvec), shape)
                        for q in range(N)]
        pr, qr = N - k_row + 1, k_row * J * (2 if vc else 1)
        pc, qc = M - k_col + 1, k_col * J * (2 if vc else 1)
        self.rshape, self.cshape = (pr, qr), (pc, qc)
        self.Zr = [np.zeros((pr, qr), complex) for _ in range(M)]
        self.Dr = [np.full((pr, qr), d0, complex) for _ in range(M)]
        self.Zc = [np.zeros((pc, qc), complex) for _ in range(N)]
        self.Dc = [np.full((pc, qc), d0, complex) for _ in range(N)]
        if lam1 > 0:
            Gk = spirit_kspace_matrix(g, M, N)
            F2 = np.kron(np.eye(J), np.kron(FM, FN))
            Gimg = F2.conj().T @ Gk @ F2
            GI = Gimg - np.eye(J * M * N)
            self.GI = real_matrix(lambda X: (GI @ X.ravel()), shape)
        else:
            self.GI = None
        self.X = np.einsum("ab,jbc,dc->jad", FM.conj().T, self.Y, FN.conj().T)   # X^0 = F^-1 Y

    def x_update(self):
        b = 0
        A = self.beta * sum(O.T @ O for O in self.row_ops + self.col_ops)
        b = self.beta * sum(O.T @ realify(Z - D / self.beta)
                            for O, Z, D in zip(self.row_ops + self.col_ops, self.Zr + self.Zc, self.Dr + self.Dc))
        if self.GI is not None:
            A = A + self.lam1 * self.GI.T @ self.GI
        ys = realify(self.Y[:, self.mask])
        if self.hard_dc:
            C = self.UF
            nc = C.shape[0]
            KKT = np.block([[A, C.T], [C, np.zeros((nc, nc))]])
            sol = np.linalg.lstsq(KKT, np.concatenate([b, ys]), rcond=None)[0]
            x = sol[:A.shape[0]]
        else:
            A = A + self.lam * self.UF.T @ self.UF
            b = b + self.lam * self.UF.T @ ys
            x = np.linalg.solve(A, b)
        self.X = complexify(x, self.shape)

    def zd_update(self):
        t = 1.0 / self.beta
        x = realify(self.X)
        for ops, Zs, Ds, shp in ((self.row_ops, self.Zr, self.Dr, self.rshape),
                                 (self.col_ops, self.Zc, self.Dc, self.cshape)):
            for i, O in enumerate(ops):
                LX = complexify(O @ x, shp)
                Zs[i] = svt_loop(LX + Ds[i] / self.beta, t)
                Ds[i] = Ds[i] + self.tau * (LX - Zs[i])

    def run(self, iters):
        for _ in range(iters):
            self.x_update()
            self.zd_update()
        return self.f2(self.X)


class BruteParam:
    """SHLR-P / SHLR-VP for ONE frequency-encode position: X_m of shape (L, J, N) (PE image)."""

    def __init__(self, Ym, mask, k_pe, k_l, lam, lam2, beta, tau, vc, d0=1.0):
        self.Ym = np.asarray(Ym, dtype=np.complex128)       # (L, J, N) PE k-space
        self.mask = np.asarray(mask, dtype=bool)            # (L, N)
        L, J, N = self.Ym.shape
        self.L, self.J, self.N = L, J, N
        self.lam, self.lam2, self.beta, self.tau = lam, lam2, beta, tau
        F = dft_matrix(N)
        self.F = F
        shape = (L, J, N)
        self.shape = shape
        msk = np.broadcast_to(self.mask[:, None, :], shape)
        self.UF = real_matrix(lambda X: (X @ F.T)[msk], shape)
        # PE-direction lifts of each echo l (Q_l, with F, W, H or H_vc)
        self.pe_ops = [real_matrix(lambda X, l=l: lift_line(X[l] @ F.T, k_pe, True, vc), shape) for l in range(L)]
        # parameter-direction lifts at each PE position n (P_n, H only)
        self.ec_ops = [real_matrix(lambda X, n=n: lift_line(X[:, :, n].T, k_l, False, False), shape)
                       for n in range(N)]
        pp, qp = N - k_pe + 1, k_pe * J * (2 if vc else 1)
        pe, qe = L - k_l + 1, k_l * J
        self.pshape, self.eshape = (pp, qp), (pe, qe)
        self.Zp = [np.zeros((pp, qp), complex) for _ in range(L)]
        self.Dp = [np.full((pp, qp), d0, complex) for _ in range(L)]
        self.Ze = [np.zeros((pe, qe), complex) for _ in range(N)]
        self.De = [np.full((pe, qe), d0, complex) for _ in range(N)]
        self.X = self.Ym @ F.conj()                          # F^-1 along PE (F^-1 = F^H, F symmetric)

    def x_update(self):
        ops = self.pe_ops + self.ec_ops
        A = self.beta * sum(O.T @ O for O in ops) + self.lam * self.UF.T @ self.UF
        b = self.beta * sum(O.T @ realify(Z - D / self.beta)
                            for O, Z, D in zip(ops, self.Zp + self.Ze, self.Dp + self.De))
        msk = np.broadcast_to(self.mask[:, None, :], self.shape)
        b = b + self.lam * self.UF.T @ realify(self.Ym[msk])
        self.X = complexify(np.linalg.solve(A, b), self.shape)

    def zd_update(self):
        x = realify(self.X)
        for ops, Zs, Ds, shp, t in ((self.pe_ops, self.Zp, self.Dp, self.pshape, 1.0 / self.beta),
                                    (self.ec_ops, self.Ze, self.De, self.eshape, self.lam2 / self.beta)):
            for i, O in enumerate(ops):
                LX = complexify(O @ x, shp)
                Zs[i] = svt_loop(LX + Ds[i] / self.beta, t)
                Ds[i] = Ds[i] + self.tau * (LX - Zs[i])

    def run(self, iters):
        for _ in range(iters):
            self.x_update()
            self.zd_update()
        return self.X @ self.F.T                              # PE k-space (L, J, N)
