"""FP64 CPU oracle of the derivative of unrolled SHLR iterations.

TEST INFRASTRUCTURE ONLY (like ``shlr_oracle``): nothing in the product path
may import or call it, and it shares no code with the HIP path.

The paper gives no gradient.  What is differentiated here is the fixed
map of ``n_iter`` iterations of the parallel-imaging ADMM (Algorithm S1
order: X-update of Eq. 15, SVT of Eqs. 16-17, multiplier update of Eqs.
13-14) from the acquired k-space Y and the data-consistency weight lambda to
the k-space K after the last X-update:

    K_n = Phi_n(Y, lambda),   no normalisation of Y (the caller's scaling),
    soft data consistency, no SPIRiT term.

The map is written out in plain PyTorch complex128 CPU operations (centred
unitary FFTs, index-gather Hankel lifts, index-add adjoint lifts and a
LAPACK SVD per lifted matrix) and differentiated by reverse-mode automatic
differentiation, so the SVT derivative is the SVD route of the library
(``torch.linalg.svd``'s backward), not the Gram/eigen route of the GPU.

Gradient convention: for a real loss L = Re <gK, K_n> (sum over entries of
conj(gK) * K_n), the gradient with respect to a complex tensor Y is the
tensor gY with dL = Re <gY, dY>; this is PyTorch's convention for complex
leaves.  The forward is pinned to the NumPy oracle iterate by iterate, and
the gradient to central finite differences of the forward.
"""

from __future__ import annotations

import numpy as np
import torch

from . import shlr_oracle as O


def fftc_t(x, dim):
    """Centred unitary DFT along ``dim`` (same convention as ``shlr_oracle.fftc``)."""
    return torch.fft.fftshift(torch.fft.fft(torch.fft.ifftshift(x, dim=dim), dim=dim, norm="ortho"), dim=dim)


def ifftc_t(x, dim):
    return torch.fft.fftshift(torch.fft.ifft(torch.fft.ifftshift(x, dim=dim), dim=dim, norm="ortho"), dim=dim)


class TorchLift:
    """Torch rendering of ``shlr_oracle.LineLift`` (Eq. 2; Eq. 4 with virtual coils)."""

    def __init__(self, lift: O.LineLift):
        self.n, self.k, self.vc = lift.n, lift.k, lift.vc
        self.p = lift.p
        self.w = torch.from_numpy(lift.w())
        self.idx = torch.from_numpy(O.hankel_index(lift.n, lift.k))
        self.flip = torch.from_numpy(O.flip_index(lift.n))

    def forward(self, h):
        """(..., J, n) -> (..., p, q)."""
        blocks = [(self.w * h)[..., self.idx]]                       # (..., J, p, k)
        if self.vc:
            blocks.append((self.w * torch.conj(h[..., self.flip]))[..., self.idx])
        B = torch.cat(blocks, dim=-3).movedim(-3, -2)                 # (..., p, V*J, k)
        return B.reshape(B.shape[:-2] + (B.shape[-2] * self.k,))

    def adjoint(self, R, J):
        """Real-inner-product adjoint of :meth:`forward`: (..., p, q) -> (..., J, n)."""
        V = 2 if self.vc else 1
        Rb = R.reshape(R.shape[:-1] + (V * J, self.k)).movedim(-2, -3)   # (..., V*J, p, k)
        flat = Rb.reshape(Rb.shape[:-2] + (self.p * self.k,))
        acc = torch.zeros(Rb.shape[:-2] + (self.n,), dtype=R.dtype)
        acc = acc.index_add(-1, self.idx.reshape(-1), flat)               # anti-diagonal sums
        g = torch.conj(self.w) * acc
        out = g[..., :J, :]
        if self.vc:
            out = out + torch.conj(g[..., J:, :][..., self.flip])
        return out


def svt_t(T, t):
    """S_t of Eq. 16 through an SVD (differentiable)."""
    U, s, Vh = torch.linalg.svd(T, full_matrices=False)
    return (U * torch.clamp(s - t, min=0.0).to(U.dtype)[..., None, :]) @ Vh


def unrolled_pi(Y, lam, mask, prm: O.PIParams, n_iter: int):
    """K after ``n_iter`` iterations of Algorithm S1 (no SPIRiT, soft data consistency).

    Y: (J, M, N) complex128 tensor; lam: real scalar tensor; mask: (M, N) bool array.
    The multiplier/low-rank update of the last iteration does not reach K and
    is skipped.
    """
    if prm.lam1 > 0 or prm.hard_dc:
        raise ValueError("the derivative oracle covers soft data consistency without the SPIRiT term")
    J, M, N = Y.shape
    Lr_np, Lc_np = O.pi_lifts(M, N, prm)
    Lr, Lc = TorchLift(Lr_np), TorchLift(Lc_np)
    beta, tau = prm.beta, prm.t()
    m = torch.from_numpy(np.asarray(mask, dtype=np.float64))
    r = torch.from_numpy(Lr_np.gram_diag()[None, :] + Lc_np.gram_diag()[:, None])
    den = lam * m + beta * r
    Zr = torch.zeros((M, Lr.p, Lr_np.q(J)), dtype=torch.complex128)
    Zc = torch.zeros((N, Lc.p, Lc_np.q(J)), dtype=torch.complex128)
    Dr = torch.full_like(Zr, prm.d0)
    Dc = torch.full_like(Zc, prm.d0)
    K = None
    for it in range(n_iter):
        Br = Lr.adjoint(Zr - Dr / beta, J).permute(1, 0, 2)          # (J, M, N)
        Bc = Lc.adjoint(Zc - Dc / beta, J).permute(1, 2, 0)
        rhs = lam * m * Y + beta * fftc_t(Br, 1) + beta * fftc_t(Bc, 2)
        K = rhs / den
        if it == n_iter - 1:
            break
        Hr = ifftc_t(K, 1).permute(1, 0, 2)
        Hc = ifftc_t(K, 2).permute(2, 0, 1)
        LXr, LXc = Lr.forward(Hr), Lc.forward(Hc)
        Zr = svt_t(LXr + Dr / beta, 1.0 / beta)
        Zc = svt_t(LXc + Dc / beta, 1.0 / beta)
        Dr = Dr + tau * (LXr - Zr)
        Dc = Dc + tau * (LXc - Zc)
    return K


def unrolled_pi_vjp(Y, mask, prm: O.PIParams, n_iter: int, gK):
    """(K_n, gY, g_lambda) for the loss Re <gK, K_n>; NumPy in, NumPy out."""
    Yt = torch.tensor(np.asarray(Y, dtype=np.complex128), requires_grad=True)
    lam = torch.tensor(float(prm.lam), dtype=torch.float64, requires_grad=True)
    K = unrolled_pi(Yt, lam, mask, prm, n_iter)
    loss = (torch.conj(torch.from_numpy(np.asarray(gK, dtype=np.complex128))) * K).real.sum()
    gY, gl = torch.autograd.grad(loss, (Yt, lam))
    return K.detach().numpy(), gY.numpy(), float(gl)
