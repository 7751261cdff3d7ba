// SPIRiT term of Eq. 3 / Eq. 15 on the device (gfx950).
//
// The k-space SPIRiT operator is a circular multi-coil convolution,
//   (G K)_t(x) = sum_{s, d} g[t][s][d] K_s(x + d),
// which the centred unitary 2D DFT turns into a per-pixel J x J matrix in the
// image domain:  Gimg[t][s](r) = sum_d g[t][s][d] exp(-2 pi i (d_m r'_m / M + d_n r'_n / N)),
// r' = r - (M/2, N/2).  The X-update of Eq. 15 with lambda1 > 0 is then
//   (diag(den) + lambda1 F (Gimg - I)^H (Gimg - I) F^-1) K = rhs,
// solved by preconditioned conjugate gradients (preconditioner diag(den)).
// All reductions are two-stage with a fixed order, so runs are bitwise
// reproducible.
#include "common.h"
#include "kernels.h"

namespace shlr {

constexpr int PCG_BLOCKS = 1024;
constexpr int PCG_THREADS = 256;

// Gm[pix][t][s] = Gimg[t][s](pix) - delta_ts
template <typename R>
__global__ void k_spirit_gimg(const double2* __restrict__ g, int J, int ks, int M, int N, cplx_t<R>* __restrict__ Gm) {
    const int64_t total = (int64_t)M * N * J * J;
    const int h = ks / 2;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(e % J);
        const int t = (int)((e / J) % J);
        const int64_t pix = e / ((int64_t)J * J);
        const int rm = (int)(pix / N) - M / 2, rn = (int)(pix % N) - N / 2;
        double ar = 0, ai = 0;
        for (int dm = 0; dm < ks; ++dm) {
            for (int dn = 0; dn < ks; ++dn) {
                const double2 gv = g[(((int64_t)t * J + s) * ks + dm) * ks + dn];
                // phase exp(-2 pi i (dm' rm / M + dn' rn / N)), reduced mod 1 in exact integer arithmetic
                const int64_t am = ((int64_t)(dm - h) * rm) % M;
                const int64_t an = ((int64_t)(dn - h) * rn) % N;
                const double frac = (double)am / M + (double)an / N;
                double sn, cs;
                sincospi(-2.0 * frac, &sn, &cs);
                ar += gv.x * cs - gv.y * sn;
                ai += gv.x * sn + gv.y * cs;
            }
        }
        if (s == t) ar -= 1.0;
        Gm[e] = cmk<cplx_t<R>>(ar, ai);
    }
}

// A_pix[a][b] = sum_t conj(Gm[pix][t][a]) Gm[pix][t][b], pix = m N + n, stored at A[n][b][m][a]: the
// operator of image column n is one block, and within it entry b of the rows of all (m, a) pairs is
// contiguous in m J + a, the order in which one thread per (m, a) reads it
template <typename R>
__global__ void k_spirit_gram(const cplx_t<R>* __restrict__ Gm, int J, int M, int N, cplx_t<R>* __restrict__ A) {
    const int64_t npix = (int64_t)M * N;
    const int64_t total = npix * J * J;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(e % J);
        const int a = (int)((e / J) % J);
        const int64_t pix = e / ((int64_t)J * J);
        const cplx_t<R>* G = Gm + pix * J * J;
        double sr = 0, si = 0;
        for (int t = 0; t < J; ++t) {
            const cplx_t<R> x = G[t * J + a], y = G[t * J + b];
            sr += (double)x.x * y.x + (double)x.y * y.y;
            si += (double)x.x * y.y - (double)x.y * y.x;
        }
        const int m = (int)(pix / N), n = (int)(pix - (int64_t)m * N);
        A[(((int64_t)n * J + b) * M + m) * J + a] = cmk<cplx_t<R>>(sr, si);
    }
}

// y_a(r) = sum_b A_r[a][b] x_b(r), images in layout [J][npix], A in the layout of k_spirit_gram
template <typename R>
__global__ void k_spirit_matvec(const cplx_t<R>* __restrict__ A, const cplx_t<R>* __restrict__ x,
                                cplx_t<R>* __restrict__ y, int J, int M, int N) {
    using C = cplx_t<R>;
    const int64_t npix = (int64_t)M * N;
    for (int64_t pix = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pix < npix;
         pix += (int64_t)gridDim.x * blockDim.x) {
        const int pm = (int)(pix / N), pn = (int)(pix - (int64_t)pm * N);
        const C* Ap = A + ((int64_t)pn * J * M + pm) * J;   // + (b M + 0) J + a
        for (int a = 0; a < J; ++a) {
            R sr = 0, si = 0;
            for (int b = 0; b < J; ++b) {
                const C m = Ap[(int64_t)b * M * J + a], v = x[(int64_t)b * npix + pix];
                sr += m.x * v.x - m.y * v.y;
                si += m.x * v.y + m.y * v.x;
            }
            y[(int64_t)a * npix + pix] = cmk<C>(sr, si);
        }
    }
}

template <typename R>
__device__ inline R den_at(int64_t e, int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off,
                           R lam, R beta) {
    const int64_t pix = e % ((int64_t)M * N);
    const int m = (int)(pix / N), n = (int)(pix % N);
    return (mask[pix] ? lam : (R)0) + beta * (rtab[rr_off + n] + rtab[rc_off + m]);
}

__device__ inline void block_partial(double v, double* partials) {
    __shared__ double red[PCG_THREADS / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < PCG_THREADS / 64; ++w) t += red[w];
        partials[blockIdx.x] = t;
    }
}

// Ap = den * p + lam1 * t ; partial Re<p, Ap>
template <typename R>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_apply(const cplx_t<R>* __restrict__ p,
                                                           const cplx_t<R>* __restrict__ t, cplx_t<R>* __restrict__ Ap,
                                                           int64_t count, int M, int N, const uint8_t* mask,
                                                           const R* rtab, int64_t rr_off, int64_t rc_off, R lam,
                                                           R beta, R lam1, double* partials) {
    double acc = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const R d = den_at(e, M, N, mask, rtab, rr_off, rc_off, lam, beta);
        const cplx_t<R> pv = p[e], tv = t[e];
        const cplx_t<R> a = cmk<cplx_t<R>>(d * pv.x + lam1 * tv.x, d * pv.y + lam1 * tv.y);
        Ap[e] = a;
        acc += (double)pv.x * a.x + (double)pv.y * a.y;
    }
    block_partial(acc, partials);
}

// r = b - Ax; z = r / den; p = z; partial Re<r, z>
template <typename R>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_init(const cplx_t<R>* __restrict__ b,
                                                          const cplx_t<R>* __restrict__ Ax, cplx_t<R>* __restrict__ r,
                                                          cplx_t<R>* __restrict__ z, cplx_t<R>* __restrict__ p,
                                                          int64_t count, int M, int N, const uint8_t* mask,
                                                          const R* rtab, int64_t rr_off, int64_t rc_off, R lam,
                                                          R beta, double* partials) {
    double acc = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const R d = den_at(e, M, N, mask, rtab, rr_off, rc_off, lam, beta);
        const cplx_t<R> rv = csub(b[e], Ax[e]);
        const cplx_t<R> zv = cscale(rv, (R)1 / d);
        r[e] = rv;
        z[e] = zv;
        p[e] = zv;
        acc += (double)rv.x * zv.x + (double)rv.y * zv.y;
    }
    block_partial(acc, partials);
}

// scal: [0] rz, [1] pAp, [2] alpha, [3] beta_cg
// mode 0: rz = sum(partials); mode 1: pAp = sum, alpha = rz / pAp; mode 2: rz_new = sum, beta_cg = rz_new / rz, rz = rz_new
__global__ void k_pcg_scalar(const double* __restrict__ partials, int n, double* scal, int mode) {
    __shared__ double red[PCG_THREADS];
    double v = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += partials[i];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        if (mode == 0) {
            scal[0] = t;
            scal[4] = t;   // first slot of the alternating rz pair of the fused loop
        } else if (mode == 1) {
            scal[1] = t;
            scal[2] = (t != 0.0 && scal[0] != 0.0) ? scal[0] / t : 0.0;
        } else {
            scal[3] = scal[0] != 0.0 ? t / scal[0] : 0.0;
            scal[0] = t;
        }
    }
}

// x += alpha p; r -= alpha Ap; z = r / den; partial Re<r, z>
template <typename R>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_update(cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ r,
                                                            cplx_t<R>* __restrict__ z, const cplx_t<R>* __restrict__ p,
                                                            const cplx_t<R>* __restrict__ Ap, int64_t count, int M,
                                                            int N, const uint8_t* mask, const R* rtab, int64_t rr_off,
                                                            int64_t rc_off, R lam, R beta, const double* scal,
                                                            double* partials) {
    const R alpha = (R)scal[2];
    double acc = 0;
#pragma unroll 4
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const R d = den_at(e, M, N, mask, rtab, rr_off, rc_off, lam, beta);
        const cplx_t<R> pv = p[e], av = Ap[e];
        cplx_t<R> xv = x[e], rv = r[e];
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        rv.x -= alpha * av.x;
        rv.y -= alpha * av.y;
        const cplx_t<R> zv = cscale(rv, (R)1 / d);
        x[e] = xv;
        r[e] = rv;
        z[e] = zv;
        acc += (double)rv.x * zv.x + (double)rv.y * zv.y;
    }
    block_partial(acc, partials);
}

// p = z + beta_cg p
template <typename R>
__global__ void k_pcg_dir(cplx_t<R>* __restrict__ p, const cplx_t<R>* __restrict__ z, int64_t count,
                          const double* scal) {
    const R bc = (R)scal[3];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const cplx_t<R> pv = p[e], zv = z[e];
        p[e] = cmk<cplx_t<R>>(zv.x + bc * pv.x, zv.y + bc * pv.y);
    }
}

static inline int ew_grid(int64_t count) {
    int64_t b = (count + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename R>
hipError_t launch_spirit_build(hipStream_t st, const double2* g_dev, int J, int ks, int M, int N, cplx_t<R>* Gtmp,
                               cplx_t<R>* A) {
    const int64_t tot = (int64_t)M * N * J * J;
    hipLaunchKernelGGL((k_spirit_gimg<R>), dim3(ew_grid(tot)), dim3(256), 0, st, g_dev, J, ks, M, N, Gtmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spirit_gram<R>), dim3(ew_grid(tot)), dim3(256), 0, st, Gtmp, J, M, N, A);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_spirit_matvec(hipStream_t st, const cplx_t<R>* A, const cplx_t<R>* x, cplx_t<R>* y, int J, int M,
                                int N) {
    hipLaunchKernelGGL((k_spirit_matvec<R>), dim3(ew_grid((int64_t)M * N)), dim3(256), 0, st, A, x, y, J, M, N);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pcg_apply(hipStream_t st, const cplx_t<R>* p, const cplx_t<R>* t, cplx_t<R>* Ap, int64_t count,
                            int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off,
                            double lam, double beta, double lam1, double* partials) {
    hipLaunchKernelGGL((k_pcg_apply<R>), dim3(PCG_BLOCKS), dim3(PCG_THREADS), 0, st, p, t, Ap, count, M, N, mask, rtab,
                       rr_off, rc_off, (R)lam, (R)beta, (R)lam1, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pcg_init(hipStream_t st, const cplx_t<R>* b, const cplx_t<R>* Ax, cplx_t<R>* r, cplx_t<R>* z,
                           cplx_t<R>* p, int64_t count, int M, int N, const uint8_t* mask, const R* rtab,
                           int64_t rr_off, int64_t rc_off, double lam, double beta, double* partials) {
    hipLaunchKernelGGL((k_pcg_init<R>), dim3(PCG_BLOCKS), dim3(PCG_THREADS), 0, st, b, Ax, r, z, p, count, M, N, mask,
                       rtab, rr_off, rc_off, (R)lam, (R)beta, partials);
    return hipGetLastError();
}

hipError_t launch_pcg_scalar(hipStream_t st, const double* partials, int n_partials, double* scal, int mode) {
    hipLaunchKernelGGL(k_pcg_scalar, dim3(1), dim3(PCG_THREADS), 0, st, partials, n_partials, scal, mode);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pcg_update(hipStream_t st, cplx_t<R>* x, cplx_t<R>* r, cplx_t<R>* z, const cplx_t<R>* p,
                             const cplx_t<R>* Ap, int64_t count, int M, int N, const uint8_t* mask, const R* rtab,
                             int64_t rr_off, int64_t rc_off, double lam, double beta, const double* scal,
                             double* partials) {
    hipLaunchKernelGGL((k_pcg_update<R>), dim3(PCG_BLOCKS), dim3(PCG_THREADS), 0, st, x, r, z, p, Ap, count, M, N,
                       mask, rtab, rr_off, rc_off, (R)lam, (R)beta, scal, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pcg_dir(hipStream_t st, cplx_t<R>* p, const cplx_t<R>* z, int64_t count, const double* scal) {
    hipLaunchKernelGGL((k_pcg_dir<R>), dim3(ew_grid(count)), dim3(256), 0, st, p, z, count, scal);
    return hipGetLastError();
}

#define SPIRIT_INST(R)                                                                                                \
    template hipError_t launch_spirit_build<R>(hipStream_t, const double2*, int, int, int, int, cplx_t<R>*,           \
                                               cplx_t<R>*);                                                           \
    template hipError_t launch_spirit_matvec<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, cplx_t<R>*, int, int, \
                                                int);                                                                 \
    template hipError_t launch_pcg_apply<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, cplx_t<R>*, int64_t, int, \
                                            int, const uint8_t*, const R*, int64_t, int64_t, double, double, double,  \
                                            double*);                                                                 \
    template hipError_t launch_pcg_init<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, cplx_t<R>*, cplx_t<R>*,   \
                                           cplx_t<R>*, int64_t, int, int, const uint8_t*, const R*, int64_t, int64_t, \
                                           double, double, double*);                                                  \
    template hipError_t launch_pcg_update<R>(hipStream_t, cplx_t<R>*, cplx_t<R>*, cplx_t<R>*, const cplx_t<R>*,       \
                                             const cplx_t<R>*, int64_t, int, int, const uint8_t*, const R*, int64_t,  \
                                             int64_t, double, double, const double*, double*);                        \
    template hipError_t launch_pcg_dir<R>(hipStream_t, cplx_t<R>*, const cplx_t<R>*, int64_t, const double*);       \

SPIRIT_INST(float)
SPIRIT_INST(double)

}  // namespace shlr
