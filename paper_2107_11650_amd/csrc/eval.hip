// Evaluation step after a reconstruction: SSOS coil combination, RLNE (Eq. S10), MSSIM (Eq. S11)
// and the pixel-wise mono-exponential T2 fit of the parameter-imaging experiment.
//
// All of it is HBM- or latency-light work on M x N images: one pass per quantity, sums kept in FP64
// and reduced in a fixed order (per-block partials, then one block), so results repeat bit for bit.
#include <float.h>
#include <math.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace shlr {

constexpr int EV_THREADS = 256;

// out[i][p] = sqrt(sum_j |x[i][j][p]|^2) for images i of J coils, MN pixels each
template <typename R>
__global__ __launch_bounds__(EV_THREADS) void k_ssos(const cplx_t<R>* __restrict__ x, R* __restrict__ out, int J,
                                                     int64_t MN, int64_t total) {
    for (int64_t e = blockIdx.x * (int64_t)EV_THREADS + threadIdx.x; e < total; e += (int64_t)gridDim.x * EV_THREADS) {
        const int64_t i = e / MN, p = e - i * MN;
        const cplx_t<R>* xi = x + i * J * MN + p;
        double s = 0;
        for (int j = 0; j < J; ++j) {
            const cplx_t<R> v = xi[(int64_t)j * MN];
            s += (double)v.x * v.x + (double)v.y * v.y;
        }
        out[e] = (R)sqrt(s);
    }
}

// fixed-order sum of a block's values (all threads call; the total is valid in thread 0)
__device__ inline double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = EV_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double t = sh[0];
    __syncthreads();
    return t;
}

// per block: sum (a - b)^2 and sum a^2 over the pixels of the ROI (all pixels when roi is null)
template <typename R>
__global__ __launch_bounds__(EV_THREADS) void k_rlne_partials(const R* __restrict__ a, const R* __restrict__ b,
                                                              const uint8_t* __restrict__ roi, int64_t count,
                                                              double* __restrict__ partials) {
    __shared__ double sh[EV_THREADS];
    double d = 0, n = 0;
    for (int64_t e = blockIdx.x * (int64_t)EV_THREADS + threadIdx.x; e < count; e += (int64_t)gridDim.x * EV_THREADS) {
        if (roi && !roi[e]) continue;
        const double x = a[e], y = b[e];
        d += (x - y) * (x - y);
        n += x * x;
    }
    d = block_sum(d, sh);
    n = block_sum(n, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = d;
        partials[2 * blockIdx.x + 1] = n;
    }
}

// MSSIM: one block per 16 x 16 tile of window positions.  The 26 x 26 input patch of both images
// sits in LDS; the separable Gaussian (g g^T, g of unit sum) filters the five moments a, b, a^2,
// b^2, ab along rows, then along columns; SSIM of each window; one fixed-order sum per block.
constexpr int SS_T = 16;
constexpr int SS_W = 11;
constexpr int SS_P = SS_T + SS_W - 1;   // 26
struct GaussTaps {
    double g[SS_W];
};

template <typename R>
__global__ __launch_bounds__(EV_THREADS) void k_mssim_partials(const R* __restrict__ a, const R* __restrict__ b, int M,
                                                               int N, GaussTaps w, double c1, double c2,
                                                               double* __restrict__ partials) {
    __shared__ double pa[SS_P][SS_P + 1], pb[SS_P][SS_P + 1];
    __shared__ double h[5][SS_P][SS_T + 1];
    __shared__ double sh[EV_THREADS];
    const int RM = M - SS_W + 1, RN = N - SS_W + 1;   // window positions
    const int i0 = blockIdx.y * SS_T, j0 = blockIdx.x * SS_T;
    const int tid = threadIdx.x;
    for (int e = tid; e < SS_P * SS_P; e += EV_THREADS) {
        const int r = e / SS_P, c = e - r * SS_P;
        const int gi = i0 + r, gj = j0 + c;
        const bool in = gi < M && gj < N;
        pa[r][c] = in ? (double)a[(int64_t)gi * N + gj] : 0.0;
        pb[r][c] = in ? (double)b[(int64_t)gi * N + gj] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < SS_P * SS_T; e += EV_THREADS) {
        const int r = e / SS_T, c = e - r * SS_T;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
#pragma unroll
        for (int k = 0; k < SS_W; ++k) {
            const double x = pa[r][c + k], y = pb[r][c + k], g = w.g[k];
            s0 = fma(g, x, s0);
            s1 = fma(g, y, s1);
            s2 = fma(g, x * x, s2);
            s3 = fma(g, y * y, s3);
            s4 = fma(g, x * y, s4);
        }
        h[0][r][c] = s0;
        h[1][r][c] = s1;
        h[2][r][c] = s2;
        h[3][r][c] = s3;
        h[4][r][c] = s4;
    }
    __syncthreads();
    double acc = 0;
    {
        const int r = tid / SS_T, c = tid - (tid / SS_T) * SS_T;
        if (i0 + r < RM && j0 + c < RN) {
            double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < SS_W; ++k) {
                const double g = w.g[k];
#pragma unroll
                for (int q = 0; q < 5; ++q) m[q] = fma(g, h[q][r + k][c], m[q]);
            }
            const double mu_a = m[0], mu_b = m[1];
            const double va = m[2] - mu_a * mu_a, vb = m[3] - mu_b * mu_b, cab = m[4] - mu_a * mu_b;
            acc = ((2 * mu_a * mu_b + c1) * (2 * cab + c2)) / ((mu_a * mu_a + mu_b * mu_b + c1) * (va + vb + c2));
        }
    }
    acc = block_sum(acc, sh);
    if (tid == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// per block: the largest value of a real image
template <typename R>
__global__ __launch_bounds__(EV_THREADS) void k_max_partials(const R* __restrict__ a, int64_t count,
                                                             double* __restrict__ partials) {
    __shared__ double sh[EV_THREADS];
    double m = -DBL_MAX;
    for (int64_t e = blockIdx.x * (int64_t)EV_THREADS + threadIdx.x; e < count; e += (int64_t)gridDim.x * EV_THREADS)
        m = fmax(m, (double)a[e]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = EV_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// fixed-order sum (mode 0) or max (mode 1) of n partials into out[0]; one block
__global__ __launch_bounds__(EV_THREADS) void k_reduce_partials(const double* __restrict__ partials, int n,
                                                                int stride, int mode, double* __restrict__ out) {
    __shared__ double sh[EV_THREADS];
    double v = mode ? -DBL_MAX : 0.0;
    for (int i = threadIdx.x; i < n; i += EV_THREADS) v = mode ? fmax(v, partials[(int64_t)i * stride])
                                                               : v + partials[(int64_t)i * stride];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = EV_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = mode ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                                         : sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Pixel-wise fit of S(TE) = rho exp(-r TE), T2 = 1 / r, in FP64, one thread per pixel:
// log-linear least-squares start, then Levenberg-Marquardt on the two parameters (2 x 2 normal
// equations with diagonal damping).  Pixels whose first echo is below the ROI threshold, fits that
// fail and T2 outside [t2_min, t2_max] give 0 (and roi = 0).
template <typename R>
__global__ __launch_bounds__(EV_THREADS) void k_t2_fit(const R* __restrict__ img, int64_t npix, TeList te,
                                                       const double* __restrict__ maxv, double roi_frac,
                                                       double t2_min, double t2_max, R* __restrict__ t2_out,
                                                       R* __restrict__ rho_out, uint8_t* __restrict__ roi_out) {
    const int64_t p = blockIdx.x * (int64_t)EV_THREADS + threadIdx.x;
    if (p >= npix) return;
    const int L = te.L;
    double s[T2_MAX_ECHOES];
    for (int l = 0; l < L; ++l) s[l] = (double)img[(int64_t)l * npix + p];
    double T2 = 0, rho = 0;
    bool ok = s[0] >= roi_frac * maxv[0];
    if (ok) {
        // log-linear start over the positive samples: ln s = c0 - r TE
        double n = 0, sx = 0, sy = 0, sxx = 0, sxy = 0;
        for (int l = 0; l < L; ++l) {
            if (!(s[l] > 0)) continue;
            const double x = -te.te[l], y = log(s[l]);
            n += 1;
            sx += x;
            sy += y;
            sxx += x * x;
            sxy += x * y;
        }
        const double det = n * sxx - sx * sx;
        ok = n >= 2 && det > 0;
        double r = ok ? (n * sxy - sx * sy) / det : 0.0;
        double a = ok ? exp((sy - r * sx) / n) : 0.0;
        r = fmax(r, 1e-6);
        auto cost_at = [&](double aa, double rr) {
            double c = 0;
            for (int l = 0; l < L; ++l) {
                const double f = aa * exp(-rr * te.te[l]) - s[l];
                c = fma(f, f, c);
            }
            return c;
        };
        double cost = ok ? cost_at(a, r) : 0.0;
        double mu = 1e-3;
        for (int it = 0; ok && it < 200; ++it) {
            double A00 = 0, A01 = 0, A11 = 0, g0 = 0, g1 = 0;
            for (int l = 0; l < L; ++l) {
                const double e = exp(-r * te.te[l]);
                const double f = a * e - s[l];
                const double j0 = e, j1 = -a * te.te[l] * e;
                A00 = fma(j0, j0, A00);
                A01 = fma(j0, j1, A01);
                A11 = fma(j1, j1, A11);
                g0 = fma(j0, f, g0);
                g1 = fma(j1, f, g1);
            }
            bool moved = false;
            for (int tries = 0; tries < 30; ++tries) {
                const double B00 = A00 * (1 + mu), B11 = A11 * (1 + mu);
                const double dt = B00 * B11 - A01 * A01;
                if (!(dt > 0)) {
                    mu *= 4;
                    continue;
                }
                const double d0 = -(B11 * g0 - A01 * g1) / dt, d1 = -(B00 * g1 - A01 * g0) / dt;
                const double an = a + d0, rn = r + d1;
                const double cn = cost_at(an, rn);
                if (cn < cost) {
                    const double step = fabs(d0) / fmax(fabs(a), 1e-300) + fabs(d1) / fmax(fabs(r), 1e-300);
                    a = an;
                    r = rn;
                    cost = cn;
                    mu = fmax(mu / 3, 1e-12);
                    moved = step > 1e-15;
                    break;
                }
                mu *= 4;
            }
            if (!moved) break;
        }
        ok = ok && isfinite(a) && isfinite(r) && r > 0;
        if (ok) {
            T2 = 1.0 / r;
            rho = a;
            ok = T2 >= t2_min && T2 <= t2_max;
        }
    }
    t2_out[p] = ok ? (R)T2 : (R)0;
    if (rho_out) rho_out[p] = ok ? (R)rho : (R)0;
    if (roi_out) roi_out[p] = ok ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static int ev_grid(int64_t count, int cap) {
    int64_t b = (count + EV_THREADS - 1) / EV_THREADS;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <typename R>
hipError_t launch_ssos(hipStream_t st, const cplx_t<R>* x, R* out, int n_img, int J, int64_t MN) {
    const int64_t total = (int64_t)n_img * MN;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ssos<R>), dim3(ev_grid(total, 8192)), dim3(EV_THREADS), 0, st, x, out, J, MN, total);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rlne(hipStream_t st, const R* a, const R* b, const uint8_t* roi, int64_t count, double* work,
                       int* n_partials) {
    const int nb = ev_grid(count, EVAL_MAX_PARTIALS / 2);
    *n_partials = nb;
    hipLaunchKernelGGL((k_rlne_partials<R>), dim3(nb), dim3(EV_THREADS), 0, st, a, b, roi, count, work);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_mssim(hipStream_t st, const R* a, const R* b, int M, int N, double c1, double c2, double sigma,
                        double* work, int* n_partials) {
    GaussTaps w;
    double tot = 0;
    for (int k = 0; k < SS_W; ++k) {
        const double t = k - SS_W / 2;
        w.g[k] = exp(-t * t / (2 * sigma * sigma));
        tot += w.g[k];
    }
    for (int k = 0; k < SS_W; ++k) w.g[k] /= tot;
    const int RM = M - SS_W + 1, RN = N - SS_W + 1;
    const dim3 grid((RN + SS_T - 1) / SS_T, (RM + SS_T - 1) / SS_T);
    if ((int64_t)grid.x * grid.y > EVAL_MAX_PARTIALS) return hipErrorInvalidValue;
    *n_partials = grid.x * grid.y;
    hipLaunchKernelGGL((k_mssim_partials<R>), grid, dim3(EV_THREADS), 0, st, a, b, M, N, w, c1, c2, work);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(hipStream_t st, const double* partials, int n, int stride, int mode, double* out) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(EV_THREADS), 0, st, partials, n, stride, mode, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_max_real(hipStream_t st, const R* a, int64_t count, double* work, double* out) {
    const int nb = ev_grid(count, EVAL_MAX_PARTIALS);
    hipLaunchKernelGGL((k_max_partials<R>), dim3(nb), dim3(EV_THREADS), 0, st, a, count, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(st, work, nb, 1, 1, out);
}

template <typename R>
hipError_t launch_t2_fit(hipStream_t st, const R* img, int64_t npix, const TeList& te, double roi_frac, double t2_min,
                         double t2_max, R* t2, R* rho, uint8_t* roi, double* work) {
    if (npix <= 0) return hipSuccess;
    // the largest first-echo value, then the fit (the ROI threshold read on the device)
    const int nb = ev_grid(npix, EVAL_MAX_PARTIALS - 1);
    hipLaunchKernelGGL((k_max_partials<R>), dim3(nb), dim3(EV_THREADS), 0, st, img, npix, work + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_reduce_partials(st, work + 1, nb, 1, 1, work);
    if (e != hipSuccess) return e;
    const int fb = (int)((npix + EV_THREADS - 1) / EV_THREADS);
    hipLaunchKernelGGL((k_t2_fit<R>), dim3(fb), dim3(EV_THREADS), 0, st, img, npix, te, (const double*)work,
                       roi_frac, t2_min, t2_max, t2, rho, roi);
    return hipGetLastError();
}

#define SHLR_EVAL_INST(R)                                                                                        \
    template hipError_t launch_ssos<R>(hipStream_t, const cplx_t<R>*, R*, int, int, int64_t);                    \
    template hipError_t launch_rlne<R>(hipStream_t, const R*, const R*, const uint8_t*, int64_t, double*, int*); \
    template hipError_t launch_mssim<R>(hipStream_t, const R*, const R*, int, int, double, double, double,       \
                                        double*, int*);                                                          \
    template hipError_t launch_t2_fit<R>(hipStream_t, const R*, int64_t, const TeList&, double, double, double,  \
                                         R*, R*, uint8_t*, double*);                                             \
    template hipError_t launch_max_real<R>(hipStream_t, const R*, int64_t, double*, double*);
SHLR_EVAL_INST(float)
SHLR_EVAL_INST(double)

}  // namespace shlr
