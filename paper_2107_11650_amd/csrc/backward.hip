// Reverse mode of the X-update (Eq. 15 without the SPIRiT term):
//   K = (lambda U Y + beta F_m(B_row) + beta F_n(B_col)) / den,
//   den = lambda U + beta (r_row[n] + r_col[m]),  U the 0/1 sampling mask.
// Given the cotangent Kbar of K:
//   rbar = Kbar / den                    (cotangent of the right-hand side),
//   Ybar += lambda U rbar,
//   lambda_bar += Re <rbar, U (Y - K)>   (d den / d lambda = U),
// and the caller maps rbar to the line cotangents beta F^-1 rbar.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace shlr {

constexpr int DC_THREADS = 256;

template <typename R>
__global__ __launch_bounds__(DC_THREADS) void k_dc_vjp(const cplx_t<R>* __restrict__ gk,
                                                       const cplx_t<R>* __restrict__ K,
                                                       const cplx_t<R>* __restrict__ Y,
                                                       const uint8_t* __restrict__ mask,
                                                       const R* __restrict__ rr, const R* __restrict__ rc, int M,
                                                       int N, int64_t total, double lam, double beta,
                                                       cplx_t<R>* __restrict__ rbar, cplx_t<R>* __restrict__ gy,
                                                       double* __restrict__ partials) {
    using C = cplx_t<R>;
    __shared__ double red[DC_THREADS / 64];
    double part = 0;
    for (int64_t e = (int64_t)blockIdx.x * DC_THREADS + threadIdx.x; e < total; e += (int64_t)gridDim.x * DC_THREADS) {
        const int n = (int)(e % N);
        const int m = (int)((e / N) % M);
        const bool smp = mask[(int64_t)m * N + n] != 0;
        const double den = (smp ? lam : 0.0) + beta * ((double)rr[n] + (double)rc[m]);
        const C g = gk[e];
        const double br = (double)g.x / den, bi = (double)g.y / den;
        C o;
        o.x = (R)br;
        o.y = (R)bi;
        rbar[e] = o;
        if (smp) {
            C y = gy[e];
            y.x += (R)(lam * br);
            y.y += (R)(lam * bi);
            gy[e] = y;
            const C yv = Y[e], kv = K[e];
            part += br * ((double)yv.x - (double)kv.x) + bi * ((double)yv.y - (double)kv.y);
        }
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < DC_THREADS / 64; ++w) t += red[w];
        partials[blockIdx.x] = t;
    }
}

template <typename R>
__global__ void k_add(cplx_t<R>* __restrict__ a, const cplx_t<R>* __restrict__ b, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        cplx_t<R> v = a[e];
        const cplx_t<R> w = b[e];
        v.x += w.x;
        v.y += w.y;
        a[e] = v;
    }
}

template <typename R>
hipError_t launch_dc_vjp(hipStream_t st, const cplx_t<R>* gk, const cplx_t<R>* K, const cplx_t<R>* Y,
                         const uint8_t* mask, const R* rr, const R* rc, int J, int M, int N, double lam, double beta,
                         cplx_t<R>* rbar, cplx_t<R>* gy, double* partials) {
    const int64_t total = (int64_t)J * M * N;
    hipLaunchKernelGGL((k_dc_vjp<R>), dim3(DC_VJP_BLOCKS), dim3(DC_THREADS), 0, st, gk, K, Y, mask, rr, rc, M, N,
                       total, lam, beta, rbar, gy, partials);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_add(hipStream_t st, cplx_t<R>* a, const cplx_t<R>* b, int64_t n) {
    const int blocks = (int)std::min<int64_t>(2048, (n + 255) / 256);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_add<R>), dim3(blocks), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

template hipError_t launch_dc_vjp<float>(hipStream_t, const float2*, const float2*, const float2*, const uint8_t*,
                                         const float*, const float*, int, int, int, double, double, float2*, float2*,
                                         double*);
template hipError_t launch_dc_vjp<double>(hipStream_t, const double2*, const double2*, const double2*,
                                          const uint8_t*, const double*, const double*, int, int, int, double, double,
                                          double2*, double2*, double*);
template hipError_t launch_add<float>(hipStream_t, float2*, const float2*, int64_t);
template hipError_t launch_add<double>(hipStream_t, double2*, const double2*, int64_t);

}  // namespace shlr
