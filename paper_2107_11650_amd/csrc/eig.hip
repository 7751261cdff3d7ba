// Batched FP64 Hermitian eigen-solver that turns a Gram matrix into the
// singular-value-threshold factor of Eq. 16:
//   G = A^H A = V Lambda V^H,   sigma_i = sqrt(lambda_i),
//   f_i = max(1 - thr / sigma_i, 0),   S = V diag(f) V^H,
// so that A S = U max(Sigma - thr, 0) V^H (the SVT of A).
// Only eigenpairs with lambda_i > thr^2 contribute, and only those are computed.
//
// One workgroup per matrix, all arithmetic in FP64:
//  1. Householder reduction to tridiagonal form with Hermitian reflectors
//     P = I - u u^H / h (the matrix lives in the per-slot scratch in HBM/L2);
//  2. a diagonal unitary makes the off-diagonal real and non-negative;
//  3. Sturm-sequence bisection for every eigenvalue above thr^2, in parallel;
//  4. inverse iteration (tridiagonal LU with partial pivoting) per eigenvalue,
//     eigenvalues closer than ortol are grouped and re-orthogonalised (MGS);
//  5. back-transformation through the reflectors, scaling by sqrt(f), and
//     S = X X^H written in the working precision (row-major, ld = s).
#include <float.h>

#include "common.h"

namespace shlr {

constexpr int EIG_THREADS = 256;

__device__ inline double block_sum(double v, double* red) {
    // all threads must call; returns the total to every thread
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0;
    for (int w = 0; w < EIG_THREADS / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

__device__ inline double block_max(double v, double* red) {
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = red[0];
    for (int w = 1; w < EIG_THREADS / 64; ++w) t = fmax(t, red[w]);
    __syncthreads();
    return t;
}

// number of eigenvalues of the symmetric tridiagonal (d, e2 = e^2) below x
__device__ inline int sturm_count(const double* d, const double* e2, int s, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    for (int i = 1; i < s; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// deterministic start vector entry in [-1, 1]
__device__ inline double start_entry(int i, int k) {
    uint32_t x = (uint32_t)(i * 2654435761u) ^ (uint32_t)(k * 40503u + 0x9e3779b9u);
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return ((double)(x & 0xffffff) / (double)0xffffff) * 2.0 - 1.0;
}

template <typename OC>
__global__ __launch_bounds__(EIG_THREADS) void k_heig_svt(const LRDesc* __restrict__ descs, int m0,
                                                          double2* __restrict__ Gs, int64_t g_stride,
                                                          OC* __restrict__ Ss, int64_t s_stride,
                                                          double* __restrict__ scr, int64_t scr_stride,
                                                          int32_t* __restrict__ ranks, double ortol_rel,
                                                          uint32_t* __restrict__ flags) {
    __shared__ double red[EIG_THREADS / 64];
    __shared__ double2 uvec[512];
    __shared__ double2 pvec[512];
    __shared__ double sh[8];
    __shared__ double sdd[512];
    __shared__ double se2[512];
    const LRDesc dsc = descs[m0 + blockIdx.x];
    const int s = lr_s(dsc);
    const double thr = dsc.thr;
    const int tid = threadIdx.x;
    double2* A = Gs + (int64_t)blockIdx.x * g_stride;   // column-major, ld = s
    OC* S = Ss + (int64_t)blockIdx.x * s_stride;
    double* base = scr + (int64_t)blockIdx.x * scr_stride;
    double* hv = base;                 // s
    double* dd = hv + s;               // s
    double* ee = dd + s;               // s
    double* e2 = ee + s;               // s
    double* dre = e2 + s;              // s   phase re
    double* dim_ = dre + s;            // s   phase im
    double* lam = dim_ + s;            // s
    double* ecr = lam + s;             // s   complex sub-diagonal re
    double* eci = ecr + s;             // s   complex sub-diagonal im
    double* W = base + 16 * s + 64;    // s*s interleaved [i*s + k]
    double* LU = W + (int64_t)s * s;   // 5*s*s interleaved (du1, du2, lmul, u0, x)
    double2* X = reinterpret_cast<double2*>(LU);  // s*s complex, reused after inverse iteration

    // ---- 1. tridiagonalisation -------------------------------------------
    for (int i = 0; i + 1 < s; ++i) {
        const int ni = s - i - 1;
        double part = 0;
        for (int t = tid; t < ni; t += EIG_THREADS) {
            double2 v = A[(int64_t)i * s + i + 1 + t];
            uvec[t] = v;
            if (t > 0) part += cabs2(v);
        }
        const double tail = block_sum(part, red);  // has barriers
        const double2 alpha = uvec[0];
        if (tid == 0) dd[i] = A[(int64_t)i * s + i].x;
        if (!(tail > 0.0)) {
            if (tid == 0) { ecr[i] = alpha.x; eci[i] = alpha.y; hv[i] = 0.0; }
            __syncthreads();
            continue;
        }
        const double aabs = sqrt(cabs2(alpha));
        const double xn = sqrt(aabs * aabs + tail);
        double2 ph = aabs > 0 ? make_double2(alpha.x / aabs, alpha.y / aabs) : make_double2(1.0, 0.0);
        const double hh = xn * xn + aabs * xn;
        __syncthreads();
        if (tid == 0) {
            uvec[0] = make_double2(alpha.x + ph.x * xn, alpha.y + ph.y * xn);
            ecr[i] = -ph.x * xn;
            eci[i] = -ph.y * xn;
            hv[i] = hh;
        }
        __syncthreads();
        // p = A22 u / h
        for (int r = tid; r < ni; r += EIG_THREADS) {
            double ar = 0, ai = 0;
            const double2* col = A + (int64_t)(i + 1) * s + i + 1 + r;
            for (int c = 0; c < ni; ++c) {
                const double2 a = col[(int64_t)c * s];
                const double2 u = uvec[c];
                ar += a.x * u.x - a.y * u.y;
                ai += a.x * u.y + a.y * u.x;
            }
            pvec[r] = make_double2(ar / hh, ai / hh);
        }
        __syncthreads();
        // K = u^H p / (2h) (real)
        double kp = 0;
        for (int t = tid; t < ni; t += EIG_THREADS) kp += uvec[t].x * pvec[t].x + uvec[t].y * pvec[t].y;
        const double Kc = block_sum(kp, red) / (2.0 * hh);
        for (int t = tid; t < ni; t += EIG_THREADS) {
            pvec[t].x -= Kc * uvec[t].x;
            pvec[t].y -= Kc * uvec[t].y;
        }
        __syncthreads();
        // A22 -= q u^H + u q^H ; store u in column i below the diagonal
        for (int r = tid; r < ni; r += EIG_THREADS) {
            const double2 qr = pvec[r], ur = uvec[r];
            double2* col = A + (int64_t)(i + 1) * s + i + 1 + r;
            for (int c = 0; c < ni; ++c) {
                const double2 uc = uvec[c], qc = pvec[c];
                double2 a = col[(int64_t)c * s];
                // q_r conj(u_c) + u_r conj(q_c)
                a.x -= qr.x * uc.x + qr.y * uc.y + ur.x * qc.x + ur.y * qc.y;
                a.y -= qr.y * uc.x - qr.x * uc.y + ur.y * qc.x - ur.x * qc.y;
                col[(int64_t)c * s] = a;
            }
            A[(int64_t)i * s + i + 1 + r] = ur;
        }
        __syncthreads();
    }
    if (tid == 0) dd[s - 1] = A[(int64_t)(s - 1) * s + s - 1].x;
    __syncthreads();

    // ---- 2. real tridiagonal via a diagonal unitary --------------------------
    if (tid == 0) {
        double pr = 1.0, pi = 0.0;
        dre[0] = 1.0;
        dim_[0] = 0.0;
        for (int i = 0; i + 1 < s; ++i) {
            const double er = ecr[i], ei = eci[i];
            const double m = sqrt(er * er + ei * ei);
            ee[i] = m;
            e2[i] = m * m;
            if (m > 0) {
                const double ur = er / m, ui = ei / m;
                const double nr = pr * ur - pi * ui, ni2 = pr * ui + pi * ur;
                pr = nr;
                pi = ni2;
            }
            dre[i + 1] = pr;
            dim_[i + 1] = pi;
        }
        // Gershgorin bounds and scale
        double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0;
        for (int i = 0; i < s; ++i) {
            const double off = (i > 0 ? ee[i - 1] : 0.0) + (i + 1 < s ? ee[i] : 0.0);
            gl = fmin(gl, dd[i] - off);
            gu = fmax(gu, dd[i] + off);
            if (i + 1 < s) emax2 = fmax(emax2, e2[i]);
        }
        const double tnorm = fmax(fabs(gl), fabs(gu));
        sh[0] = gl;
        sh[1] = gu;
        sh[2] = tnorm;
        sh[3] = DBL_MIN * fmax(1.0, emax2) * 4.0 + DBL_MIN;
    }
    __syncthreads();
    for (int t = tid; t < s; t += EIG_THREADS) {
        sdd[t] = dd[t];
        se2[t] = (t + 1 < s) ? e2[t] : 0.0;
    }
    __syncthreads();
    const double gl = sh[0], gu = sh[1], tnorm = sh[2], pivmin = sh[3];
    (void)gl;
    bool bad = !(tnorm < DBL_MAX);  // NaN or Inf in the Gram matrix
    const double t2 = thr * thr;

    // ---- 3. eigenvalues above thr^2 ------------------------------------------
    int nabove = 0;
    if (!bad) nabove = s - sturm_count(sdd, se2, s, t2, pivmin);
    const double slack = 2.0 * DBL_EPSILON * tnorm + pivmin;
    for (int kk = tid; kk < nabove; kk += EIG_THREADS) {
        const int idx = s - nabove + kk;   // ascending index
        double lo = t2, hi = gu + slack + fabs(gu) * 4.0 * DBL_EPSILON;
        for (int it = 0; it < 128; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
            if (sturm_count(sdd, se2, s, mid, pivmin) > idx) hi = mid;
            else lo = mid;
        }
        lam[kk] = 0.5 * (lo + hi);
    }
    __syncthreads();

    // ---- 4. inverse iteration, clusters re-orthogonalised --------------------
    const double ortol = ortol_rel * tnorm;
    const int64_t ss = (int64_t)s * s;
    double* du1 = LU;
    double* du2 = LU + ss;
    double* lmul = LU + 2 * ss;
    double* u0 = LU + 3 * ss;
    double* xv = LU + 4 * ss;
    for (int kk = tid; kk < nabove; kk += EIG_THREADS) {
        if (kk > 0 && lam[kk] - lam[kk - 1] <= ortol) continue;   // not a cluster leader
        int kend = kk + 1;
        while (kend < nabove && lam[kend] - lam[kend - 1] <= ortol) ++kend;
        double prev = 0;
        for (int k = kk; k < kend; ++k) {
            double lk = lam[k];
            if (k > kk) {
                const double pertol = 10.0 * DBL_EPSILON * fmax(fabs(lk), tnorm * 1e-3);
                if (lk - prev < pertol) lk = prev + pertol;
            }
            prev = lk;
            // LU with partial pivoting of T - lk I; column k of the interleaved arrays
            double dcur = dd[0] - lk;
            double ucur = s > 1 ? ee[0] : 0.0;
            const double tiny = DBL_EPSILON * tnorm + pivmin;
            for (int i = 0; i + 1 < s; ++i) {
                const double c = ee[i];                   // sub-diagonal below row i
                const double a1 = dd[i + 1] - lk;
                const double b1 = (i + 2 < s) ? ee[i + 1] : 0.0;
                if (fabs(dcur) >= fabs(c)) {
                    double a = dcur == 0.0 ? tiny : dcur;
                    const double f = c / a;
                    u0[(int64_t)i * s + k] = a;
                    du1[(int64_t)i * s + k] = ucur;
                    du2[(int64_t)i * s + k] = 0.0;
                    lmul[(int64_t)i * s + k] = f;          // positive sign: no row swap
                    dcur = a1 - f * ucur;
                    ucur = b1;
                } else {
                    const double f = dcur / c;
                    u0[(int64_t)i * s + k] = c;
                    du1[(int64_t)i * s + k] = a1;
                    du2[(int64_t)i * s + k] = b1;
                    lmul[(int64_t)i * s + k] = -(f + 4.0);   // encodes a swap; f in [-1, 1]
                    dcur = ucur - f * a1;
                    ucur = -f * b1;
                }
            }
            u0[(int64_t)(s - 1) * s + k] = dcur == 0.0 ? tiny : dcur;
            // start vector
            for (int i = 0; i < s; ++i) xv[(int64_t)i * s + k] = start_entry(i, k);
            for (int it = 0; it < 3; ++it) {
                // forward: apply the row operations
                for (int i = 0; i + 1 < s; ++i) {
                    const double lm = lmul[(int64_t)i * s + k];
                    double yi = xv[(int64_t)i * s + k], yi1 = xv[(int64_t)(i + 1) * s + k];
                    if (lm <= -3.0) {  // swapped
                        const double f = -lm - 4.0;
                        const double t = yi;
                        yi = yi1;
                        yi1 = t - f * yi;
                    } else {
                        yi1 -= lm * yi;
                    }
                    xv[(int64_t)i * s + k] = yi;
                    xv[(int64_t)(i + 1) * s + k] = yi1;
                }
                // back substitution
                double x1 = 0, x2 = 0;
                for (int i = s - 1; i >= 0; --i) {
                    double v = xv[(int64_t)i * s + k];
                    if (i + 1 < s) v -= du1[(int64_t)i * s + k] * x1;
                    if (i + 2 < s) v -= du2[(int64_t)i * s + k] * x2;
                    v /= u0[(int64_t)i * s + k];
                    xv[(int64_t)i * s + k] = v;
                    x2 = x1;
                    x1 = v;
                }
                // re-orthogonalise against earlier members of the cluster
                for (int k2 = kk; k2 < k; ++k2) {
                    double dot = 0;
                    for (int i = 0; i < s; ++i) dot += W[(int64_t)i * s + k2] * xv[(int64_t)i * s + k];
                    for (int i = 0; i < s; ++i) xv[(int64_t)i * s + k] -= dot * W[(int64_t)i * s + k2];
                }
                double nrm = 0, amax = 0;
                for (int i = 0; i < s; ++i) amax = fmax(amax, fabs(xv[(int64_t)i * s + k]));
                if (!(amax > 0) || !(amax < DBL_MAX)) {
                    for (int i = 0; i < s; ++i) xv[(int64_t)i * s + k] = start_entry(i, k + 7 * it + 1);
                    continue;
                }
                for (int i = 0; i < s; ++i) {
                    const double v = xv[(int64_t)i * s + k] / amax;
                    nrm += v * v;
                }
                nrm = 1.0 / (amax * sqrt(nrm));
                for (int i = 0; i < s; ++i) xv[(int64_t)i * s + k] *= nrm;
            }
            for (int i = 0; i < s; ++i) W[(int64_t)i * s + k] = xv[(int64_t)i * s + k];
        }
    }
    __syncthreads();

    // ---- 5. back-transform: X = Q diag(phase) W sqrt(f) ----------------------
    const int r = nabove;
    for (int e = tid; e < s * r; e += EIG_THREADS) {
        const int i = e / r, k = e - i * r;
        const double sig = sqrt(fmax(lam[k], 0.0));
        const double f = sig > 0 ? fmax(1.0 - thr / sig, 0.0) : 0.0;
        const double w = W[(int64_t)i * s + k] * sqrt(f);
        X[(int64_t)i * s + k] = make_double2(dre[i] * w, dim_[i] * w);
    }
    __syncthreads();
    for (int i = s - 2; i >= 0 && r > 0; --i) {
        const double hh = hv[i];
        if (!(hh > 0)) continue;     // uniform: hv is in global memory, same for all threads
        const int ni = s - i - 1;
        for (int t = tid; t < ni; t += EIG_THREADS) uvec[t] = A[(int64_t)i * s + i + 1 + t];
        __syncthreads();
        for (int k = tid; k < r; k += EIG_THREADS) {
            double dr = 0, di = 0;
            for (int t = 0; t < ni; ++t) {
                const double2 u = uvec[t], x = X[(int64_t)(i + 1 + t) * s + k];
                dr += u.x * x.x + u.y * x.y;
                di += u.x * x.y - u.y * x.x;
            }
            dr /= hh;
            di /= hh;
            for (int t = 0; t < ni; ++t) {
                const double2 u = uvec[t];
                double2 x = X[(int64_t)(i + 1 + t) * s + k];
                x.x -= u.x * dr - u.y * di;
                x.y -= u.x * di + u.y * dr;
                X[(int64_t)(i + 1 + t) * s + k] = x;
            }
        }
        __syncthreads();
    }
    // ---- 6. S = X X^H ---------------------------------------------------------
    for (int e = tid; e < s * s; e += EIG_THREADS) {
        const int a = e / s, b = e - a * s;
        double sr = 0, si = 0;
        for (int k = 0; k < r; ++k) {
            const double2 xa = X[(int64_t)a * s + k], xb = X[(int64_t)b * s + k];
            sr += xa.x * xb.x + xa.y * xb.y;
            si += xa.y * xb.x - xa.x * xb.y;
        }
        OC o;
        o.x = sr;
        o.y = si;
        S[(int64_t)a * s + b] = o;
    }
    if (tid == 0) {
        int pos = 0;
        for (int k = 0; k < r; ++k) pos += sqrt(fmax(lam[k], 0.0)) > thr;
        if (ranks) ranks[m0 + blockIdx.x] = pos;
        if (bad && flags) atomicOr(flags, 1u);
    }
}

template <typename OC>
hipError_t launch_heig_svt(hipStream_t st, const LRDesc* descs, int m0, int count, double2* Gs, int64_t g_stride,
                           OC* Ss, int64_t s_stride, double* scr, int64_t scr_stride, int32_t* ranks,
                           double ortol_rel, uint32_t* flags) {
    hipLaunchKernelGGL((k_heig_svt<OC>), dim3(count), dim3(EIG_THREADS), 0, st, descs, m0, Gs, g_stride, Ss, s_stride,
                       scr, scr_stride, ranks, ortol_rel, flags);
    return hipGetLastError();
}

template hipError_t launch_heig_svt<float2>(hipStream_t, const LRDesc*, int, int, double2*, int64_t, float2*, int64_t,
                                            double*, int64_t, int32_t*, double, uint32_t*);
template hipError_t launch_heig_svt<double2>(hipStream_t, const LRDesc*, int, int, double2*, int64_t, double2*,
                                             int64_t, double*, int64_t, int32_t*, double, uint32_t*);

}  // namespace shlr
