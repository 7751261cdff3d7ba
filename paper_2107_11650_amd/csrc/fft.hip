// Centred unitary 1D DFTs of batched lines, the fused X-update of Eq. 15 /
// Eq. S7, and small element-wise kernels (gfx950).
//
// DFT convention: DC at index n/2 on both sides, 1/sqrt(n) scaling, so the
// transform is unitary and its adjoint is its inverse (as Eq. 15 requires).
// The transform itself is a mixed-radix Stockham FFT in LDS (radix 4, 2 and
// every remaining small prime; a prime radix is applied as a direct small DFT).
// A length with a prime factor above 31 goes through Bluestein's chirp-z form
// instead: X_k = conj(w_k) sum_j (x_j conj(w_j)) w_{k-j}, w_j = exp(i pi j^2 / n),
// the convolution done by power-of-two FFTs of size f >= 2n - 1 in LDS.
// The centring is folded into the load and store indices.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace shlr {

constexpr int FFT_THREADS = 512;
__device__ inline int64_t line_off(const LineAddr& a, int g) {
    const int g1 = g < (1 << 21) ? div_small(g, a.n0) : g / a.n0, g0 = g - g1 * a.n0;
    return a.base + (int64_t)g1 * a.s1 + (int64_t)g0 * a.s0;
}

template <typename C>
__device__ inline void make_twiddles(C* tw, int n, int tid, int nth) {
    for (int j = tid; j < n; j += nth) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)n, &sn, &cs);
        tw[j] = cmk<C>(cs, sn);
    }
}

template <typename C>
__device__ inline C twid(const C* tw, int idx, int n, bool inv) {
    C w = tw[idx];
    if (inv) w.y = -w.y;
    (void)n;
    return w;
}

// Runs the stages on NL lines stored contiguously in b0; returns the buffer holding the result.
template <typename C>
__device__ C* fft_run(C* b0, C* b1, const C* tw, int n, int NL, const FftPlan& pl, bool inv, int tid, int nth) {
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        const int r = pl.radix[st];
        const int nb = n / r;
        const int tsc = n / (Ns * r);
        for (int e = tid; e < NL * nb; e += nth) {
            const int line = div_small(e, nb), j = e - line * nb;
            const C* in = b0 + line * n;
            C* out = b1 + line * n;
            const int jq = div_small(j, Ns), kq = j - jq * Ns;
            const int tstep = kq * tsc;
            const int od = jq * Ns * r + kq;
            if (r == 4) {
                C x0 = in[j];
                // kq < Ns gives tstep < n / r, so u tstep < n for u < r: no reduction mod n
                C x1 = cmul(in[j + nb], twid(tw, tstep, n, inv));
                C x2 = cmul(in[j + 2 * nb], twid(tw, 2 * tstep, n, inv));
                C x3 = cmul(in[j + 3 * nb], twid(tw, 3 * tstep, n, inv));
                C s02 = cadd(x0, x2), d02 = csub(x0, x2);
                C s13 = cadd(x1, x3), d13 = csub(x1, x3);
                // forward: -i * d13 ; inverse: +i * d13
                C jd = inv ? cmk<C>(-d13.y, d13.x) : cmk<C>(d13.y, -d13.x);
                out[od] = cadd(s02, s13);
                out[od + Ns] = cadd(d02, jd);
                out[od + 2 * Ns] = csub(s02, s13);
                out[od + 3 * Ns] = csub(d02, jd);
            } else if (r == 2) {
                C x0 = in[j];
                C x1 = cmul(in[j + nb], twid(tw, tstep, n, inv));
                out[od] = cadd(x0, x1);
                out[od + Ns] = csub(x0, x1);
            } else {
                for (int u = 0; u < r; ++u) {
                    C acc = cmk<C>(0, 0);
                    // t step mod n, stepped: step = tstep + u nb < n / r + (r - 1) n / r = n
                    const int step = tstep + u * nb;
                    int idx = 0;
                    for (int t = 0; t < r; ++t) {
                        acc = cadd(acc, cmul(in[j + t * nb], twid(tw, idx, n, inv)));
                        idx += step;
                        if (idx >= n) idx -= n;
                    }
                    out[od + u * Ns] = acc;
                }
            }
        }
        __syncthreads();
        C* t = b0;
        b0 = b1;
        b1 = t;
        Ns *= r;
    }
    return b0;
}

// LDS of a line-transform block: twiddles of size f, then (Bluestein) the FFT of
// the chirp (f) and the chirp (n), then two line buffers of NL x f.
template <typename C>
struct FftLds {
    C *tw, *bt, *wch, *b0, *b1;
};
template <typename C>
__device__ inline FftLds<C> fft_setup(unsigned char* smem, const FftPlan& pl, int NL, int tid, int nth) {
    FftLds<C> L;
    const int f = pl.f, n = pl.n;
    L.tw = reinterpret_cast<C*>(smem);
    L.bt = L.tw + f;
    L.wch = L.bt + (pl.blue ? f : 0);
    L.b0 = L.wch + (pl.blue ? n : 0);
    L.b1 = L.b0 + NL * f;
    make_twiddles(L.tw, f, tid, nth);
    if (pl.blue) {
        // chirp w_j = exp(i pi j^2 / n), the angle reduced exactly (j^2 mod 2n)
        for (int j = tid; j < n; j += nth) {
            const int64_t q = ((int64_t)j * j) % (2 * (int64_t)n);
            double sn, cs;
            sincospi((double)q / (double)n, &sn, &cs);
            L.wch[j] = cmk<C>(cs, sn);
        }
        __syncthreads();
        // b_j = w_j for |j| < n (circularly), transformed once per block
        for (int j = tid; j < f; j += nth) {
            C v = cmk<C>(0, 0);
            if (j < n) v = L.wch[j];
            else if (f - j < n) v = L.wch[f - j];
            L.b0[j] = v;
        }
        __syncthreads();
        C* r = fft_run(L.b0, L.b1, L.tw, f, 1, pl, false, tid, nth);
        for (int j = tid; j < f; j += nth) L.bt[j] = r[j];
    }
    __syncthreads();
    return L;
}

// DFT (inverse if inv, unnormalised) of NL lines of length n held with line stride
// f in b0; returns the buffer that holds the result (same stride).
template <typename C>
__device__ C* dft_run(const FftLds<C>& L, int NL, const FftPlan& pl, bool inv, int tid, int nth) {
    if (!pl.blue) return fft_run(L.b0, L.b1, L.tw, pl.f, NL, pl, inv, tid, nth);
    const int n = pl.n, f = pl.f;
    // inverse by conjugation: conj(DFT(conj(x)))
    for (int e = tid; e < NL * f; e += nth) {
        const int line = div_small(e, f), j = e - line * f;
        C v = cmk<C>(0, 0);
        if (j < n) {
            C x = L.b0[line * f + j];
            if (inv) x.y = -x.y;
            v = cmulc(L.wch[j], x);   // conj(w_j) x_j
        }
        L.b0[line * f + j] = v;
    }
    __syncthreads();
    C* r = fft_run(L.b0, L.b1, L.tw, f, NL, pl, false, tid, nth);
    for (int e = tid; e < NL * f; e += nth) r[e] = cmul(r[e], L.bt[e - div_small(e, f) * f]);
    __syncthreads();
    C* o = (r == L.b0) ? L.b1 : L.b0;
    C* r2 = fft_run(r, o, L.tw, f, NL, pl, true, tid, nth);
    const double invf = 1.0 / (double)f;
    for (int e = tid; e < NL * n; e += nth) {
        const int line = div_small(e, n), k = e - line * n;
        C v = cmulc(L.wch[k], r2[line * f + k]);   // conj(w_k) c_k
        v.x *= invf;
        v.y *= invf;
        if (inv) v.y = -v.y;
        r2[line * f + k] = v;
    }
    __syncthreads();
    return r2;
}

// dst[line][(i - c) mod n] = src[line][i]  (centred load), for nl lines
template <typename C>
__device__ inline void load_lines_centred(C* dst, const C* src, const LineAddr& a, int g0, int nl, int n, int ls,
                                          int tid, int nth) {
    const int c = n / 2;
    if (a.es == 1) {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += nth) {
            const int line = div_small(e, n), i = e - line * n;
            int t = i - c;
            if (t < 0) t += n;
            dst[line * ls + t] = src[line_off(a, g0 + line) + i];
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += nth) {
            const int i = div_small(e, nl), line = e - i * nl;
            int t = i - c;
            if (t < 0) t += n;
            dst[line * ls + t] = src[line_off(a, g0 + line) + (int64_t)i * a.es];
        }
    }
}

template <typename C, typename R>
__device__ inline void store_lines_centred(C* dstg, const C* res, const LineAddr& a, int g0, int nl, int n, int ls,
                                           R scale, int tid, int nth) {
    const int c = n / 2;
    if (a.es == 1) {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += nth) {
            const int line = div_small(e, n), i = e - line * n;
            int f = i - c;
            if (f < 0) f += n;
            dstg[line_off(a, g0 + line) + i] = cscale(res[line * ls + f], scale);
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += nth) {
            const int i = div_small(e, nl), line = e - i * nl;
            int f = i - c;
            if (f < 0) f += n;
            dstg[line_off(a, g0 + line) + (int64_t)i * a.es] = cscale(res[line * ls + f], scale);
        }
    }
}

// block `blk` of a line-transform launch: lines [blk NL, blk NL + NL)
template <typename R>
__device__ inline void fft_lines_block(unsigned char* smem, const cplx_t<R>* in, cplx_t<R>* out, const LineAddr& ia,
                                       const LineAddr& oa, const FftPlan& pl, int n_lines, int NL, int inverse,
                                       R scale, int blk) {
    using C = cplx_t<R>;
    const int n = pl.n, ls = pl.f;
    const int tid = threadIdx.x;
    const FftLds<C> L = fft_setup<C>(smem, pl, NL, tid, FFT_THREADS);
    const int g0 = blk * NL;
    const int nl = min(NL, n_lines - g0);
    load_lines_centred(L.b0, in, ia, g0, nl, n, ls, tid, FFT_THREADS);
    __syncthreads();
    C* res = dft_run(L, nl, pl, inverse != 0, tid, FFT_THREADS);
    store_lines_centred(out, res, oa, g0, nl, n, ls, scale, tid, FFT_THREADS);
}

template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_lines(const cplx_t<R>* in, cplx_t<R>* out, LineAddr ia,
                                                           LineAddr oa, FftPlan pl, int n_lines, int NL, int inverse,
                                                           R scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fft_lines_block<R>(smem_raw, in, out, ia, oa, pl, n_lines, NL, inverse, scale, blockIdx.x);
}

// the segment of a segmented launch that owns block b (segments sorted by first block)
template <typename S>
__device__ inline int find_seg(const S* segs, int n_seg, int b) {
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One launch over the lines of several slices (segments of their own length and plan).
template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_lines_seg(const cplx_t<R>* in, cplx_t<R>* out,
                                                               const FftSeg* __restrict__ segs, int n_seg) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int si = find_seg(segs, n_seg, blockIdx.x);
    const FftSeg& sg = segs[si];   // read in place (a local copy of the plan's arrays would go to scratch)
    fft_lines_block<R>(smem_raw, in, out, sg.ia, sg.oa, sg.pl, sg.n_lines, sg.NL, sg.inverse, (R)sg.scale,
                       blockIdx.x - sg.block0);
}

// ---------------------------------------------------------------------------
// Fused X-update over rows (Eq. 15 for the PI model, Eq. S7 for PARAM):
//   c   = F(bo_row)                      other-direction adjoint term to k-space
//   K   = (lam m Y + beta (a + c)) / (lam m + beta (rr[i] + rc[row]))
//         (hard data consistency: K = Y where m, else (a + c)/(rr + rc))
//   out = F^-1(K_row)                    hybrid line for the next lifts
// Row index g -> digits (d2, d1, d0) with sizes (., n1, n0).
// ---------------------------------------------------------------------------
__device__ inline void row_digits(const XupdRows& x, int g, int& d2, int& d1, int& d0) {
    d0 = g % x.n0;
    const int t = g / x.n0;
    d1 = t % x.n1;
    d2 = t / x.n1;
}
__device__ inline int64_t row_off(const RowAddr& a, int d2, int d1, int d0) {
    return (int64_t)d2 * a.s2 + (int64_t)d1 * a.s1 + (int64_t)d0 * a.s0;
}

template <typename R>
__device__ inline void xupd_rows_block(unsigned char* smem_raw, const cplx_t<R>* __restrict__ base_bo,
                                       const cplx_t<R>* __restrict__ base_a, const cplx_t<R>* __restrict__ base_y,
                                       cplx_t<R>* __restrict__ base_k, cplx_t<R>* __restrict__ base_out,
                                       const uint8_t* __restrict__ base_m, const R* __restrict__ rtab,
                                       const XupdRows& x, const FftPlan& pl, int NL, R lam, R beta, int hard_dc,
                                       double* __restrict__ change_acc, const int32_t* __restrict__ active,
                                       int rhs_only, int blk) {
    using C = cplx_t<R>;
    const int n = x.n, ls = pl.f;
    const int tid = threadIdx.x;
    const FftLds<C> L = fft_setup<C>(smem_raw, pl, NL, tid, FFT_THREADS);
    C* b0 = L.b0;
    const int g0 = blk * NL;
    const int nl = min(NL, x.n_rows - g0);
    const int c = n / 2;
    const R sc = (R)(1.0 / sqrt((double)n));
    // 1. load the other-direction adjoint rows (centred)
    if (x.bo.es == 1) {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += FFT_THREADS) {
            const int line = div_small(e, n), i = e - line * n;
            int d2, d1, d0;
            row_digits(x, g0 + line, d2, d1, d0);
            int t = i - c;
            if (t < 0) t += n;
            b0[line * ls + t] = base_bo[row_off(x.bo, d2, d1, d0) + i];
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += FFT_THREADS) {
            const int i = div_small(e, nl), line = e - i * nl;
            int d2, d1, d0;
            row_digits(x, g0 + line, d2, d1, d0);
            int t = i - c;
            if (t < 0) t += n;
            b0[line * ls + t] = base_bo[row_off(x.bo, d2, d1, d0) + (int64_t)i * x.bo.es];
        }
    }
    __syncthreads();
    C* res = dft_run(L, nl, pl, false, tid, FFT_THREADS);
    C* oth = (res == L.b0) ? L.b1 : L.b0;
    // 2. combine; write K and stage K (centred) for the inverse transform.  Rows of a unit that
    // the stop test has retired keep K (their staged line is the old K); the change sums are
    // kept per unit and flushed when a thread's unit changes.
    double dsum = 0, osum = 0;
    int cur_u = -1;
    bool cur_act = true;
#pragma unroll 4
    for (int e = tid; e < nl * n; e += FFT_THREADS) {
        const int line = div_small(e, n), i = e - line * n;
        int d2, d1, d0;
        row_digits(x, g0 + line, d2, d1, d0);
        int f = i - c;
        if (f < 0) f += n;
        const int u = x.unit_digit == 2 ? d2 : 0;
        if (u != cur_u) {
            if (change_acc && cur_u >= 0 && (dsum != 0 || osum != 0)) {
                atomicAdd(change_acc + 2 * cur_u, dsum);
                atomicAdd(change_acc + 2 * cur_u + 1, osum);
            }
            dsum = osum = 0;
            cur_u = u;
            cur_act = !active || active[u] != 0;
        }
        const C cv = cscale(res[line * ls + f], sc);
        const C av = base_a[row_off(x.a, d2, d1, d0) + (int64_t)i * x.a.es];
        const int64_t yo = row_off(x.y, d2, d1, d0) + (int64_t)i * x.y.es;
        const int64_t ko = row_off(x.k, d2, d1, d0) + (int64_t)i * x.k.es;
        const uint8_t mk = base_m[row_off(x.msk, d2, d1, d0) + (int64_t)i * x.msk.es];
        const int rci = x.rc_digit == 0 ? d0 : (x.rc_digit == 1 ? d1 : d2);
        const R rsum = rtab[x.rr_off + i] + rtab[x.rc_off + rci];
        C kv;
        if (rhs_only) {
            const C yv = base_y[yo];
            const R lm = mk ? lam : (R)0;
            base_k[ko] = cmk<C>(lm * yv.x + beta * (av.x + cv.x), lm * yv.y + beta * (av.y + cv.y));
            continue;
        }
        if (!cur_act) {
            oth[line * ls + f] = base_k[ko];
            continue;
        }
        if (hard_dc) {
            if (mk) kv = base_y[yo];
            else kv = cmk<C>((av.x + cv.x) / rsum, (av.y + cv.y) / rsum);
        } else {
            const C yv = base_y[yo];
            const R lm = mk ? lam : (R)0;
            const R den = lm + beta * rsum;
            kv = cmk<C>((lm * yv.x + beta * (av.x + cv.x)) / den, (lm * yv.y + beta * (av.y + cv.y)) / den);
        }
        if (change_acc) {
            const C ko_old = base_k[ko];
            dsum += (double)(kv.x - ko_old.x) * (kv.x - ko_old.x) + (double)(kv.y - ko_old.y) * (kv.y - ko_old.y);
            osum += (double)ko_old.x * ko_old.x + (double)ko_old.y * ko_old.y;
        }
        base_k[ko] = kv;
        oth[line * ls + f] = kv;
    }
    if (rhs_only) return;   // uniform: the right-hand side of Eq. 15 only
    if (change_acc) {
        // one atomic pair per wave when its lanes end on one unit (lanes without rows hold -1)
        int umax = cur_u;
        for (int off = 32; off > 0; off >>= 1) umax = max(umax, __shfl_xor(umax, off, 64));
        if (__all(cur_u == umax || cur_u < 0)) {
            for (int off = 32; off > 0; off >>= 1) {
                dsum += __shfl_down(dsum, off, 64);
                osum += __shfl_down(osum, off, 64);
            }
            if ((tid & 63) == 0 && umax >= 0) {
                atomicAdd(change_acc + 2 * umax, dsum);
                atomicAdd(change_acc + 2 * umax + 1, osum);
            }
        } else if (cur_u >= 0 && (dsum != 0 || osum != 0)) {
            atomicAdd(change_acc + 2 * cur_u, dsum);
            atomicAdd(change_acc + 2 * cur_u + 1, osum);
        }
    }
    __syncthreads();
    // 3. inverse transform of K and store the hybrid rows
    FftLds<C> L2 = L;   // the staged K is in oth
    L2.b0 = oth;
    L2.b1 = res;
    C* res2 = dft_run(L2, nl, pl, true, tid, FFT_THREADS);
    if (x.out.es == 1) {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += FFT_THREADS) {
            const int line = div_small(e, n), i = e - line * n;
            int d2, d1, d0;
            row_digits(x, g0 + line, d2, d1, d0);
            int f = i - c;
            if (f < 0) f += n;
            base_out[row_off(x.out, d2, d1, d0) + i] = cscale(res2[line * ls + f], sc);
        }
    } else {
#pragma unroll 4
        for (int e = tid; e < nl * n; e += FFT_THREADS) {
            const int i = div_small(e, nl), line = e - i * nl;
            int d2, d1, d0;
            row_digits(x, g0 + line, d2, d1, d0);
            int f = i - c;
            if (f < 0) f += n;
            base_out[row_off(x.out, d2, d1, d0) + (int64_t)i * x.out.es] = cscale(res2[line * ls + f], sc);
        }
    }
}

template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_xupd_rows(const cplx_t<R>* __restrict__ base_bo,
                                                           const cplx_t<R>* __restrict__ base_a,
                                                           const cplx_t<R>* __restrict__ base_y,
                                                           cplx_t<R>* __restrict__ base_k,
                                                           cplx_t<R>* __restrict__ base_out,
                                                           const uint8_t* __restrict__ base_m,
                                                           const R* __restrict__ rtab, XupdRows x, FftPlan pl,
                                                           int NL, R lam, R beta, int hard_dc,
                                                           double* __restrict__ change_acc,
                                                           const int32_t* __restrict__ active, int rhs_only) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    xupd_rows_block<R>(smem_raw, base_bo, base_a, base_y, base_k, base_out, base_m, rtab, x, pl, NL, lam, beta,
                       hard_dc, change_acc, active, rhs_only, blockIdx.x);
}

// One launch of the fused X-update over the rows of several slices; each segment's arrays sit at its
// own offsets from the arena bases, and its stop unit indexes the change sums and the active flags.
template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_xupd_rows_seg(cplx_t<R>* cbase, const uint8_t* mbase,
                                                               const R* __restrict__ rtab,
                                                               const XupdSeg* __restrict__ segs, int n_seg, R lam,
                                                               R beta, int hard_dc, double* change,
                                                               const int32_t* active) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int si = find_seg(segs, n_seg, blockIdx.x);
    const XupdSeg& sg = segs[si];   // read in place (a local copy of the plan's arrays would go to scratch)
    xupd_rows_block<R>(smem_raw, cbase + sg.bo, cbase + sg.a, cbase + sg.y, cbase + sg.k, cbase + sg.out,
                       mbase + sg.m, rtab, sg.x, sg.pl, sg.NL, lam, beta, hard_dc,
                       change ? change + 2 * sg.unit : nullptr, active ? active + sg.unit : nullptr, 0,
                       blockIdx.x - sg.block0);
}

// ---------------------------------------------------------------------------
// SPIRiT operator of the X-update (Eq. 3 inside Eq. 15) with fewer passes:
//   k_spirit_cols: for one image column n of all J coils, the inverse column
//     transform, the per-pixel product with Aimg = (Gimg - I)^H (Gimg - I)
//     (J x J per pixel, stored [n][b][m][a]) and the forward column transform, in one block;
//     t and y are [J][M][N] with t already transformed along its rows;
//   k_fft_rows_apply: the forward row transform of y fused with the PCG
//     operator Ap = den p + lambda1 y, in place, and one partial Re<p, Ap>
//     per block (fixed order).
// ---------------------------------------------------------------------------
constexpr int SPC_THREADS = 1024;
template <typename R>
__global__ __launch_bounds__(SPC_THREADS) void k_spirit_cols(const cplx_t<R>* __restrict__ t,
                                                             cplx_t<R>* __restrict__ y,
                                                             const cplx_t<R>* __restrict__ A, int J, int M, int N,
                                                             FftPlan pl) {
    using C = cplx_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // blocks are dealt to the 8 XCDs in turn: give each XCD a contiguous range of columns, so that a
    // cache line of 16 neighbouring columns is fetched into (and written back from) one L2 only
    const int per = (N + 7) / 8;
    const int n = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (n >= N) return;   // uniform over the block
    const int tid = threadIdx.x, ls = pl.f, c = M / 2;
    const int64_t MN = (int64_t)M * N;
    const FftLds<C> L = fft_setup<C>(smem_raw, pl, J, tid, SPC_THREADS);
#pragma unroll 4
    for (int e = tid; e < J * M; e += SPC_THREADS) {
        const int j = div_small(e, M), m = e - j * M;
        int q = m - c;
        if (q < 0) q += M;
        L.b0[j * ls + q] = t[j * MN + (int64_t)m * N + n];
    }
    __syncthreads();
    C* res = dft_run(L, J, pl, true, tid, SPC_THREADS);
    C* oth = (res == L.b0) ? L.b1 : L.b0;
    const R sc = (R)(1.0 / sqrt((double)M));
    // one (pixel m, output coil a) pair per thread, e = m J + a: entry b of the operator rows of
    // all pairs of the column is contiguous in e, so every operator read is coalesced.  Two pairs per
    // thread at a time, their rows read in groups of 8 entries before the products, so that a group
    // waits for memory once rather than once per entry.
    constexpr int GB = 8;
    for (int e0 = tid; e0 < M * J; e0 += 2 * SPC_THREADS) {
        R sr[2] = {0, 0}, si[2] = {0, 0};
        int qq[2], aa[2];
        const C* Ar[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = min(e0 + h * SPC_THREADS, M * J - 1);
            const int m = div_small(e, J), a = e - m * J;
            int q = m - c;
            if (q < 0) q += M;
            qq[h] = q;
            aa[h] = a;
            Ar[h] = A + (int64_t)n * J * M * J + e;   // entry b of this row at + b M J
        }
        for (int b0 = 0; b0 < J; b0 += GB) {
            C mv[2][GB];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < GB; ++u) mv[h][u] = b0 + u < J ? Ar[h][(int64_t)(b0 + u) * M * J] : cmk<C>(0, 0);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < GB; ++u) {
                    if (b0 + u < J) {
                        const C v = res[(b0 + u) * ls + qq[h]];
                        sr[h] += mv[h][u].x * v.x - mv[h][u].y * v.y;
                        si[h] += mv[h][u].x * v.y + mv[h][u].y * v.x;
                    }
                }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (e0 + h * SPC_THREADS < M * J) oth[aa[h] * ls + qq[h]] = cmk<C>(sr[h] * sc, si[h] * sc);
    }
    __syncthreads();
    FftLds<C> L2 = L;   // the product is staged in oth
    L2.b0 = oth;
    L2.b1 = res;
    C* r2 = dft_run(L2, J, pl, false, tid, SPC_THREADS);
#pragma unroll 4
    for (int e = tid; e < J * M; e += SPC_THREADS) {
        const int j = div_small(e, M), m = e - j * M;
        int q = m - c;
        if (q < 0) q += M;
        y[j * MN + (int64_t)m * N + n] = cscale(r2[j * ls + q], sc);
    }
}

template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_rows_apply(cplx_t<R>* __restrict__ io,
                                                                const cplx_t<R>* __restrict__ p, int J, int M, int N,
                                                                FftPlan pl, int NL, const uint8_t* __restrict__ mask,
                                                                const R* __restrict__ rtab, int64_t rr_off,
                                                                int64_t rc_off, R lam, R beta, R lam1,
                                                                double* __restrict__ partials) {
    using C = cplx_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[FFT_THREADS / 64];
    const int tid = threadIdx.x, ls = pl.f, c = N / 2;
    const FftLds<C> L = fft_setup<C>(smem_raw, pl, NL, tid, FFT_THREADS);
    const int g0 = blockIdx.x * NL;
    const int nl = min(NL, J * M - g0);
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        L.b0[line * ls + q] = io[(int64_t)(g0 + line) * N + i];
    }
    __syncthreads();
    C* res = dft_run(L, nl, pl, false, tid, FFT_THREADS);
    const R sc = (R)(1.0 / sqrt((double)N));
    double acc = 0;
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        const int m = (g0 + line) % M;
        const int64_t ge = (int64_t)(g0 + line) * N + i;
        const C tv = cscale(res[line * ls + q], sc);
        const R d = (mask[(int64_t)m * N + i] ? lam : (R)0) + beta * (rtab[rr_off + i] + rtab[rc_off + m]);
        const C pv = p[ge];
        const C a = cmk<C>(d * pv.x + lam1 * tv.x, d * pv.y + lam1 * tv.y);
        io[ge] = a;
        acc += (double)pv.x * a.x + (double)pv.y * a.y;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double tsum = 0;
        for (int w = 0; w < FFT_THREADS / 64; ++w) tsum += red[w];
        partials[blockIdx.x] = tsum;
    }
}

// ---------------------------------------------------------------------------
// PCG of the SPIRiT X-update in the Chronopoulos-Gear form (one reduction phase per step: both
// inner products of a step are formed before its direction update), so that a step is three
// launches: first row pass, column pass (k_spirit_cols), second row pass.  With u = M^-1 r,
// w = A u, gamma = <r, u>, delta = <u, w>:
//   beta_i = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}  (s_i = A p_i),
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i;
// in exact arithmetic the iterates of PCG.  Inner products are sums of per-block partials in a
// fixed order, formed again in every block that needs them.
// ---------------------------------------------------------------------------

// fixed-order sums of two sets of n partials (the same bits in every block): per-thread strided
// sums, lane 0's butterfly sum per wave, then the waves in order; a null set sums to 0.  All
// FFT_THREADS threads call; red holds 2 * FFT_THREADS / 64 doubles.
__device__ inline double2 rows_sum2(const double* __restrict__ va, const double* __restrict__ vb, int n,
                                    double* red) {
    constexpr int NW = FFT_THREADS / 64;
    const int tid = threadIdx.x;
    double a = 0, b = 0;
    for (int i = tid; i < n; i += FFT_THREADS) {
        if (va) a += va[i];
        if (vb) b += vb[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = a;
        red[NW + (tid >> 6)] = b;
    }
    __syncthreads();
    double sa = 0, sb = 0;
    for (int w = 0; w < NW; ++w) {
        sa += red[w];
        sb += red[NW + w];
    }
    __syncthreads();   // red is free again
    return make_double2(sa, sb);
}

// alpha of step cs.step; block 0 keeps its gamma and alpha in the slots of the step's parity (the
// previous step's slots are the other pair, so no block reads a slot this launch writes)
__device__ inline double cg_alpha(const CgStep& cs, double* red) {
    const double2 gd = rows_sum2(cs.step == 0 ? nullptr : cs.gpart_in, cs.dpart_in, cs.np, red);
    const double g = cs.step == 0 ? *cs.gam0 : gd.x;
    const double d = gd.y;
    double den = d;
    if (cs.step > 0) {
        const double gp = cs.slots[(cs.step - 1) & 1], ap = cs.slots[2 + ((cs.step - 1) & 1)];
        const double b = gp != 0.0 ? g / gp : 0.0;
        den = ap != 0.0 ? d - b * g / ap : 0.0;
    }
    const double a = (den != 0.0 && g != 0.0) ? g / den : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cs.slots[cs.step & 1] = g;
        cs.slots[2 + (cs.step & 1)] = a;
    }
    return a;
}

// preconditioner: the X-update's diagonal den at (row m, column i)
template <typename R>
__device__ inline R cg_den(const uint8_t* __restrict__ mask, const R* __restrict__ rtab, int64_t rr_off,
                           int64_t rc_off, R lam, R beta, int m, int i, int N) {
    return (mask[(int64_t)m * N + i] ? lam : (R)0) + beta * (rtab[rr_off + i] + rtab[rc_off + m]);
}

// block partial of a per-thread sum into out[blockIdx.x]; all threads call
__device__ inline void rows_partial(double acc, double* red, double* out) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < FFT_THREADS / 64; ++w) t += red[w];
        out[blockIdx.x] = t;
    }
}

// First row pass of step i: alpha_i, x += alpha_i p, r -= alpha_i s, u = r / den, partials of
// <r, u> (gamma_{i+1}), t = F_n^-1 u along rows.  Rows are the J*M lines of length N.
template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_rows_cg1(cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ r,
                                                              const cplx_t<R>* __restrict__ p,
                                                              const cplx_t<R>* __restrict__ s,
                                                              cplx_t<R>* __restrict__ t, int J, int M, int N,
                                                              FftPlan pl, int NL, const uint8_t* __restrict__ mask,
                                                              const R* __restrict__ rtab, int64_t rr_off,
                                                              int64_t rc_off, R lam, R beta, CgStep cs) {
    using C = cplx_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[FFT_THREADS];
    const int tid = threadIdx.x, ls = pl.f, c = N / 2;
    const R al = (R)cg_alpha(cs, red);
    const FftLds<C> L = fft_setup<C>(smem_raw, pl, NL, tid, FFT_THREADS);
    const int g0 = blockIdx.x * NL;
    const int nl = min(NL, J * M - g0);
    double acc = 0;
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        const int g = g0 + line, m = g - div_small(g, M) * M;
        const int64_t ge = (int64_t)g * N + i;
        const R d = cg_den(mask, rtab, rr_off, rc_off, lam, beta, m, i, N);
        const C pv = p[ge], sv = s[ge];
        C xv = x[ge], rv = r[ge];
        xv.x += al * pv.x;
        xv.y += al * pv.y;
        rv.x -= al * sv.x;
        rv.y -= al * sv.y;
        const C uv = cscale(rv, (R)1 / d);
        x[ge] = xv;
        r[ge] = rv;
        L.b0[line * ls + q] = uv;
        acc += (double)rv.x * uv.x + (double)rv.y * uv.y;
    }
    rows_partial(acc, red, cs.gpart_out);   // ends with a barrier: the staged rows are complete
    C* res = dft_run(L, nl, pl, true, tid, FFT_THREADS);
    const R sc = (R)(1.0 / sqrt((double)N));
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        t[(int64_t)(g0 + line) * N + i] = cscale(res[line * ls + q], sc);
    }
}

// Second row pass of step i (set-up: of step -1, beta = 0): y is the column pass's output, so that
// F_n y along rows completes the SPIRiT part of w = A u = den u + lambda1 F (G-I)^H (G-I) F^-1 u;
// u = r / den again, partials of <u, w> (delta_{i+1}), beta_{i+1} = gamma_{i+1} / gamma_i,
// p = u + beta p, s = w + beta s.
template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_rows_cg3(const cplx_t<R>* __restrict__ y,
                                                              const cplx_t<R>* __restrict__ r,
                                                              cplx_t<R>* __restrict__ p, cplx_t<R>* __restrict__ s,
                                                              int J, int M, int N, FftPlan pl, int NL,
                                                              const uint8_t* __restrict__ mask,
                                                              const R* __restrict__ rtab, int64_t rr_off,
                                                              int64_t rc_off, R lam, R beta, R lam1, CgStep cs) {
    using C = cplx_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[FFT_THREADS];
    const int tid = threadIdx.x, ls = pl.f, c = N / 2;
    R bc = 0;
    if (!cs.setup) {   // uniform
        const double gn = rows_sum2(cs.gpart_in, nullptr, cs.np, red).x, go = cs.slots[cs.step & 1];
        bc = (R)(go != 0.0 ? gn / go : 0.0);
    }
    const FftLds<C> L = fft_setup<C>(smem_raw, pl, NL, tid, FFT_THREADS);
    const int g0 = blockIdx.x * NL;
    const int nl = min(NL, J * M - g0);
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        L.b0[line * ls + q] = y[(int64_t)(g0 + line) * N + i];
    }
    __syncthreads();
    C* res = dft_run(L, nl, pl, false, tid, FFT_THREADS);
    const R sc = (R)(1.0 / sqrt((double)N));
    double acc = 0;
#pragma unroll 4
    for (int e = tid; e < nl * N; e += FFT_THREADS) {
        const int line = div_small(e, N), i = e - line * N;
        int q = i - c;
        if (q < 0) q += N;
        const int g = g0 + line, m = g - div_small(g, M) * M;
        const int64_t ge = (int64_t)g * N + i;
        const R d = cg_den(mask, rtab, rr_off, rc_off, lam, beta, m, i, N);
        const C uv = cscale(r[ge], (R)1 / d);
        const C tv = cscale(res[line * ls + q], sc);
        const C wv = cmk<C>(d * uv.x + lam1 * tv.x, d * uv.y + lam1 * tv.y);
        acc += (double)uv.x * wv.x + (double)uv.y * wv.y;
        if (cs.setup) {
            p[ge] = uv;
            s[ge] = wv;
        } else {
            const C pv = p[ge], sv = s[ge];
            p[ge] = cmk<C>(uv.x + bc * pv.x, uv.y + bc * pv.y);
            s[ge] = cmk<C>(wv.x + bc * sv.x, wv.y + bc * sv.y);
        }
    }
    rows_partial(acc, red, cs.dpart_out);
}

// the last step's x += alpha p (its r, u and w are not needed)
template <typename R>
__global__ __launch_bounds__(FFT_THREADS) void k_cg_final(cplx_t<R>* __restrict__ x, const cplx_t<R>* __restrict__ p,
                                                          int64_t count, CgStep cs) {
    __shared__ double red[FFT_THREADS];
    const R al = (R)cg_alpha(cs, red);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const cplx_t<R> pv = p[e];
        cplx_t<R> xv = x[e];
        xv.x += al * pv.x;
        xv.y += al * pv.y;
        x[e] = xv;
    }
}

// ---------------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------------

template <typename R>
__global__ void k_scale_copy(const cplx_t<R>* in, cplx_t<R>* out, int64_t count, const double* scale_ptr, int invert) {
    const double sc = scale_ptr ? (invert ? 1.0 / scale_ptr[0] : scale_ptr[0]) : 1.0;
    const R s = (R)sc;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = cscale(in[i], s);
}

// out[idx] = table[(idx / div) % mod]
template <typename R>
__global__ void k_fill_pattern(cplx_t<R>* out, int64_t count, const cplx_t<R>* table, int64_t div, int64_t mod) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = table[(i / div) % mod];
}

template <typename R>
__global__ void k_fill_const(cplx_t<R>* out, int64_t count, R re, R im) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = cmk<cplx_t<R>>(re, im);
}

// deterministic pseudo-random values in [-scale, scale] (tuning data): a 64-bit mix of the index
template <typename R>
__global__ void k_fill_hash(cplx_t<R>* out, int64_t count, uint64_t seed, R scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t x = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 27;
        x *= 0x94D049BB133111EBull;
        x ^= x >> 33;
        const R a = (R)((double)(x & 0xffffffull) / 8388608.0 - 1.0);
        const R b = (R)((double)((x >> 24) & 0xffffffull) / 8388608.0 - 1.0);
        out[i] = cmk<cplx_t<R>>(scale * a, scale * b);
    }
}

// running max of |x| (non-negative doubles order like their bit patterns); also flags non-finite values
template <typename R>
__global__ void k_maxabs(const cplx_t<R>* in, int64_t count, unsigned long long* out, uint32_t* flags) {
    double m = 0;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const cplx_t<R> v = in[i];
        const double a = sqrt((double)v.x * v.x + (double)v.y * v.y);
        if (!(a <= 1.79e308)) bad = true;
        else m = fmax(m, a);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
    if (bad && flags) atomicOr(flags, 1u);
}

__global__ void k_zero_doubles(double* p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0.0;
}

// change[0] += sum |a - b|^2, change[1] += sum |b|^2 (the relative change of an iterate a against b);
// with commit != null also commit[i] = a[i] (commit may be b)
template <typename R>
__global__ void k_change_pair(const cplx_t<R>* a, const cplx_t<R>* b, int64_t count, double* __restrict__ change,
                              const int32_t* __restrict__ gate, cplx_t<R>* commit) {
    if (gate && *gate == 0) return;
    double ds = 0, os = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const cplx_t<R> u = a[i], v = b[i];
        if (commit) commit[i] = u;
        const double dx = (double)u.x - v.x, dy = (double)u.y - v.y;
        ds += dx * dx + dy * dy;
        os += (double)v.x * v.x + (double)v.y * v.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        ds += __shfl_down(ds, off, 64);
        os += __shfl_down(os, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(change, ds);
        atomicAdd(change + 1, os);
    }
}

// the stop test of Algorithms S1 / S2, one thread per unit; one block
__global__ void k_stop_test(const double* __restrict__ change, int32_t* __restrict__ active,
                            int32_t* __restrict__ iters, double* __restrict__ rel, int n_units, double tol,
                            int32_t* __restrict__ n_active) {
    __shared__ int cnt[256];
    int c = 0;
    for (int u = threadIdx.x; u < n_units; u += blockDim.x) {
        if (!active[u]) continue;
        iters[u] += 1;
        const double num = change[2 * u], den = change[2 * u + 1];
        const double r = den > 0 ? num / den : (num > 0 ? INFINITY : 0.0);
        rel[u] = r;
        if (tol > 0 && r < tol) active[u] = 0;
        else ++c;
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_active = cnt[0];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

static void radix_stages(FftPlan& p, int m) {
    p.nst = 0;
    while (m % 4 == 0 && p.nst < FFT_MAX_STAGES) { p.radix[p.nst++] = 4; m /= 4; }
    while (m % 2 == 0 && p.nst < FFT_MAX_STAGES) { p.radix[p.nst++] = 2; m /= 2; }
    for (int f = 3; m > 1 && p.nst < FFT_MAX_STAGES; f += 2) {
        while (m % f == 0 && p.nst < FFT_MAX_STAGES) { p.radix[p.nst++] = f; m /= f; }
    }
}

constexpr int FFT_BLUE_PRIME = 31;    // a larger prime factor goes through the chirp-z form
constexpr int FFT_BLUE_MAXF = 2048;   // largest chirp-z FFT held in LDS

FftPlan make_fft_plan(int n) {
    FftPlan p;
    p.n = n;
    p.f = n;
    p.blue = 0;
    int m = n, lpf = 1;
    for (int f = 2; (int64_t)f * f <= m; ++f)
        while (m % f == 0) {
            lpf = f;
            m /= f;
        }
    if (m > 1) lpf = std::max(lpf, m);
    int f2 = 1;
    while (f2 < 2 * n - 1) f2 *= 2;
    if (lpf > FFT_BLUE_PRIME && f2 <= FFT_BLUE_MAXF) {
        p.blue = 1;
        p.f = f2;
    }
    radix_stages(p, p.f);
    return p;
}

template <typename R>
static int fft_lines_per_block(const FftPlan& pl, bool strided) {
    int budget = (sizeof(R) == 4 ? 2048 : 1024) * (strided ? 2 : 1);
    if (pl.blue) budget = sizeof(R) == 4 ? 4096 : 2048;
    int nl = budget / pl.f;
    if (nl < 1) nl = 1;
    if (nl > 64) nl = 64;
    return nl;
}
template <typename R>
static size_t fft_lds_bytes(const FftPlan& pl, int NL) {
    return (size_t)(pl.f + (pl.blue ? pl.f + pl.n : 0) + 2 * NL * pl.f) * sizeof(cplx_t<R>);
}

template <typename R>
hipError_t launch_fft_lines(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, const LineAddr& ia,
                            const LineAddr& oa, int n, int n_lines, int inverse, double scale) {
    if (n_lines <= 0) return hipSuccess;
    FftPlan pl = make_fft_plan(n);
    const int NL = fft_lines_per_block<R>(pl, ia.es != 1 || oa.es != 1);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_lines<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (n_lines + NL - 1) / NL;
    hipLaunchKernelGGL((k_fft_lines<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, in, out, ia, oa, pl, n_lines, NL,
                       inverse, (R)scale);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_xupd_rows(hipStream_t st, const cplx_t<R>* bo, const cplx_t<R>* a, const cplx_t<R>* y,
                            cplx_t<R>* k, cplx_t<R>* out, const uint8_t* m, const R* rtab, const XupdRows& x,
                            double lam, double beta, int hard_dc, double* change_acc, const int32_t* active) {
    if (x.n_rows <= 0) return hipSuccess;
    FftPlan pl = make_fft_plan(x.n);
    const int NL = fft_lines_per_block<R>(pl, x.bo.es != 1 || x.out.es != 1);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    hipError_t e = hipFuncSetAttribute((const void*)k_xupd_rows<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (x.n_rows + NL - 1) / NL;
    hipLaunchKernelGGL((k_xupd_rows<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, bo, a, y, k, out, m, rtab, x, pl,
                       NL, (R)lam, (R)beta, hard_dc, change_acc, active, 0);
    return hipGetLastError();
}

template <typename R>
FftSeg make_fft_seg(int n, int n_lines, int inverse, double scale, const LineAddr& ia, const LineAddr& oa, int block0,
                    size_t* lds) {
    FftSeg g;
    g.pl = make_fft_plan(n);
    g.NL = fft_lines_per_block<R>(g.pl, ia.es != 1 || oa.es != 1);
    g.ia = ia;
    g.oa = oa;
    g.n_lines = n_lines;
    g.block0 = block0;
    g.inverse = inverse;
    g.scale = scale;
    *lds = fft_lds_bytes<R>(g.pl, g.NL);
    return g;
}
template <typename R>
XupdSeg make_xupd_seg(const XupdRows& x, int block0, int unit, int64_t bo, int64_t a, int64_t y, int64_t k,
                      int64_t out, int64_t m, size_t* lds) {
    XupdSeg g;
    g.pl = make_fft_plan(x.n);
    g.NL = fft_lines_per_block<R>(g.pl, x.bo.es != 1 || x.out.es != 1);
    g.x = x;
    g.block0 = block0;
    g.unit = unit;
    g.bo = bo;
    g.a = a;
    g.y = y;
    g.k = k;
    g.out = out;
    g.m = m;
    *lds = fft_lds_bytes<R>(g.pl, g.NL);
    return g;
}
int fft_seg_blocks(const FftSeg& g) { return (g.n_lines + g.NL - 1) / g.NL; }
int xupd_seg_blocks(const XupdSeg& g) { return (g.x.n_rows + g.NL - 1) / g.NL; }

template <typename R>
hipError_t launch_fft_lines_seg(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, const FftSeg* segs_dev,
                                int n_seg, int blocks, size_t lds) {
    if (blocks <= 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_lines_seg<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fft_lines_seg<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, in, out, segs_dev, n_seg);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_xupd_rows_seg(hipStream_t st, cplx_t<R>* cbase, const uint8_t* mbase, const R* rtab,
                                const XupdSeg* segs_dev, int n_seg, int blocks, size_t lds, double lam, double beta,
                                int hard_dc, double* change, const int32_t* active) {
    if (blocks <= 0) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_xupd_rows_seg<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_xupd_rows_seg<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, cbase, mbase, rtab, segs_dev,
                       n_seg, (R)lam, (R)beta, hard_dc, change, active);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_xupd_rows_rhs(hipStream_t st, const cplx_t<R>* bo, const cplx_t<R>* a, const cplx_t<R>* y,
                                cplx_t<R>* rhs, const uint8_t* m, const R* rtab, const XupdRows& x, double lam,
                                double beta) {
    if (x.n_rows <= 0) return hipSuccess;
    FftPlan pl = make_fft_plan(x.n);
    const int NL = fft_lines_per_block<R>(pl, x.bo.es != 1 || x.out.es != 1);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    hipError_t e = hipFuncSetAttribute((const void*)k_xupd_rows<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (x.n_rows + NL - 1) / NL;
    hipLaunchKernelGGL((k_xupd_rows<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, bo, a, y, rhs, (cplx_t<R>*)nullptr,
                       m, rtab, x, pl, NL, (R)lam, (R)beta, 0, (double*)nullptr, (const int32_t*)nullptr, 1);
    return hipGetLastError();
}

static inline int ew_blocks(int64_t count) {
    int64_t b = (count + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename R>
hipError_t launch_scale_copy(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, int64_t count,
                             const double* scale_ptr, int invert) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_scale_copy<R>), dim3(ew_blocks(count)), dim3(256), 0, st, in, out, count, scale_ptr, invert);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_fill_pattern(hipStream_t st, cplx_t<R>* out, int64_t count, const cplx_t<R>* table, int64_t div,
                               int64_t mod) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_pattern<R>), dim3(ew_blocks(count)), dim3(256), 0, st, out, count, table, div, mod);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_fill_const(hipStream_t st, cplx_t<R>* out, int64_t count, double re, double im) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_const<R>), dim3(ew_blocks(count)), dim3(256), 0, st, out, count, (R)re, (R)im);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_fill_hash(hipStream_t st, cplx_t<R>* out, int64_t count, uint64_t seed, double scale) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_hash<R>), dim3(ew_blocks(count)), dim3(256), 0, st, out, count, seed, (R)scale);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_maxabs(hipStream_t st, const cplx_t<R>* in, int64_t count, unsigned long long* out,
                         uint32_t* flags) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_maxabs<R>), dim3(ew_blocks(count)), dim3(256), 0, st, in, count, out, flags);
    return hipGetLastError();
}
hipError_t launch_zero_doubles(hipStream_t st, double* p, int count) {
    hipLaunchKernelGGL(k_zero_doubles, dim3(1), dim3(256), 0, st, p, count);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_change_pair(hipStream_t st, const cplx_t<R>* a, const cplx_t<R>* b, int64_t count, double* change,
                              const int32_t* gate, cplx_t<R>* commit) {
    if (count <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(1024, (count + 255) / 256);
    hipLaunchKernelGGL((k_change_pair<R>), dim3(blocks), dim3(256), 0, st, a, b, count, change, gate, commit);
    return hipGetLastError();
}
hipError_t launch_stop_test(hipStream_t st, const double* change, int32_t* active, int32_t* iters, double* rel,
                            int n_units, double tol, int32_t* n_active) {
    hipLaunchKernelGGL(k_stop_test, dim3(1), dim3(256), 0, st, change, active, iters, rel, n_units, tol, n_active);
    return hipGetLastError();
}

template <typename R>
int spirit_fused_blocks(int J, int M, int N) {
    const FftPlan pm = make_fft_plan(M), pn = make_fft_plan(N);
    if (fft_lds_bytes<R>(pm, J) > 160 * 1024) return 0;
    const int NL = fft_lines_per_block<R>(pn, false);
    return (J * M + NL - 1) / NL;
}

template <typename R>
hipError_t launch_spirit_cols(hipStream_t st, const cplx_t<R>* t, cplx_t<R>* y, const cplx_t<R>* A, int J, int M,
                              int N) {
    const FftPlan pl = make_fft_plan(M);
    const size_t lds = fft_lds_bytes<R>(pl, J);
    hipError_t e = hipFuncSetAttribute((const void*)k_spirit_cols<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spirit_cols<R>), dim3(8 * ((N + 7) / 8)), dim3(SPC_THREADS), lds, st, t, y, A, J, M, N,
                       pl);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_rows_cg1(hipStream_t st, cplx_t<R>* x, cplx_t<R>* r, const cplx_t<R>* p, const cplx_t<R>* s,
                               cplx_t<R>* t, int J, int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off,
                               int64_t rc_off, double lam, double beta, const CgStep& cs) {
    const FftPlan pl = make_fft_plan(N);
    const int NL = fft_lines_per_block<R>(pl, false);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    const int blocks = (J * M + NL - 1) / NL;
    if (blocks != cs.np) return hipErrorInvalidValue;   // the partial sets are one entry per block
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows_cg1<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fft_rows_cg1<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, x, r, p, s, t, J, M, N, pl, NL,
                       mask, rtab, rr_off, rc_off, (R)lam, (R)beta, cs);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_rows_cg3(hipStream_t st, const cplx_t<R>* y, const cplx_t<R>* r, cplx_t<R>* p, cplx_t<R>* s,
                               int J, int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off,
                               double lam, double beta, double lam1, const CgStep& cs) {
    const FftPlan pl = make_fft_plan(N);
    const int NL = fft_lines_per_block<R>(pl, false);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    const int blocks = (J * M + NL - 1) / NL;
    if (blocks != cs.np) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows_cg3<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fft_rows_cg3<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, y, r, p, s, J, M, N, pl, NL,
                       mask, rtab, rr_off, rc_off, (R)lam, (R)beta, (R)lam1, cs);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_final(hipStream_t st, cplx_t<R>* x, const cplx_t<R>* p, int64_t count, const CgStep& cs) {
    const int64_t need = (count + FFT_THREADS - 1) / FFT_THREADS;
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>(need, 1), 1024);
    hipLaunchKernelGGL((k_cg_final<R>), dim3(blocks), dim3(FFT_THREADS), 0, st, x, p, count, cs);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_rows_apply(hipStream_t st, cplx_t<R>* io, const cplx_t<R>* p, int J, int M, int N,
                                 const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off, double lam,
                                 double beta, double lam1, double* partials) {
    const FftPlan pl = make_fft_plan(N);
    const int NL = fft_lines_per_block<R>(pl, false);
    const size_t lds = fft_lds_bytes<R>(pl, NL);
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows_apply<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (J * M + NL - 1) / NL;
    hipLaunchKernelGGL((k_fft_rows_apply<R>), dim3(blocks), dim3(FFT_THREADS), lds, st, io, p, J, M, N, pl, NL, mask,
                       rtab, rr_off, rc_off, (R)lam, (R)beta, (R)lam1, partials);
    return hipGetLastError();
}

#define SHLR_INST(R)                                                                                                 \
    template hipError_t launch_fft_lines<R>(hipStream_t, const cplx_t<R>*, cplx_t<R>*, const LineAddr&,              \
                                            const LineAddr&, int, int, int, double);                                 \
    template hipError_t launch_xupd_rows<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, const cplx_t<R>*,       \
                                            cplx_t<R>*, cplx_t<R>*, const uint8_t*, const R*, const XupdRows&,       \
                                            double, double, int, double*, const int32_t*);                           \
    template hipError_t launch_xupd_rows_rhs<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, const cplx_t<R>*,   \
                                                cplx_t<R>*, const uint8_t*, const R*, const XupdRows&, double,        \
                                                double);                                                              \
    template hipError_t launch_scale_copy<R>(hipStream_t, const cplx_t<R>*, cplx_t<R>*, int64_t, const double*, int); \
    template hipError_t launch_fill_pattern<R>(hipStream_t, cplx_t<R>*, int64_t, const cplx_t<R>*, int64_t, int64_t); \
    template hipError_t launch_fill_const<R>(hipStream_t, cplx_t<R>*, int64_t, double, double);                      \
    template hipError_t launch_fill_hash<R>(hipStream_t, cplx_t<R>*, int64_t, uint64_t, double);                     \
    template hipError_t launch_maxabs<R>(hipStream_t, const cplx_t<R>*, int64_t, unsigned long long*, uint32_t*);   \
    template int spirit_fused_blocks<R>(int, int, int);                                                              \
    template FftSeg make_fft_seg<R>(int, int, int, double, const LineAddr&, const LineAddr&, int, size_t*);       \
    template XupdSeg make_xupd_seg<R>(const XupdRows&, int, int, int64_t, int64_t, int64_t, int64_t, int64_t,     \
                                      int64_t, size_t*);                                                          \
    template hipError_t launch_fft_lines_seg<R>(hipStream_t, const cplx_t<R>*, cplx_t<R>*, const FftSeg*, int, int,  \
                                                size_t);                                                         \
    template hipError_t launch_xupd_rows_seg<R>(hipStream_t, cplx_t<R>*, const uint8_t*, const R*, const XupdSeg*,   \
                                                int, int, size_t, double, double, int, double*, const int32_t*);  \
    template hipError_t launch_change_pair<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, int64_t, double*,     \
                                              const int32_t*, cplx_t<R>*);                                           \
    template hipError_t launch_fft_rows_cg1<R>(hipStream_t, cplx_t<R>*, cplx_t<R>*, const cplx_t<R>*, const cplx_t<R>*, \
                                               cplx_t<R>*, int, int, int, const uint8_t*, const R*, int64_t, int64_t, \
                                               double, double, const CgStep&);                                       \
    template hipError_t launch_fft_rows_cg3<R>(hipStream_t, const cplx_t<R>*, const cplx_t<R>*, cplx_t<R>*,           \
                                               cplx_t<R>*, int, int, int, const uint8_t*, const R*, int64_t, int64_t, \
                                               double, double, double, const CgStep&);                               \
    template hipError_t launch_cg_final<R>(hipStream_t, cplx_t<R>*, const cplx_t<R>*, int64_t, const CgStep&);        \
    template hipError_t launch_spirit_cols<R>(hipStream_t, const cplx_t<R>*, cplx_t<R>*, const cplx_t<R>*, int, int, \
                                              int);                                                                  \
    template hipError_t launch_fft_rows_apply<R>(hipStream_t, cplx_t<R>*, const cplx_t<R>*, int, int, int,           \
                                                 const uint8_t*, const R*, int64_t, int64_t, double, double, double, \
                                                 double*);
SHLR_INST(float)
SHLR_INST(double)

}  // namespace shlr
