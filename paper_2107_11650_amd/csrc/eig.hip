// Batched FP64 Hermitian eigen-solver that turns a Gram matrix into the
// singular-value-threshold factor of Eq. 16:
//   G = A^H A = V Lambda V^H,   sigma_i = sqrt(lambda_i),
//   f_i = max(1 - thr / sigma_i, 0),   S = V diag(f) V^H,
// so that A S = U max(Sigma - thr, 0) V^H (the SVT of A).
// Only eigenpairs with lambda_i > thr^2 contribute, and only those are computed.
//
// One workgroup per matrix, all arithmetic in FP64:
//  1. Householder reduction to tridiagonal form with Hermitian reflectors
//     P = I - u u^H / h (the matrix lives in the per-slot scratch in HBM/L2),
//     unless a register-resident reduction (k_tridiag_rr in FP64,
//     k_tridiag_rr32 in FP32 for the mixed form) already ran;
//  2. a diagonal unitary makes the off-diagonal real and non-negative;
//  3. Sturm-sequence bisection for every eigenvalue above thr^2, in parallel;
//  4. eigenvectors from a twisted factorisation of T - lambda I per eigenvalue;
//     eigenvalues closer than ortol are grouped, and the later members of a
//     group are refined by inverse iteration and re-orthogonalised by the
//     whole workgroup (classical Gram-Schmidt, twice);
//  5. back-transformation through the reflectors, scaling by sqrt(f), and
//     S = X X^H written in the working precision (row-major, ld = s).
#include <float.h>

#include "common.h"

namespace shlr {

constexpr int EIG_THREADS = 512;
constexpr int EIG_MAXS = 320;                    // largest supported order
constexpr int EIG_STAGE = 6 + EIG_THREADS / 64;  // smax-sized double2 rows of LDS region A (staging)

// double2 entries of LDS region A: the staging rows, and at least one 16 x 16 tile per wave plus
// one more for the blocked back-transform.  Beyond that it grows, up to 19 rows, while the
// kernel's LDS stays within half a compute unit's (two workgroups per CU): the eigenvector step
// keeps the factors of one eigenvalue per 2 s + 1 doubles of it, and more of them at once means
// fewer sequential batches.
__host__ __device__ inline int heig_region_a(int smax) {
    const int a = EIG_STAGE * smax, b = (EIG_THREADS / 64 + 1) * 256;
    const int rest = 9 * smax * 8 + (2 * (EIG_THREADS / 64) + 8) * 8;      // bytes after region A
    const int half = (80 * 1024 - rest) / 16;                               // double2 entries
    const int c = 19 * smax < half ? 19 * smax : half;
    const int ab = a > b ? a : b;
    return ab > c ? ab : c;
}

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

// 1 / q from the hardware reciprocal and one Newton step (q is kept away from 0)
__device__ inline double rcp_nr(double q) {
    const double r = __builtin_amdgcn_rcp(q);
    return fma(r, fma(-q, r, 1.0), r);
}

// number of eigenvalues of the symmetric tridiagonal (d, e2 = e^2) below x; the entries
// are read four at a time ahead of the dependent steps
__device__ inline int sturm_count(const double* d, const double* e2, int s, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0;
    int i = 1;
    for (; i + 3 < s; i += 4) {
        const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
        const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
        q = d0 - x - f0 * rcp_nr(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
        q = d1 - x - f1 * rcp_nr(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
        q = d2 - x - f2 * rcp_nr(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
        q = d3 - x - f3 * rcp_nr(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    for (; i < s; ++i) {
        q = d[i] - x - e2[i - 1] * rcp_nr(q);
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

// x <- P_i x for every column of Xv (s x nvec, column-major, global), with the
// Hermitian reflectors P_i = I - u_i u_i^H / h_i of the tridiagonalisation
// (u_i below the diagonal of column i of the packed matrix A, h_i = shv[i]):
// i = s-2 .. 0 gives Q x (back-transform), i = 0 .. s-2 gives Q^H x.
// Reflectors are staged in LDS in chunks shared by all waves; one wave per
// column, lane l owning rows l, l + 64, ... in registers.  All threads call.
template <int SL, int VB>
__device__ void apply_reflectors_t(double2* __restrict__ Xv, int nvec, int s, int smax,
                                   const double2* __restrict__ A, const double* shv, double2* stage,
                                   bool adjoint) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nw = EIG_THREADS / 64;
    // every wave's columns fit one batch: they stay in registers across the chunks
    const bool resident = nvec <= nw * VB;
    double2 xr[VB][SL];
    auto load_cols = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VB; ++v)
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const int row = sl * 64 + lane;
                xr[v][sl] = (k0 + v < nvec && row < s) ? Xv[(int64_t)(k0 + v) * s + row] : make_double2(0.0, 0.0);
            }
    };
    auto store_cols = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VB; ++v)
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const int row = sl * 64 + lane;
                if (k0 + v < nvec && row < s) Xv[(int64_t)(k0 + v) * s + row] = xr[v][sl];
            }
    };
    auto apply_chunk = [&](int c0, int cnt) {
        for (int j = 0; j < cnt; ++j) {
            const int i = adjoint ? c0 + j : s - 2 - c0 - j;
            const double hh = shv[i];
            if (!(hh > 0)) continue;
            double2 ul[SL];
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const int row = sl * 64 + lane;
                ul[sl] = row < s ? stage[j * smax + row] : make_double2(0.0, 0.0);
            }
            double dr[VB], di[VB];
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                dr[v] = 0;
                di[v] = 0;
#pragma unroll
                for (int sl = 0; sl < SL; ++sl) {
                    dr[v] += ul[sl].x * xr[v][sl].x + ul[sl].y * xr[v][sl].y;
                    di[v] += ul[sl].x * xr[v][sl].y - ul[sl].y * xr[v][sl].x;
                }
            }
#pragma unroll
            for (int v = 0; v < VB; ++v) {
                dr[v] = wave_sum_all(dr[v]) / hh;
                di[v] = wave_sum_all(di[v]) / hh;
            }
#pragma unroll
            for (int v = 0; v < VB; ++v)
#pragma unroll
                for (int sl = 0; sl < SL; ++sl) {
                    xr[v][sl].x -= ul[sl].x * dr[v] - ul[sl].y * di[v];
                    xr[v][sl].y -= ul[sl].x * di[v] + ul[sl].y * dr[v];
                }
        }
    };
    __syncthreads();   // Xv was written by every thread
    if (resident && wave * VB < nvec) load_cols(wave * VB);
    for (int c0 = 0; c0 + 1 < s && nvec > 0; c0 += EIG_STAGE) {
        const int cnt = min(EIG_STAGE, s - 1 - c0);
        __syncthreads();
        for (int e = tid; e < cnt * s; e += EIG_THREADS) {
            const int j = e / s, row = e - j * s;
            const int i = adjoint ? c0 + j : s - 2 - c0 - j;
            stage[j * smax + row] = (row > i && shv[i] > 0) ? A[pk(row, i, s)] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (resident) {
            if (wave * VB < nvec) apply_chunk(c0, cnt);
        } else {
            for (int k0 = wave * VB; k0 < nvec; k0 += nw * VB) {
                load_cols(k0);
                apply_chunk(c0, cnt);
                store_cols(k0);
            }
        }
    }
    if (resident && wave * VB < nvec) store_cols(wave * VB);
    __syncthreads();
}

// x <- P_i x for every column of Xv (see apply_reflectors_t); the batch width follows the column count
template <int SL>
__device__ void apply_reflectors(double2* __restrict__ Xv, int nvec, int s, int smax,
                                 const double2* __restrict__ A, const double* shv, double2* stage,
                                 bool adjoint) {
    constexpr int nw = EIG_THREADS / 64;
    if (nvec <= nw) apply_reflectors_t<SL, 1>(Xv, nvec, s, smax, A, shv, stage, adjoint);
    else if (nvec <= 2 * nw) apply_reflectors_t<SL, 2>(Xv, nvec, s, smax, A, shv, stage, adjoint);
    else apply_reflectors_t<SL, 4>(Xv, nvec, s, smax, A, shv, stage, adjoint);
}

// ---------------------------------------------------------------------------
// Blocked back-transformation on the FP64 matrix cores.  The reflectors of
// columns 16g .. 16g+15 form V_g (s x 16, zero above each reflector's first
// row), and P_16g P_16g+1 ... P_16g+15 = I - V_g T_g V_g^H with T_g upper
// triangular: T_jj = 1/h_j, T[0:j, j] = -(1/h_j) T[0:j, 0:j] V_g[:, 0:j]^H v_j
// (a skipped reflector, h = 0, gives a zero row and column).
// MFMA 16x16x4 operand layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element q of the accumulator is D[l / 16 + 4 q][l % 16].
// ---------------------------------------------------------------------------

// element (row, i) of reflector i (u_i below the diagonal of column i of the packed matrix)
__device__ inline double2 refl_elem(const double2* __restrict__ A, const double* shv, int row, int i, int s) {
    return (i < s - 1 && row > i && row < s && shv[i] > 0) ? A[pk(row, i, s)] : make_double2(0.0, 0.0);
}

// Every T_g, one wave per group (groups dealt out in snake order by size): G = V_g^H V_g on the
// matrix cores into the wave's LDS tile, then lane a forms row a of T_g.  Tg: [group][16][16].
__device__ __attribute__((always_inline)) void wy_factors(const double2* __restrict__ A, const double* shv, int s, double2* __restrict__ Tg,
                           double2* gbuf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int nw = EIG_THREADS / 64;
    const int ng = wy_groups(s);
    const int lr = lane & 15, lk = lane >> 4;
    double2* G = gbuf + wave * 256;
    for (int m = 0; nw * m < ng; ++m) {
        const int g = nw * m + ((m & 1) ? nw - 1 - wave : wave);
        if (g >= ng) continue;   // uniform over the wave
        doublex4 gr = {0.0, 0.0, 0.0, 0.0}, gi = {0.0, 0.0, 0.0, 0.0};
        const int i = 16 * g + lr;
        for (int row0 = 16 * g; row0 < s; row0 += 32) {
            // A = conj(V)^T and B = V take the same element in each lane; eight 4-row steps
            // with their loads issued first
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = refl_elem(A, shv, row0 + 4 * u + lk, i, s);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                gr = mfma16(v[u].x, v[u].x, gr);
                gr = mfma16(v[u].y, v[u].y, gr);
                gi = mfma16(v[u].x, v[u].y, gi);
                gi = mfma16(-v[u].y, v[u].x, gi);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) G[(lk + 4 * q) * 16 + lr] = make_double2(gr[q], gi[q]);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the wave's own LDS tile, read below
        if (lane < 16) {
            const int a = lane;
            double2 trow[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int ij = 16 * g + j;
                const double hj = ij < s - 1 ? shv[ij] : 0.0;
                const double tau = hj > 0 ? 1.0 / hj : 0.0;
                double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                for (int b = 0; b < j; ++b) acc = cfma(trow[b], G[b * 16 + j], acc);   // zero for b < a
                trow[j] = j < a ? make_double2(0.0, 0.0)
                        : j == a ? make_double2(tau, 0.0)
                                 : make_double2(-tau * acc.x, -tau * acc.y);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) Tg[(g * 16 + a) * 16 + j] = trow[j];
        }
    }
}

// X <- Q X for the s x r column-major X (global), Q = P_0 P_1 ... P_{s-2}: groups g = last .. 0,
// each X <- X - V_g T_g V_g^H X.  Per 16-column tile of X, wave w holds the 16-row tiles
// w, w + 8, ... as MFMA accumulators; the partial tiles of W = V_g^H X go to LDS (pbuf, one
// 16 x 16 tile per wave), wave 0 sums them and forms Y = T_g W (ybuf), whose accumulator
// layout is the B operand layout of X -= V_g Y.  Two barriers per group.  All threads call.
template <int SL>
__device__ __attribute__((always_inline)) void backtransform_wy(double2* __restrict__ X, int r, int s, const double2* __restrict__ A,
                                 const double* shv, const double2* __restrict__ Tg, double2* pbuf, double2* ybuf) {
    constexpr int RTW = (SL + 1) / 2;   // 16-row tiles per wave (SL * 64 >= s rows)
    constexpr int nw = EIG_THREADS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int ng = wy_groups(s), nrt = (s + 15) / 16;
    __syncthreads();   // X, Tg written by every thread
    for (int ct = 0; ct * 16 < r; ++ct) {
        const int col = ct * 16 + lr;
        doublex4 xr[RTW], xi[RTW];
#pragma unroll
        for (int m = 0; m < RTW; ++m) {
            const int rt = wave + nw * m;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = rt * 16 + lk + 4 * q;
                const double2 v = (rt < nrt && row < s && col < r) ? X[(int64_t)col * s + row] : make_double2(0.0, 0.0);
                xr[m][q] = v.x;
                xi[m][q] = v.y;
            }
        }
        for (int g = ng - 1; g >= 0; --g) {
            // W = V_g^H X over this wave's row tiles (rows below 16 g + 1 are zero in V_g)
            doublex4 wr = {0.0, 0.0, 0.0, 0.0}, wi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int m = 0; m < RTW; ++m) {
                const int rt = wave + nw * m;
                if (rt >= nrt || rt < g) continue;   // uniform over the wave
                double2 v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = refl_elem(A, shv, rt * 16 + 4 * q + lk, 16 * g + lr, s);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    wr = mfma16(v[q].x, xr[m][q], wr);
                    wr = mfma16(v[q].y, xi[m][q], wr);
                    wi = mfma16(v[q].x, xi[m][q], wi);
                    wi = mfma16(-v[q].y, xr[m][q], wi);
                }
            }
            // operands of Y = T_g W (wave 0) and of X -= V_g Y, loaded while the partial sums are combined
            double2 tv[4], vd[RTW][4];
            if (wave == 0) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) tv[ks] = Tg[(g * 16 + lr) * 16 + 4 * ks + lk];
            }
#pragma unroll
            for (int m = 0; m < RTW; ++m) {
                const int rt = wave + nw * m;
#pragma unroll
                for (int kq = 0; kq < 4; ++kq)
                    vd[m][kq] = (rt < nrt && rt >= g) ? refl_elem(A, shv, rt * 16 + lr, 16 * g + 4 * kq + lk, s)
                                                      : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) pbuf[wave * 256 + (lk + 4 * q) * 16 + lr] = make_double2(wr[q], wi[q]);
            __syncthreads();
            // wave 0: W = sum of the partial tiles (fixed order), Y = T_g W into ybuf
            if (wave == 0) {
                doublex4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int e = (4 * ks + lk) * 16 + lr;
                    double2 w = pbuf[e];
#pragma unroll
                    for (int w8 = 1; w8 < nw; ++w8) w = cadd(w, pbuf[w8 * 256 + e]);
                    const double2 t = tv[ks];
                    yr = mfma16(t.x, w.x, yr);
                    yr = mfma16(-t.y, w.y, yr);
                    yi = mfma16(t.x, w.y, yi);
                    yi = mfma16(t.y, w.x, yi);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) ybuf[(lk + 4 * q) * 16 + lr] = make_double2(yr[q], yi[q]);
            }
            __syncthreads();
            // B operand of step kq: Y[4 kq + l / 16][l % 16]
            double2 yv[4];
#pragma unroll
            for (int kq = 0; kq < 4; ++kq) yv[kq] = ybuf[(lk + 4 * kq) * 16 + lr];
            // X -= V_g Y
#pragma unroll
            for (int m = 0; m < RTW; ++m) {
                const int rt = wave + nw * m;
                if (rt >= nrt || rt < g) continue;
#pragma unroll
                for (int kq = 0; kq < 4; ++kq) {
                    const double2 v = vd[m][kq];
                    xr[m] = mfma16(-v.x, yv[kq].x, xr[m]);
                    xr[m] = mfma16(v.y, yv[kq].y, xr[m]);
                    xi[m] = mfma16(-v.x, yv[kq].y, xi[m]);
                    xi[m] = mfma16(-v.y, yv[kq].x, xi[m]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < RTW; ++m) {
            const int rt = wave + nw * m;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = rt * 16 + lk + 4 * q;
                if (rt < nrt && row < s && col < r) X[(int64_t)col * s + row] = make_double2(xr[m][q], xi[m][q]);
            }
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Register-resident Householder tridiagonalisation (orders s <= RR_MAXS).
// One workgroup of 768 threads holds the Hermitian matrix in registers as the
// 16 x 16 blocks (I, J), I >= J, of its lower triangle (diagonal blocks held
// in full): wave w owns blocks w, w + 12, ... in column-major block order, in
// the accumulator layout of the FP64 matrix cores (lane l holds column
// J*16 + l%16, rows I*16 + l/16 + 4q, q = 0..3).  Step i:
//  (a) every wave applies the pending rank-2 update of step i-1 to its live
//      blocks as two 16x16x4 MFMAs per block ([u q] times [q u]^H), captures
//      column i+1, and forms the products with u_i: column partials (in-lane,
//      then across the four rows of lanes) and, in off-diagonal blocks, row
//      partials (transposed through a per-wave LDS tile, summed by quads);
//  (b) one thread per row gathers p = A u_i / h_i in a fixed block order;
//      then q = p - (u^H p / 2h) u, column i+1 finished with the update of
//      step i, and the reflector of step i+1.
// Four barriers per step; the matrix never leaves the registers.  Outputs the
// same quantities as the in-memory reduction of k_heig_svt: the reflectors
// u_i below the diagonal of the packed matrix, and per matrix the diagonal,
// the complex off-diagonal and h_i as 4 s doubles at the start of the scratch.
// ---------------------------------------------------------------------------
constexpr int RR_MAXS = 208;
constexpr int RR_THREADS = 768;
constexpr int RR_WAVES = RR_THREADS / 64;
constexpr int RR_TILE = 16 * 17;

__device__ inline int rr_bidx(int I, int J, int nb) { return J * nb - (J * (J - 1)) / 2 + (I - J); }

// Sum of the partials of row 16 I + rr over the blocks t = jlo .. nb-1 of the trailing matrix: row
// partials of blocks (I, t) for t <= I, then column partials of blocks (t, I) for t > I, added in
// that order.  The loads are issued BATCH at a time before their sums (one LDS round trip per
// batch instead of one per block); lanes past the last block load entry 0 and skip the sum.
template <int NBMAX, int BATCH, typename T, typename V>
__device__ inline void gather_partials(const V* yrow, const V* ycol, int I, int rr, int jlo, int nb, T& ax, T& ay) {
    // block indices stepped along t: rr_bidx(I, t + 1) = rr_bidx(I, t) + nb - 1 - t, and
    // rr_bidx(t, I) = rr_bidx(I, I) + t - I
    int bl = rr_bidx(I, jlo, nb);
    const int bu = rr_bidx(I, I, nb) - I;
#pragma unroll
    for (int m0 = 0; m0 < NBMAX; m0 += BATCH) {
        if (jlo + m0 >= nb) break;   // uniform over the block
        V v[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            if (m0 + u < NBMAX) {
                const int t = jlo + m0 + u;
                const bool lower = t <= I;
                const int b = lower ? bl : bu + t;
                v[u] = (lower ? yrow : ycol)[(t < nb ? b : 0) * 16 + rr];
                bl += nb - 1 - t;
            }
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            if (m0 + u < NBMAX && jlo + m0 + u < nb) {
                ax += v[u].x;
                ay += v[u].y;
            }
        }
    }
}

// a - (u_r conj(q_c) + q_r conj(u_c)): one element of the pending Hermitian rank-2 update
__device__ inline double2 rank2_sub(double2 a, double2 ur, double2 qr, double2 uc, double2 qc) {
    a.x = fma(-ur.x, qc.x, a.x);
    a.x = fma(-ur.y, qc.y, a.x);
    a.x = fma(-qr.x, uc.x, a.x);
    a.x = fma(-qr.y, uc.y, a.x);
    a.y = fma(-ur.y, qc.x, a.y);
    a.y = fma(ur.x, qc.y, a.y);
    a.y = fma(-qr.y, uc.x, a.y);
    a.y = fma(qr.x, uc.y, a.y);
    return a;
}


// sum of the NW per-wave partials v[0 .. NW-1] as a fixed pairwise tree (the same value in every thread)
template <int NW>
__device__ inline double tree_sum(const double* v) {
    double a[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) a[i] = v[i];
#pragma unroll
    for (int w = 1; w < NW; w *= 2)
#pragma unroll
        for (int i = 0; i + w < NW; i += 2 * w) a[i] += a[i + w];
    return a[0];
}
// the same total in groups of four (fewer registers at once): ((v0 + v1) + (v2 + v3)) + ...
template <int NW>
__device__ inline double group_sum(const double* v) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < NW; g += 4) {
        double a = v[g];
        if (g + 1 < NW) a += v[g + 1];
        double b = g + 2 < NW ? v[g + 2] : 0.0;
        if (g + 3 < NW) b += v[g + 3];
        t = g == 0 ? a + b : t + (a + b);
    }
    return t;
}

template <int MAXB>
__global__ __launch_bounds__(RR_THREADS) void k_tridiag_rr(const LRDesc* __restrict__ descs, int m0,
                                                              double2* __restrict__ Gs, int64_t g_stride,
                                                              double* __restrict__ scr, int64_t scr_stride) {
    // separate LDS objects, so that the stores of partial sums do not order the vector loads
    constexpr int RR_SP = ((RR_MAXS + 15) / 16) * 16;
    constexpr int RR_NB = RR_SP / 16;
    // operands of the pending update in the lane order of the matrix cores (negated):
    // opA[I][lane] = (a, a') of row I*16 + lane%16, opB[J][lane] = b of column J*16 + lane%16
    __shared__ double2 opA[RR_NB * 64];
    __shared__ double opB[RR_NB * 64];
    __shared__ double2 uc[RR_SP];                 // current reflector u_i
    __shared__ double2 xraw[RR_SP];               // captured column i+1
    // partial products with u of the rows of block-row I: ypart[I][t][16] holds the row partials of
    // block (I, t) for t <= I and the column partials of block (t, I) for t > I, so that row
    // 16 I + rr sums ypart[I][jlo .. nb-1][rr] with fixed strides.  Rows of RR_PS >= nb + 3
    // entries, zero past nb: the sum reads whole batches of four
    constexpr int RR_PS = ((RR_NB + 3 + 3) / 4) * 4;
    __shared__ double2 ypart[RR_NB * RR_PS * 16];
    __shared__ double2 rtile[RR_WAVES * RR_TILE];  // per wave: products of a block, 16 rows of 17
    __shared__ double2 salpha[2];                 // [0] alpha of the reflector, [1] p_j
    __shared__ double red[2 * (RR_THREADS / 64)];  // per-wave partial sums: u^H p, then tails
    __shared__ double rh[2];                      // h of the current reflector and 1 / h
    __shared__ int rrefl;                         // whether the current column is reflected
    const LRDesc dsc = descs[m0 + blockIdx.x];
    const int s = lr_s(dsc);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = (s + 15) >> 4, sp = nb * 16;
    const int nblk = nb * (nb + 1) / 2;
    double2* A = Gs + (int64_t)blockIdx.x * g_stride;
    double* tri = scr + (int64_t)blockIdx.x * scr_stride;   // diag | off re | off im | h
    double* tdd = tri;
    double* ter = tri + s;
    double* tei = tri + 2 * s;
    double* thv = tri + 3 * s;

    // block coordinates of this wave's blocks (column-major block order)
    int bI[MAXB], bJ[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        int b = wave + RR_WAVES * t, J = 0;
        while (J < nb && b >= nb - J) {
            b -= nb - J;
            ++J;
        }
        bJ[t] = J;
        bI[t] = J + b;
    }
    // block (I, J) in the accumulator layout of the FP64 matrix cores: element q of lane l is
    // (row I*16 + l/16 + 4q, column J*16 + l%16); real and imaginary parts in separate registers
    doublex4 ar_[MAXB], ai_[MAXB];
    {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            const bool has = wave + RR_WAVES * t < nblk;
            const int c = bJ[t] * 16 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = bI[t] * 16 + lk + 4 * q;
                double2 v = make_double2(0.0, 0.0);
                if (has && r < s && c < s) {
                    if (r >= c) v = A[pk(r, c, s)];
                    else {
                        v = A[pk(c, r, s)];
                        v.y = -v.y;
                    }
                }
                ar_[t][q] = v.x;
                ai_[t][q] = v.y;
            }
        }
        for (int e = tid; e < sp; e += RR_THREADS) uc[e] = make_double2(0.0, 0.0);
        for (int e = tid; e < RR_NB * RR_PS * 16; e += RR_THREADS) ypart[e] = make_double2(0.0, 0.0);
        for (int e = tid; e < nb * 64; e += RR_THREADS) {
            opA[e] = make_double2(0.0, 0.0);
            opB[e] = 0.0;
        }
        // column 0 into xraw
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            if (wave + RR_WAVES * t < nblk && bJ[t] == 0 && lr == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = bI[t] * 16 + lk + 4 * q;
                    if (r < s) xraw[r] = make_double2(ar_[t][q], ai_[t][q]);
                }
            }
        }
    }
    __syncthreads();

    // Thread t works on row j + t of the current column j (every row count here is below 512).
    // the thread index, recomputed where it is used (the wave index is a scalar), so that no
    // vector register keeps it across the step loop
    auto tid_now = [&]() {
        int ln;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
        return wave * 64 + ln;
    };
    // Reflection of column j, v being this thread's entry (row r = j + t) finished with every update
    // before step j.  norm_part: the diagonal entry, alpha, and the per-wave sums of the squared
    // entries below the subdiagonal.  After a barrier, reflect: the reflector of column j into uc
    // (and the packed matrix), h and whether the column is reflected.
    auto norm_part = [&](int j, int r, double2 v) {
        double tail = 0;
        if (r < s) {
            if (r == j) tdd[j] = v.x;
            if (r == j + 1) salpha[0] = v;
            if (r > j + 1) tail = cabs2(v);
        }
        tail = wave_sum_to63(tail);
        if (((r - j) & 63) == 63) red[RR_THREADS / 64 + wave] = tail;
    };
    auto reflect = [&](int j, int r, double2 v) {
        if (j + 1 >= s) return;
        const double tail = tree_sum<RR_THREADS / 64>(red + RR_THREADS / 64);
        const double2 al = salpha[0];
        const bool refl = tail > 0.0;
        double hh = 1.0, xn = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (refl) {
            // |alpha| and its phase from one reciprocal square root, beside the norm of the column
            const double a2 = al.x * al.x + al.y * al.y;
            xn = sqrt(a2 + tail);
            double aabs = 0.0;
            if (a2 > 0) {
                const double ia = rsqrt(a2);
                ph = make_double2(al.x * ia, al.y * ia);
                aabs = a2 * ia;
            }
            hh = xn * (xn + aabs);
        }
        if (r == j) {
            ter[j] = refl ? -ph.x * xn : al.x;
            tei[j] = refl ? -ph.y * xn : al.y;
            thv[j] = refl ? hh : 0.0;
            // entries at and above the column stay zero (the zero is made here rather than kept
            // in registers across the loop)
            double zx, zy;
            asm volatile("v_mov_b64 %0, 0\n\tv_mov_b64 %1, 0" : "=v"(zx), "=v"(zy));
            uc[j] = make_double2(zx, zy);
            rh[0] = hh;   // 1 / h is formed at the start of the next step, off this chain
            rrefl = refl;
        }
        if (r > j && r < s) {
            double2 u = make_double2(0.0, 0.0);
            if (refl) {
                u = (r == j + 1) ? make_double2(al.x + ph.x * xn, al.y + ph.y * xn) : v;
                A[pk(r, j, s)] = u;
            }
            uc[r] = u;
        }
    };
    // column c of the blocks as they stand (rows c .. s-1) into xraw
    auto capture = [&](int c) {
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            const int b = wave + RR_WAVES * t;
            if (b >= nblk || bJ[t] != (c >> 4)) continue;   // uniform over the wave
            int ln;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
            if ((ln & 15) == (c & 15)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = bI[t] * 16 + (ln >> 4) + 4 * q;
                    if (r >= c && r < s) xraw[r] = make_double2(ar_[t][q], ai_[t][q]);
                }
            }
        }
    };

    {
        const int r = tid_now();
        const double2 v = r < s ? xraw[r] : make_double2(0.0, 0.0);
        norm_part(0, r, v);
        __syncthreads();
        reflect(0, r, v);
        capture(1);   // xraw is no longer read for column 0
    }
    __syncthreads();

    // Step i: the blocks hold the matrix with the updates of steps < i applied, xraw column i+1
    // of it (rows > i), uc the reflector u_i.
    for (int i = 0; i + 1 < s; ++i) {
        const int jlo = (i + 1) >> 4;
        // (a) products of the live blocks with u_i
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            int b = wave + RR_WAVES * t;
            if (b >= nblk || bJ[t] < jlo) continue;   // uniform over the wave
            int I = bI[t], J = bJ[t];
            // keep the block's index arithmetic inside the step (it would otherwise be hoisted
            // into vector registers that the matrix needs); the lane index is recomputed too
            asm volatile("" : "+s"(I), "+s"(J), "+s"(b));
            int ln;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
            const int lr = ln & 15, lk = ln >> 4;
            // column partials conj(A)^T u over the block's rows: in-lane, then across the four rows
            // of lanes; lanes of row 0 end with the real part, lanes of row 1 the imaginary part
            const double2 uC = uc[J * 16 + lr];
            double ycx = 0.0, ycy = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 uR = uc[I * 16 + lk + 4 * q];
                ycx = fma(ar_[t][q], uR.x, fma(ai_[t][q], uR.y, ycx));
                ycy = fma(ar_[t][q], uR.y, fma(-ai_[t][q], uR.x, ycy));
            }
            const double ycs = colsum4_pair(ycx, ycy);
            // a diagonal block is held in full and Hermitian: its column sums are its row sums
            if (lk < 2) reinterpret_cast<double*>(ypart + (J * RR_PS + I) * 16 + lr)[lk] = ycs;
            if (I != J) {
                // row partials A u_C: the lane's products go through a per-wave LDS tile (rows of
                // 17 entries, so that neither pass conflicts on banks); a quad of lanes then sums
                // one row, four columns per lane
                double2* tile = rtile + wave * RR_TILE;
                const int wr = (int)__umul24(lk, 17) + lr;        // row lk, column lr (rows of 17)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    tile[wr + 68 * q] = cmul(make_double2(ar_[t][q], ai_[t][q]), uC);
                __builtin_amdgcn_wave_barrier();
                const int rho = ln >> 2;
                const int rd = (int)__umul24(rho, 17) + ((ln & 3) << 2);   // row rho, columns 4 (ln % 4) ..
                double2 rs = tile[rd];
#pragma unroll
                for (int m = 1; m < 4; ++m) {
                    const double2 v = tile[rd + m];
                    rs.x += v.x;
                    rs.y += v.y;
                }
                __builtin_amdgcn_wave_barrier();
                rs = quad_sum_z(rs);
                if ((ln & 3) == 0) ypart[(I * RR_PS + J) * 16 + rho] = rs;
            }
        }
        // 1 / h of the reflector of step i, for (b); formed here by the first wave (the least loaded)
        if (wave == 0) {
            const double ih = 1.0 / rh[0];
            if ((threadIdx.x & 63) == 0) rh[1] = ih;
        }
        __syncthreads();
        // (b) p = A u_i / h and u^H p over all threads, then q_i, column i+1 finished with the
        // update of step i, and the next reflector.
        {
            const int j = i + 1;
            const int r = j + tid_now();
            const bool refl = rrefl != 0;
            const double ihh = rh[1];
            const bool live = r < s;
            const double2 zero = make_double2(0.0, 0.0);
            const double2 ur = (live && refl) ? uc[r] : zero;
            double2 pv = zero;
            double uhp = 0;
            if (live && refl) {
                // row partials of blocks (I, jlo .. I), then column partials of blocks (I + 1 .. nb-1, I)
                // (in batches of four loads; entries past nb are zero)
                const double2* yp = ypart + ((r >> 4) * RR_PS + jlo) * 16 + (r & 15);
                const int nt = nb - jlo;   // uniform over the block
#pragma unroll
                for (int t0 = 0; t0 < RR_PS; t0 += 4) {
                    if (t0 >= nt) break;
                    double2 y[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) y[u] = yp[(t0 + u) * 16];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        pv.x += y[u].x;
                        pv.y += y[u].y;
                    }
                }
                pv.x *= ihh;
                pv.y *= ihh;
                uhp = ur.x * pv.x + ur.y * pv.y;   // Re(conj(u) p)
                if (r == j) salpha[1] = pv;
            }
            uhp = wave_sum_to63(uhp);
            if (((r - j) & 63) == 63) red[wave] = uhp;
            __syncthreads();
            const double2 xr = live ? xraw[r] : zero;
            const double2 u0 = uc[j];
            const double2 pj = salpha[1];
            uhp = group_sum<RR_THREADS / 64>(red);
            const double Kc = 0.5 * uhp * ihh;   // u^H p / 2h
            double2 qj = zero;
            if (refl) qj = make_double2(pj.x - Kc * u0.x, pj.y - Kc * u0.y);
            double2 v = xr;
            if (live) {
                const double2 q = make_double2(pv.x - Kc * ur.x, pv.y - Kc * ur.y);
                // the update D -= [u_r q_r] [q_c u_c]^H as 16x16x4 products: lane (k, c) supplies
                // A[c][k] = (u.x, u.y, q.x, q.y)[k] of row c (and A'[c][k] = (u.y, -u.x, q.y, -q.x)[k]
                // for the imaginary part) and B[k][c] = (q.x, q.y, u.x, u.y)[k] of column c
                const int o = (r >> 4) * 64 + (r & 15);
                opA[o] = make_double2(-ur.x, -ur.y);
                opA[o + 16] = make_double2(-ur.y, ur.x);
                opA[o + 32] = make_double2(-q.x, -q.y);
                opA[o + 48] = make_double2(-q.y, q.x);
                opB[o] = q.x;
                opB[o + 16] = q.y;
                opB[o + 32] = ur.x;
                opB[o + 48] = ur.y;
                // column i+1 minus the update of step i: v -= q conj(u_j) + u conj(q_j)
                if (refl) {
                    v.x -= q.x * u0.x + q.y * u0.y + ur.x * qj.x + ur.y * qj.y;
                    v.y -= q.y * u0.x - q.x * u0.y + ur.y * qj.x - ur.x * qj.y;
                }
            }
            norm_part(j, r, v);
            __syncthreads();
            // the reflector of column i+1 (waves that hold rows of it), then the update of step i,
            // D -= [u_i q_i] [q_i u_i]^H, on the matrix cores by every wave for the blocks live in
            // step i+1 (the entries of u, q at and above the reduced columns are zero, so the stale
            // values there never reach a live product), and the capture of column i+2
            if (j + wave * 64 < s) reflect(j, r, v);
            if (i + 2 < s) {
                const int jlo2 = (i + 2) >> 4;
#pragma unroll
                for (int t = 0; t < MAXB; ++t) {
                    int b = wave + RR_WAVES * t;
                    if (b >= nblk || bJ[t] < jlo2) continue;   // uniform over the wave
                    int I = bI[t], J = bJ[t];
                    asm volatile("" : "+s"(I), "+s"(J), "+s"(b));
                    int ln;
                    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
                    const double2 a = opA[I * 64 + ln];
                    const double bq = opB[J * 64 + ln];
                    ar_[t] = mfma16(a.x, bq, ar_[t]);
                    ai_[t] = mfma16(a.y, bq, ai_[t]);
                }
                capture(i + 2);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The same reduction with the matrix held in FP32 (the mixed form's forward
// iterations, whose Gram matrices come from FP32 products).  Half the registers
// per matrix let two workgroups of 512 threads share a compute unit (at most 128
// registers per thread: four waves per SIMD, two of each workgroup), so that the
// serial part of one matrix's step (the gather, the two reductions over all
// threads and the reflector) overlaps the block products of the other's.  Blocks
// sit in the accumulator layout of the FP32 matrix cores (lane l holds column
// J*16 + l%16, rows I*16 + 4(l/16) + r, r = 0..3); the update is two 16x16x4
// FP32 MFMAs per block with the operands of the FP64 form.  Scalars (norms, h,
// u^H p, q, the finished column) are formed in FP64 from the FP32 sums; the
// reflector is rounded to FP32 once, and the rounded vector is both the one the
// matrix is updated with and the one written out.  Outputs as k_tridiag_rr.
// ---------------------------------------------------------------------------
// two shapes: 512 threads for orders up to 208 (two workgroups per CU), and 1024 threads for
// orders 209 .. 256 (one workgroup per CU, still at most 128 registers per thread)
constexpr int RR32_MAXS_WIDE = 256;

template <int CTRL>
__device__ inline float dpp_move_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
// colsum4_pair for single precision: lanes of rows 0 and 2 end with the sum of x over the
// four rows of 16 lanes, lanes of rows 1 and 3 with the sum of y
__device__ inline float colsum4_pair_f(float x, float y) {
    const auto a = __builtin_amdgcn_permlane16_swap((unsigned)__float_as_int(x), (unsigned)__float_as_int(y),
                                                    false, false);
    const float c = __int_as_float((int)a[0]) + __int_as_float((int)a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap((unsigned)__float_as_int(c), (unsigned)__float_as_int(c),
                                                    false, false);
    return __int_as_float((int)b[0]) + __int_as_float((int)b[1]);
}

template <int MAXB, int NTHR, int MAXS>
__global__ __launch_bounds__(NTHR, 4) void k_tridiag_rr32(const LRDesc* __restrict__ descs, int m0,
                                                                  double2* __restrict__ Gs, int64_t g_stride,
                                                                  double* __restrict__ scr, int64_t scr_stride) {
    constexpr int RR32_THREADS = NTHR, RR32_WAVES = NTHR / 64;
    constexpr int RR_SP = ((MAXS + 15) / 16) * 16;
    constexpr int RR_NB = RR_SP / 16, RR_NBLK = RR_NB * (RR_NB + 1) / 2;
    __shared__ float2 opA[RR_NB * 64];              // update operands in lane order (negated), as above
    __shared__ float opB[RR_NB * 64];
    __shared__ double2 qp[RR_SP];                   // pending q, read back by the thread that wrote it
    __shared__ float2 uc[RR_SP];                    // current reflector (FP32-rounded)
    __shared__ double2 xraw[RR_SP];                 // captured column i+1
    __shared__ float2 yrow[RR_NBLK * 16];           // [block][16] row partials
    __shared__ float2 ycol[RR_NBLK * 16];           // [block][16] column partials
    __shared__ double2 salpha[2];
    __shared__ double red[2 * RR32_WAVES];
    __shared__ double rh[2];
    __shared__ int rrefl;
    const LRDesc dsc = descs[m0 + blockIdx.x];
    const int s = lr_s(dsc);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = (s + 15) >> 4, sp = nb * 16;
    const int nblk = nb * (nb + 1) / 2;
    double2* A = Gs + (int64_t)blockIdx.x * g_stride;
    double* tri = scr + (int64_t)blockIdx.x * scr_stride;   // diag | off re | off im | h
    double* tdd = tri;
    double* ter = tri + s;
    double* tei = tri + 2 * s;
    double* thv = tri + 3 * s;

    int bI[MAXB], bJ[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        int b = wave + RR32_WAVES * t, J = 0;
        while (J < nb && b >= nb - J) {
            b -= nb - J;
            ++J;
        }
        bJ[t] = J;
        bI[t] = J + b;
    }
    floatx4 ar_[MAXB], ai_[MAXB];
    {
        const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            const bool has = wave + RR32_WAVES * t < nblk;
            const int c = bJ[t] * 16 + lr;
            // branch-free with 32-bit packed indices (orders up to MAXS): every lane loads a
            // valid entry (the upper triangle as the conjugate of the lower one), and entries
            // outside the matrix are zeroed after the load
            double2 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = bI[t] * 16 + 4 * lg + q;
                const int hi = max(r, c), lo = min(r, c);
                const bool ok = has && hi < s;
                const int e = (int)((unsigned)(lo * (2 * s - lo - 1)) >> 1) + hi;
                v[q] = A[ok ? e : 0];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = bI[t] * 16 + 4 * lg + q;
                const bool ok = has && r < s && c < s;
                float xr = ok ? (float)v[q].x : 0.f;
                float xi = ok ? (r >= c ? (float)v[q].y : -(float)v[q].y) : 0.f;
                // converted here, so that no FP64 load result stays live until the step loop
                asm volatile("" : "+v"(xr), "+v"(xi));
                ar_[t][q] = xr;
                ai_[t][q] = xi;
            }
            // one block of FP64 loads in flight at a time, so that the load results fit in registers
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int e = tid; e < sp; e += RR32_THREADS) {
            qp[e] = make_double2(0.0, 0.0);
            uc[e] = make_float2(0.f, 0.f);
        }
        for (int e = tid; e < nb * 64; e += RR32_THREADS) {
            opA[e] = make_float2(0.f, 0.f);
            opB[e] = 0.f;
        }
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            if (wave + RR32_WAVES * t < nblk && bJ[t] == 0 && lr == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = bI[t] * 16 + 4 * lg + q;
                    if (r < s) xraw[r] = make_double2(ar_[t][q], ai_[t][q]);
                }
            }
        }
    }
    __syncthreads();

    auto tid_now = [&]() {
        int ln;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
        return wave * 64 + ln;
    };
    // column j minus the update of step j-1, its diagonal entry, and the reflector of column j
    auto finish_and_reflect = [&](int j, bool pending, double2 q_j) {
        const int tl = tid_now();
        const int r = j + tl;
        double tail = 0;
        if (r < s) {
            double2 v = xraw[r];
            if (pending) {
                const float2 u0f = uc[j], urf = uc[r];
                const double2 u0 = make_double2(u0f.x, u0f.y), ur = make_double2(urf.x, urf.y);
                const double2 qr = qp[r];
                v.x -= qr.x * u0.x + qr.y * u0.y + ur.x * q_j.x + ur.y * q_j.y;
                v.y -= qr.y * u0.x - qr.x * u0.y + ur.y * q_j.x - ur.x * q_j.y;
            }
            xraw[r] = v;
            if (r == j) tdd[j] = v.x;
            if (r == j + 1) salpha[0] = v;
            if (r > j + 1) tail = cabs2(v);
        }
        tail = wave_sum_to63(tail);
        if ((tl & 63) == 63) red[RR32_WAVES + wave] = tail;
        __syncthreads();
        if (j + 1 >= s) return;
        tail = 0;
        for (int w = 0; w < RR32_WAVES; ++w) tail += red[RR32_WAVES + w];
        const double2 al = salpha[0];
        const bool refl = tail > 0.0;
        double hh = 1.0, xn = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (refl) {
            // reciprocals by the hardware estimate and a Newton step (FP32-accurate data)
            const double a2 = al.x * al.x + al.y * al.y;
            const double aabs = sqrt(a2);
            xn = sqrt(a2 + tail);
            if (aabs > 0) {
                const double ia = rcp_nr(aabs);
                ph = make_double2(al.x * ia, al.y * ia);
            }
            hh = xn * xn + aabs * xn;
        }
        if (tl == 0) {
            ter[j] = refl ? -ph.x * xn : al.x;
            tei[j] = refl ? -ph.y * xn : al.y;
            thv[j] = refl ? hh : 0.0;
        }
        if (r >= j && r < s) {
            float2 u = make_float2(0.f, 0.f);   // entry j of the reflector is zero
            if (refl && r > j) {
                const double2 ud = (r == j + 1) ? make_double2(al.x + ph.x * xn, al.y + ph.y * xn) : xraw[r];
                u = make_float2((float)ud.x, (float)ud.y);
                A[pk(r, j, s)] = make_double2(u.x, u.y);
            }
            uc[r] = u;
        }
        if (tl == 0) {
            rh[0] = hh;
            rh[1] = rcp_nr(hh);
            rrefl = refl;
        }
    };

    finish_and_reflect(0, false, make_double2(0.0, 0.0));
    __syncthreads();

    for (int i = 0; i + 1 < s; ++i) {
        const int jlo = (i + 1) >> 4;
        const bool pend = i > 0;
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            int b = wave + RR32_WAVES * t;
            if (b >= nblk || bJ[t] < jlo) continue;   // uniform over the wave
            int I = bI[t], J = bJ[t];
            asm volatile("" : "+s"(I), "+s"(J), "+s"(b));
            int ln;
            asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
            const int lr = ln & 15, lg = ln >> 4;
            if (pend) {
                const float2 a = opA[I * 64 + ln];
                const float bq = opB[J * 64 + ln];
                ar_[t] = mfma16(a.x, bq, ar_[t]);
                ai_[t] = mfma16(a.y, bq, ai_[t]);
            }
            const int cc = i + 1 - J * 16;
            if (cc >= 0 && cc < 16 && lr == cc) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = I * 16 + 4 * lg + q;
                    if (r > i && r < s) xraw[r] = make_double2(ar_[t][q], ai_[t][q]);
                }
            }
            // column partials conj(A)^T u: in-lane over the lane's four rows, then across the
            // four rows of lanes (real part to row 0 of lanes, imaginary part to row 1)
            const float2 uC = uc[J * 16 + lr];
            float ycx = 0.f, ycy = 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float2 uR = uc[I * 16 + 4 * lg + q];
                ycx = fmaf(ar_[t][q], uR.x, fmaf(ai_[t][q], uR.y, ycx));
                ycy = fmaf(ar_[t][q], uR.y, fmaf(-ai_[t][q], uR.x, ycy));
            }
            const float ycs = colsum4_pair_f(ycx, ycy);
            float2* ydst = I == J ? yrow : ycol;
            if (lg < 2) reinterpret_cast<float*>(ydst + b * 16 + lr)[lg] = ycs;
            if (I != J) {
                // row partials A u_C over the 16 lanes of each row of lanes, reduce-scatter: lanes
                // exchange with lane ^ 8 (rotate by 8), then with the mirror lane in each half,
                // then within quads; lane l ends with row 4(l/16) + (l%16)/4
                float2 y[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) y[q] = cmul(make_float2(ar_[t][q], ai_[t][q]), uC);
                const bool hi8 = (lr & 8) != 0, hi4 = (lr & 4) != 0;
                const float2 sA = hi8 ? y[0] : y[2], sB = hi8 ? y[1] : y[3];
                float2 kA = hi8 ? y[2] : y[0], kB = hi8 ? y[3] : y[1];
                kA.x += dpp_move_f<0x128>(sA.x);
                kA.y += dpp_move_f<0x128>(sA.y);
                kB.x += dpp_move_f<0x128>(sB.x);
                kB.y += dpp_move_f<0x128>(sB.y);
                const float2 s2 = hi4 ? kA : kB;
                float2 k2 = hi4 ? kB : kA;
                k2.x += dpp_move_f<0x141>(s2.x);
                k2.y += dpp_move_f<0x141>(s2.y);
                k2.x += dpp_move_f<0xB1>(k2.x);
                k2.y += dpp_move_f<0xB1>(k2.y);
                k2.x += dpp_move_f<0x4E>(k2.x);
                k2.y += dpp_move_f<0x4E>(k2.y);
                if ((lr & 3) == 0) yrow[b * 16 + 4 * lg + (lr >> 2)] = k2;
            }
        }
        __syncthreads();
        // the serial part of the step (gather, the two reductions, the reflector) runs at raised
        // wave priority, ahead of the block products of the other matrix on the compute unit
        __builtin_amdgcn_s_setprio(2);
        {
            const int j = i + 1;
            const int tl = tid_now();
            const int r = j + tl;
            const bool refl = rrefl != 0;
            const double hh = rh[0], ihh = rh[1];
            double2 pv = make_double2(0.0, 0.0);
            double uhp = 0;
            if (r < s && refl) {
                const int I = r >> 4, rr = r & 15;
                float ax = 0.f, ay = 0.f;
                gather_partials<RR_NB, 8>(yrow, ycol, I, rr, jlo, nb, ax, ay);
                const float2 acc = make_float2(ax, ay);
                pv = make_double2(acc.x * ihh, acc.y * ihh);
                const float2 u = uc[r];
                uhp = u.x * pv.x + u.y * pv.y;
                if (r == j) salpha[1] = pv;
            }
            uhp = wave_sum_to63(uhp);
            if ((tl & 63) == 63) red[wave] = uhp;
            __syncthreads();
            uhp = 0;
            for (int w = 0; w < RR32_WAVES; ++w) uhp += red[w];
            const double Kc = 0.5 * uhp * ihh;
            double2 qj = make_double2(0.0, 0.0);
            if (refl) {
                const double2 pj = salpha[1];
                const float2 uj = uc[j];
                qj = make_double2(pj.x - Kc * uj.x, pj.y - Kc * uj.y);
            }
            if (r < s) {
                const float2 uf = refl ? uc[r] : make_float2(0.f, 0.f);
                const double2 u = make_double2(uf.x, uf.y);
                const double2 q = make_double2(pv.x - Kc * u.x, pv.y - Kc * u.y);
                qp[r] = q;
                const float qx = (float)q.x, qy = (float)q.y;
                const int o = (r >> 4) * 64 + (r & 15);
                opA[o] = make_float2(-uf.x, -uf.y);
                opA[o + 16] = make_float2(-uf.y, uf.x);
                opA[o + 32] = make_float2(-qx, -qy);
                opA[o + 48] = make_float2(-qy, qx);
                opB[o] = qx;
                opB[o + 16] = qy;
                opB[o + 32] = uf.x;
                opB[o + 48] = uf.y;
            }
            finish_and_reflect(j, refl, qj);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
}

template <typename OC, int SL>
__global__ __launch_bounds__(EIG_THREADS, SL >= 5 ? 2 : 4) void k_heig_svt(const LRDesc* __restrict__ descs, int m0,
                                                             double2* __restrict__ Gs, int64_t g_stride,
                                                             OC* __restrict__ Ss, int64_t s_stride,
                                                             double* __restrict__ scr, int64_t scr_stride,
                                                             int32_t* __restrict__ ranks, double ortol_rel,
                                                             uint32_t* __restrict__ flags, int smax,
                                                             VjpArgs<OC> vj, int tri_in, double resid_lim) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int UNR = SL <= 3 ? 4 : (SL == 4 ? 3 : 2);   // columns per wave with loads in flight
    const LRDesc dsc = descs[m0 + blockIdx.x];
    const int s = lr_s(dsc);
    const double thr = dsc.thr;
    const int tid = threadIdx.x;
    const int nw = EIG_THREADS / 64;
    const int lane = tid & 63, wave = tid >> 6;
    // LDS: region A (tridiagonalisation work, later staging) + small persistent arrays
    double2* uvec = reinterpret_cast<double2*>(smem_raw);
    double2* pvec = uvec + smax;
    double2* up = pvec + smax;
    double2* qp = up + smax;
    double2* pcol = qp + smax;
    double2* xraw = pcol + smax;
    double2* prow = xraw + smax;                       // nw * smax
    double2* stage = uvec;                             // region A reused: EIG_STAGE * smax double2
    double* sdd = reinterpret_cast<double*>(uvec + heig_region_a(smax));
    double* se2 = sdd + smax;
    double* see = se2 + smax;
    double* shv = see + smax;
    double* secr = shv + smax;
    double* seci = secr + smax;
    double* sdre = seci + smax;
    double* sdim = sdre + smax;
    double* slam = sdim + smax;
    double* red = slam + smax;                         // nw
    double* red2 = red + nw;                           // nw
    double* sh = red2 + nw;                            // 8
    double2* A = Gs + (int64_t)blockIdx.x * g_stride;   // packed lower triangle
    OC* S = Ss + (int64_t)blockIdx.x * s_stride;
    double* base = scr + (int64_t)blockIdx.x * scr_stride;
    double* W = base + 16 * s + 64;    // s x s, column k: tridiagonal eigenvector k
    double* LU = W + (int64_t)s * s;   // 2*s*s: X (double2, column-major) of the back-transform

    if (tri_in) {
        // reduced by k_tridiag_rr: diagonal, complex off-diagonal and h_i at the start of the scratch
        for (int t = tid; t < s; t += EIG_THREADS) {
            sdd[t] = base[t];
            secr[t] = base[s + t];
            seci[t] = base[2 * s + t];
            shv[t] = base[3 * s + t];
        }
        __syncthreads();
    } else {
        // ---- 1. tridiagonalisation ---------------------------------------------
        // Step i: x = column i below the diagonal, P_i = I - u u^H / h maps x to
        // -phase |x| e_1, and the trailing block becomes A - u q^H - q u^H with
        // p = A u / h, q = p - (u^H p / 2h) u.  The rank-2 update of step i is
        // applied lazily during the Hermitian matrix-vector product of step i+1,
        // which reads (and writes back) only the lower triangle, one column per
        // wave with lanes over rows (coalesced).  The column that step i+1 reduces
        // is captured during that sweep and finished in LDS, so each step makes a
        // single round trip to memory.
        double2* xcur = uvec;                      // x_i, then u_i
        double2* xnxt = pvec;                      // x_{i+1} being formed
        bool pend = false;
        double part = 0;
        for (int t = tid; t + 1 < s; t += EIG_THREADS) {
            const double2 v = A[pk(1 + t, 0, s)];
            xcur[t] = v;
            if (t > 0) part += cabs2(v);
        }
        if (tid == 0) sdd[0] = A[pk(0, 0, s)].x;
        double tail = block_sum(part, red);
        for (int i = 0; i + 1 < s; ++i) {
            const int ni = s - i - 1;
            const double2 alpha = xcur[0];
            const bool refl = tail > 0.0;
            double hh = 1.0;
            double2 ph = make_double2(1.0, 0.0);
            double xn = 0.0;
            if (refl) {
                const double aabs = sqrt(cabs2(alpha));
                xn = sqrt(aabs * aabs + tail);
                if (aabs > 0) ph = make_double2(alpha.x / aabs, alpha.y / aabs);
                hh = xn * xn + aabs * xn;
            }
            __syncthreads();   // every thread has read xcur[0]
            if (tid == 0) {
                if (refl) {
                    xcur[0] = make_double2(alpha.x + ph.x * xn, alpha.y + ph.y * xn);
                    secr[i] = -ph.x * xn;
                    seci[i] = -ph.y * xn;
                    shv[i] = hh;
                } else {
                    secr[i] = alpha.x;
                    seci[i] = alpha.y;
                    shv[i] = 0.0;
                }
            }
            __syncthreads();
            // fused sweep: trailing block -= pending update (written back); p = A u;
            // column i+1 captured into xraw.  UNR columns per wave at a time with all
            // their loads issued first; slots outside a column are skipped.
            double2 accr[SL];
    #pragma unroll
            for (int sl = 0; sl < SL; ++sl) accr[sl] = make_double2(0.0, 0.0);
            double wur = 0;   // this wave's share of u^H (h p)
            const int ncol = (pend || refl) ? ni : 1;
            for (int tc0 = wave; tc0 < ncol; tc0 += UNR * nw) {
                double2 av[UNR][SL];
    #pragma unroll
                for (int uu = 0; uu < UNR; ++uu) {
                    const int tc = tc0 + uu * nw;
    #pragma unroll
                    for (int sl = 0; sl < SL; ++sl) {
                        const int t = sl * 64 + lane;
                        av[uu][sl] = make_double2(0.0, 0.0);
                        if (tc < ncol && t >= tc && t < ni) av[uu][sl] = A[pk(i + 1 + t, i + 1 + tc, s)];
                    }
                }
                double pcr[UNR], pci[UNR];
    #pragma unroll
                for (int uu = 0; uu < UNR; ++uu) {
                    pcr[uu] = 0;
                    pci[uu] = 0;
                    const int tc = tc0 + uu * nw;
                    if (tc >= ncol) continue;   // uniform across the wave
                    const int c = i + 1 + tc;
                    const double2 uc = refl ? xcur[tc] : make_double2(0.0, 0.0);
                    double2 upc = make_double2(0.0, 0.0), qpc = make_double2(0.0, 0.0);
                    if (pend) { upc = up[c]; qpc = qp[c]; }
    #pragma unroll
                    for (int sl = 0; sl < SL; ++sl) {
                        const int t = sl * 64 + lane;
                        if (t >= tc && t < ni) {
                            const int r = i + 1 + t;
                            double2 a = av[uu][sl];
                            if (pend) {
                                const double2 qr = qp[r], ur = up[r];
                                a.x -= qr.x * upc.x + qr.y * upc.y + ur.x * qpc.x + ur.y * qpc.y;
                                a.y -= qr.y * upc.x - qr.x * upc.y + ur.y * qpc.x - ur.x * qpc.y;
                                if (tc > 0) A[pk(r, c, s)] = a;   // column i+1 is finished in LDS instead
                            }
                            if (tc == 0) xraw[t] = a;
                            if (refl) {
                                accr[sl].x += a.x * uc.x - a.y * uc.y;
                                accr[sl].y += a.x * uc.y + a.y * uc.x;
                                if (t > tc) {
                                    const double2 ut = xcur[t];
                                    pcr[uu] += a.x * ut.x + a.y * ut.y;   // conj(a) * u_t
                                    pci[uu] += a.x * ut.y - a.y * ut.x;
                                }
                            }
                        }
                    }
                }
                if (refl) {
    #pragma unroll
                    for (int uu = 0; uu < UNR; ++uu) {
                        pcr[uu] = wave_sum_to63(pcr[uu]);
                        pci[uu] = wave_sum_to63(pci[uu]);
                    }
                    if (lane == 63) {
    #pragma unroll
                        for (int uu = 0; uu < UNR; ++uu) {
                            const int tc = tc0 + uu * nw;
                            if (tc < ncol) {
                                const double2 uc = xcur[tc];
                                pcol[tc] = make_double2(pcr[uu], pci[uu]);
                                wur += uc.x * pcr[uu] + uc.y * pci[uu];   // conj(u_tc) * pcol[tc]
                            }
                        }
                    }
                }
            }
            if (refl) {
    #pragma unroll
                for (int sl = 0; sl < SL; ++sl) {
                    const int t = sl * 64 + lane;
                    if (t < ni) {
                        prow[wave * smax + t] = accr[sl];
                        const double2 ut = xcur[t];
                        wur += ut.x * accr[sl].x + ut.y * accr[sl].y;
                    }
                }
                wur = wave_sum_to63(wur);
                if (lane == 63) red2[wave] = wur;
            }
            __syncthreads();
            // p, q = p - K u (the new pending update), u stored for the back-transform,
            // and x_{i+1} = column i+1 with this step's update, plus its tail norm
            double Kc = 0.0;
            double2 q0 = make_double2(0.0, 0.0);
            const double2 u0 = refl ? xcur[0] : make_double2(0.0, 0.0);
            if (refl) {
                double uhp = 0;
                for (int w = 0; w < nw; ++w) uhp += red2[w];
                Kc = uhp / (2.0 * hh * hh);
                double pr = pcol[0].x, pi = pcol[0].y;
                for (int w = 0; w < nw; ++w) {
                    pr += prow[w * smax].x;
                    pi += prow[w * smax].y;
                }
                q0 = make_double2(pr / hh - Kc * u0.x, pi / hh - Kc * u0.y);
            }
            part = 0;
            for (int t = tid; t < ni; t += EIG_THREADS) {
                const int r = i + 1 + t;
                double2 u = make_double2(0.0, 0.0), q = make_double2(0.0, 0.0);
                if (refl) {
                    u = xcur[t];
                    double pr = pcol[t].x, pi = pcol[t].y;
                    for (int w = 0; w < nw; ++w) {
                        pr += prow[w * smax + t].x;
                        pi += prow[w * smax + t].y;
                    }
                    q = make_double2(pr / hh - Kc * u.x, pi / hh - Kc * u.y);
                    up[r] = u;
                    qp[r] = q;
                    A[pk(r, i, s)] = u;
                }
                double2 x = xraw[t];
                // (q_r conj(u_c) + u_r conj(q_c)) at c = i + 1
                x.x -= q.x * u0.x + q.y * u0.y + u.x * q0.x + u.y * q0.y;
                x.y -= q.y * u0.x - q.x * u0.y + u.y * q0.x - u.x * q0.y;
                if (t == 0) sdd[i + 1] = x.x;
                else {
                    xnxt[t - 1] = x;
                    if (t > 1) part += cabs2(x);
                }
            }
            tail = block_sum(part, red);   // its barriers also publish xnxt, up, qp
            double2* tmp = xcur;
            xcur = xnxt;
            xnxt = tmp;
            pend = refl;
        }
        __syncthreads();
    }

    // ---- 2. real tridiagonal via a diagonal unitary ------------------------------
    // |e_i|, |e_i|^2 and the unit phase of each off-diagonal in parallel, then their
    // prefix product (one thread) and the Gershgorin bounds (block reductions).
    for (int t = tid; t < s; t += EIG_THREADS) {
        double m = 0.0, ur = 1.0, ui = 0.0;
        if (t + 1 < s) {
            const double er = secr[t], ei = seci[t];
            m = sqrt(er * er + ei * ei);
            if (m > 0) {
                ur = er / m;
                ui = ei / m;
            }
        }
        see[t] = m;
        se2[t] = m * m;
        sdre[t + 1 < s ? t + 1 : 0] = t + 1 < s ? ur : 1.0;   // unit phase of e_t, at t + 1
        sdim[t + 1 < s ? t + 1 : 0] = t + 1 < s ? ui : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double pr = 1.0, pi = 0.0;
        sdre[0] = 1.0;
        sdim[0] = 0.0;
        int i = 1;
        for (; i + 3 < s; i += 4) {
            const double a0 = sdre[i], b0 = sdim[i], a1 = sdre[i + 1], b1 = sdim[i + 1];
            const double a2 = sdre[i + 2], b2 = sdim[i + 2], a3 = sdre[i + 3], b3 = sdim[i + 3];
            double nr = pr * a0 - pi * b0, ni = pr * b0 + pi * a0;
            sdre[i] = nr;
            sdim[i] = ni;
            pr = nr * a1 - ni * b1;
            pi = nr * b1 + ni * a1;
            sdre[i + 1] = pr;
            sdim[i + 1] = pi;
            nr = pr * a2 - pi * b2;
            ni = pr * b2 + pi * a2;
            sdre[i + 2] = nr;
            sdim[i + 2] = ni;
            pr = nr * a3 - ni * b3;
            pi = nr * b3 + ni * a3;
            sdre[i + 3] = pr;
            sdim[i + 3] = pi;
        }
        for (; i < s; ++i) {
            const double a = sdre[i], b = sdim[i];
            const double nr = pr * a - pi * b, ni = pr * b + pi * a;
            pr = nr;
            pi = ni;
            sdre[i] = pr;
            sdim[i] = pi;
        }
    }
    {
        double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0, nonfin = 0.0;
        for (int t = tid; t < s; t += EIG_THREADS) {
            const double off = (t > 0 ? see[t - 1] : 0.0) + see[t];
            gl = fmin(gl, sdd[t] - off);
            gu = fmax(gu, sdd[t] + off);
            emax2 = fmax(emax2, se2[t]);
            if (!isfinite(sdd[t]) || !isfinite(se2[t])) nonfin = 1.0;
        }
        gl = -block_max(-gl, red);
        gu = block_max(gu, red);
        emax2 = block_max(emax2, red);
        nonfin = block_max(nonfin, red);
        if (tid == 0) {
            const double tnorm = nonfin > 0 ? INFINITY : fmax(fabs(gl), fabs(gu));
            sh[0] = gl;
            sh[1] = gu;
            sh[2] = tnorm;
            sh[3] = DBL_MIN * fmax(1.0, emax2) * 4.0 + DBL_MIN;
        }
    }
    __syncthreads();
    const double gu = sh[1], tnorm = sh[2], pivmin = sh[3];
    const bool bad = !(tnorm < DBL_MAX);  // NaN or Inf in the Gram matrix
    const double t2 = thr * thr;

    // ---- 3. eigenvalues above thr^2: multisection ---------------------------------
    // A group of G lanes (a power of two <= 64) brackets one eigenvalue: each
    // lane counts at one of G interior points, which shrinks the bracket by a
    // factor G + 1 per round.
    int nabove = 0;
    if (!bad) nabove = s - sturm_count(sdd, se2, s, t2, pivmin);
    {
        // at most 256 lanes count at once: with two workgroups per CU, half the block's lanes and
        // two more rounds take less time than every lane (the counts are issue-bound)
        int G = 64;
        while (G > 1 && G * nabove > EIG_THREADS / 2) G >>= 1;
        const int ngroups = EIG_THREADS / G;
        const int grp = tid / G, gl_ = tid % G;
        const double slack = 2.0 * DBL_EPSILON * tnorm + pivmin;
        // relative width at which a bracket is final: full FP64 accuracy for FP64 outputs and for the
        // derivative (its resolvent solves sit next to each eigenvalue); 1e-10 when S is rounded to
        // FP32, which is far below the FP32 rounding of the products around it
        const double bw = (sizeof(OC) == sizeof(double2) || vj.C != nullptr) ? 2.0 * DBL_EPSILON : 1e-10;
        for (int k0 = 0; k0 < nabove; k0 += ngroups) {   // uniform trip count
            const int kk = k0 + grp;
            const bool act = kk < nabove;
            const int idx = s - nabove + (act ? kk : 0);   // ascending index
            double lo = t2, hi = gu + slack + fabs(gu) * 4.0 * DBL_EPSILON;
            for (int it = 0; it < 80; ++it) {
                const double width = hi - lo;
                bool done = !(width > bw * fmax(fabs(lo), fabs(hi)) + pivmin);
                // the whole wave iterates while any of its groups is active
                const double step = width / (double)(G + 1);
                const double x = lo + step * (double)(gl_ + 1);
                int le = (act && !done && x > lo && x < hi) ? (sturm_count(sdd, se2, s, x, pivmin) <= idx) : 1;
                // number of points with count <= idx in the group (counts are monotone in x)
                int nle = le;
                for (int off = 1; off < G; off <<= 1) nle += __shfl_xor(nle, off, 64);
                if (!done) {
                    const double nlo = nle > 0 ? lo + step * (double)nle : lo;
                    const double nhi = nle < G ? lo + step * (double)(nle + 1) : hi;
                    if (!(nlo > lo || nhi < hi)) done = true;   // no progress possible
                    lo = nlo;
                    hi = fmin(nhi, hi);
                }
                const bool any = __any(!done && act);
                if (!any) break;
            }
            if (act && gl_ == 0) slam[kk] = 0.5 * (lo + hi);
        }
    }
    __syncthreads();

    // ---- 4. eigenvectors by twisted factorisation ---------------------------------
    // For an accurate eigenvalue lk of the tridiagonal T (diagonal sdd, off-
    // diagonal see): T - lk I = L D+ L^T (forward) = U D- U^T (backward);
    // gamma_i = D+_i + D-_i - (d_i - lk) is smallest at the twist r, and
    // z_r = 1, z_i = -L_i z_{i+1} (i < r), z_{i+1} = -U_i z_i (i >= r) solves
    // (T - lk I) z = gamma_r e_r, with L_i = e_i / D+_i and U_i = e_i / D-_{i+1}.
    // Eigenvalues closer than ortol form a cluster.  The first member of every
    // cluster and every single eigenvalue get their vector in parallel, one
    // thread each; D+ and U of each thread of a batch live in LDS region A
    // (2 s + 1 doubles, odd stride against bank conflicts), and z is formed in
    // place in its column of W.  The later members of a cluster follow one at a
    // time, with the whole block: thread 0 forms the twisted vector (at an
    // eigenvalue moved at least a few ulps above the previous member's) and the
    // two inverse-iteration solves with the L D+ L^T factors, in LDS; all threads
    // share the scaling and, after each solve, a classical Gram-Schmidt pass
    // repeated twice against the earlier members of the cluster (columns of W).
    const double ortol = ortol_rel * tnorm;
    {
        double* wsd = reinterpret_cast<double*>(stage);
        const int wstride = 2 * s + 1;
        const int cap = max(1, (heig_region_a(smax) * 2) / wstride);
        // the twisted-factorisation vector of eigenvalue lk into z (factors in Dp, Uf)
        auto twisted = [&](double lk, double* z, double* Dp, double* Uf) {
            double dp = sdd[0] - lk;
            for (int i = 0; i + 1 < s; ++i) {
                if (fabs(dp) < pivmin) dp = -pivmin;
                Dp[i] = dp;
                const double e = see[i];
                dp = sdd[i + 1] - lk - e * e * rcp_nr(dp);
            }
            if (fabs(dp) < pivmin) dp = -pivmin;
            Dp[s - 1] = dp;
            double dm = sdd[s - 1] - lk;
            int twist = s - 1;
            double gbest = fabs(Dp[s - 1]);
            for (int i = s - 2; i >= 0; --i) {
                if (fabs(dm) < pivmin) dm = -pivmin;
                const double e = see[i];
                const double u = e * rcp_nr(dm);
                Uf[i] = u;
                dm = sdd[i] - lk - u * e;
                const double g = fabs(Dp[i] + dm - (sdd[i] - lk));
                if (g < gbest) {
                    gbest = g;
                    twist = i;
                }
            }
            double zc = 1.0;
            z[twist] = 1.0;
            for (int i = twist - 1; i >= 0; --i) {
                zc = -see[i] * rcp_nr(Dp[i]) * zc;
                z[i] = zc;
            }
            zc = 1.0;
            for (int i = twist; i + 1 < s; ++i) {
                zc = -Uf[i] * zc;
                z[i + 1] = zc;
            }
        };
        int nlead = 0;
        for (int k = 0; k < nabove; ++k) nlead += (k == 0 || slam[k] - slam[k - 1] > ortol);
        const bool leader = tid < nabove && (tid == 0 || slam[tid] - slam[tid - 1] > ortol);
        int rank = 0;
        if (leader)
            for (int k = 1; k <= tid; ++k) rank += (slam[k] - slam[k - 1] > ortol);
        if (nlead <= cap) {   // uniform
            if (leader) {
                double* Dp = wsd + (int64_t)rank * wstride;
                twisted(slam[tid], W + (int64_t)tid * s, Dp, Dp + s);
            }
            __syncthreads();
        } else {
            // more vectors than slots of 2 s + 1: D+ and U share one array of s (+ 1, odd stride),
            // which holds twice as many at once.  Only D+ below the twist and U from it onwards
            // are read when z is formed, so U is recomputed, from the bottom up to the twist, over
            // the D+ entries that are no longer needed.
            const int cstride = s + 1;
            const int cap1 = max(1, (heig_region_a(smax) * 2) / cstride);
            for (int r0 = 0; r0 < nlead; r0 += cap1) {
                if (leader && rank >= r0 && rank < r0 + cap1) {
                    const double lk = slam[tid];
                    double* F = wsd + (int64_t)(rank - r0) * cstride;
                    double* z = W + (int64_t)tid * s;
                    double dp = sdd[0] - lk;
                    for (int i = 0; i + 1 < s; ++i) {
                        if (fabs(dp) < pivmin) dp = -pivmin;
                        F[i] = dp;
                        const double e = see[i];
                        dp = sdd[i + 1] - lk - e * e * rcp_nr(dp);
                    }
                    if (fabs(dp) < pivmin) dp = -pivmin;
                    F[s - 1] = dp;
                    double dm = sdd[s - 1] - lk;
                    int twist = s - 1;
                    double gbest = fabs(F[s - 1]);
                    for (int i = s - 2; i >= 0; --i) {
                        if (fabs(dm) < pivmin) dm = -pivmin;
                        const double e = see[i];
                        const double u = e * rcp_nr(dm);
                        dm = sdd[i] - lk - u * e;
                        const double g = fabs(F[i] + dm - (sdd[i] - lk));
                        if (g < gbest) {
                            gbest = g;
                            twist = i;
                        }
                    }
                    dm = sdd[s - 1] - lk;
                    for (int i = s - 2; i >= twist; --i) {
                        if (fabs(dm) < pivmin) dm = -pivmin;
                        const double e = see[i];
                        const double u = e * rcp_nr(dm);
                        F[i] = u;
                        dm = sdd[i] - lk - u * e;
                    }
                    double zc = 1.0;
                    z[twist] = 1.0;
                    for (int i = twist - 1; i >= 0; --i) {
                        zc = -see[i] * rcp_nr(F[i]) * zc;
                        z[i] = zc;
                    }
                    zc = 1.0;
                    for (int i = twist; i + 1 < s; ++i) {
                        zc = -F[i] * zc;
                        z[i + 1] = zc;
                    }
                }
                __syncthreads();
            }
        }
        if (nlead < nabove) {   // uniform: some eigenvalues are clustered
            double* Dp = wsd;
            double* Uf = Dp + s;
            double* zb = Uf + s + 1;   // the member being formed
            double* dts = zb + s;      // its projections on the earlier members
            // z <- z / max|z| (a zero or non-finite z is replaced by a start vector), then
            // z <- z / ||z||, over the block; every thread calls these
            auto scale_max = [&](double* z, int seed) {
                double m = block_max(tid < s ? fabs(z[tid]) : 0.0, red);
                if (!(m > 0) || !(m < DBL_MAX)) {
                    if (tid < s) z[tid] = start_entry(tid, seed);
                    m = block_max(tid < s ? fabs(z[tid]) : 0.0, red);
                }
                if (tid < s) z[tid] *= 1.0 / m;
                __syncthreads();
            };
            auto scale_unit = [&](double* z) {
                const double n2 = block_sum(tid < s ? z[tid] * z[tid] : 0.0, red);
                if (tid < s) z[tid] *= n2 > 0 ? 1.0 / sqrt(n2) : 0.0;
                __syncthreads();
            };
            int lead = 0;
            double prev = 0;
            for (int k = 1; k < nabove; ++k) {   // uniform
                if (slam[k] - slam[k - 1] > ortol) {
                    lead = k;
                    continue;
                }
                if (k - 1 == lead) {
                    // the cluster's first member, formed above, is made a unit vector first
                    double* zl = W + (int64_t)lead * s;
                    scale_max(zl, lead + 1);
                    scale_unit(zl);
                    prev = slam[lead];
                }
                double lk = slam[k];
                const double pertol = 10.0 * DBL_EPSILON * fmax(fabs(lk), tnorm * 1e-3);
                if (lk - prev < pertol) lk = prev + pertol;
                prev = lk;
                if (tid == 0) twisted(lk, zb, Dp, Uf);
                __syncthreads();
                for (int it = 0; it <= 2; ++it) {
                    if (it > 0) {
                        if (tid == 0) {
                            // z <- (L D+ L^T)^{-1} z
                            double zp = zb[0];
                            for (int i = 0; i + 1 < s; ++i) {
                                const double zn = zb[i + 1] - see[i] * rcp_nr(Dp[i]) * zp;
                                zb[i + 1] = zn;
                                zp = zn;
                            }
                            for (int i = 0; i < s; ++i) zb[i] /= Dp[i];
                            zp = zb[s - 1];
                            for (int i = s - 2; i >= 0; --i) {
                                const double zn = zb[i] - see[i] * rcp_nr(Dp[i]) * zp;
                                zb[i] = zn;
                                zp = zn;
                            }
                        }
                        __syncthreads();
                    }
                    scale_max(zb, k + it + 1);
                    for (int pass = 0; pass < 2; ++pass) {
                        // projections on columns lead .. k-1: one wave per column, lanes over rows
                        for (int j = lead + wave; j < k; j += nw) {
                            const double* wj = W + (int64_t)j * s;
                            double d = 0;
                            for (int i = lane; i < s; i += 64) d += wj[i] * zb[i];
                            d = wave_sum_all(d);
                            if (lane == 0) dts[j - lead] = d;
                        }
                        __syncthreads();
                        if (tid < s) {
                            double z = zb[tid];
                            for (int j = lead; j < k; ++j) z -= dts[j - lead] * W[(int64_t)j * s + tid];
                            zb[tid] = z;
                        }
                        __syncthreads();
                    }
                    scale_unit(zb);
                }
                if (tid < s) W[(int64_t)k * s + tid] = zb[tid];
                __syncthreads();
            }
        }
    }
    // unit scale of every column of W, one wave per column with lanes over rows: 1 / (amax ||z / amax||);
    // a zero or non-finite column is replaced by a start vector first.  Each eigenpair is checked:
    // ||T z - lk z|| <= resid_lim ||T|| ||z|| (T the real tridiagonal), else, or for a replaced column,
    // bit 1 of flags reports an eigenpair that did not converge.
    double* zsc = secr;   // the complex off-diagonal is no longer needed
    for (int k = wave; k < nabove; k += nw) {
        double zv[SL];
        double amax = 0, rr = 0;
        const double lk = slam[k];
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
            const int row = sl * 64 + lane;
            zv[sl] = row < s ? W[(int64_t)k * s + row] : 0.0;
            amax = fmax(amax, fabs(zv[sl]));
            if (row < s) {
                double t = (sdd[row] - lk) * zv[sl];
                if (row > 0) t = fma(see[row - 1], W[(int64_t)k * s + row - 1], t);
                if (row + 1 < s) t = fma(see[row], W[(int64_t)k * s + row + 1], t);
                rr = fma(t, t, rr);
            }
        }
        amax = wave_max_all(amax);
        bool fail = false;
        if (!(amax > 0) || !(amax < DBL_MAX)) fail = true;
        else {
            double zz = 0;
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const double t = zv[sl] / amax;
                zz = fma(t, t, zz);
            }
            zz = wave_sum_all(zz);
            rr = wave_sum_all(rr);
            // ||r|| > lim ||T|| ||z||, with ||z|| = amax sqrt(zz); NaN residuals fail too
            if (!(sqrt(rr) <= resid_lim * tnorm * amax * sqrt(zz))) fail = true;
        }
        if (fail && lane == 0 && flags && !bad) atomicOr(flags, 2u);
        if (!(amax > 0) || !(amax < DBL_MAX)) {
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) {
                const int row = sl * 64 + lane;
                zv[sl] = row < s ? start_entry(row, k + 1) : 0.0;
                if (row < s) W[(int64_t)k * s + row] = zv[sl];
            }
            amax = 0;
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) amax = fmax(amax, fabs(zv[sl]));
            amax = wave_max_all(amax);
        }
        const double ia = 1.0 / amax;
        double ss = 0;
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
            const double t = zv[sl] * ia;
            ss = fma(t, t, ss);
        }
        ss = wave_sum_all(ss);
        if (lane == 0) {
            // with the threshold factor sqrt(f_k), except for the derivative (unscaled vectors)
            double fk = 1.0;
            if (vj.C == nullptr) {
                const double sig = sqrt(fmax(slam[k], 0.0));
                fk = sqrt(sig > 0 ? fmax(1.0 - thr / sig, 0.0) : 0.0);
            }
            zsc[k] = ss > 0 ? fk * ia / sqrt(ss) : 0.0;
        }
    }
    __syncthreads();

    // ---- 5. back-transform: X = Q diag(phase) W sqrt(f) ----------------------
    // X is column-major in the LU region.  For the derivative the unscaled
    // eigenvectors V = Q diag(phase) W are kept and sqrt(f) enters the S step.
    const int r = nabove;
    double2* X = reinterpret_cast<double2*>(LU);
    const bool vjp = vj.C != nullptr;
    for (int e0 = tid; e0 < s * r; e0 += 4 * EIG_THREADS) {   // loads of a batch ahead of its stores
        double wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * EIG_THREADS;
            wv[u] = e < s * r ? W[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * EIG_THREADS;
            if (e < s * r) {
                const int k = e / s, row = e - k * s;
                const double w = wv[u] * zsc[k];
                X[e] = make_double2(sdre[row] * w, sdim[row] * w);
            }
        }
    }
    double2* Tg = reinterpret_cast<double2*>(LU + 2LL * s * s);
    wy_factors(A, shv, s, Tg, stage);
    backtransform_wy<SL>(X, r, s, A, shv, Tg, stage, stage + nw * 256);

    if (vjp) {
        // ---- 5b. reverse-mode derivative of the threshold map ----------------
        // Z_A = A h(G), G = A^H A, h(l) = max(1 - thr / sqrt(l), 0).  Given
        // C = A^H Zbar_A, the cotangent of A is Zbar_A S + A P2 with
        //   P2 = 2 V_all (Hd o sym(V_all^H C V_all)) V_all^H,
        //   Hd_ij = (h_i - h_j) / (l_i - l_j)  (Daleckii-Krein; h'(l_i) on ties).
        // Pairs of eigenvalues both at or below thr^2 contribute nothing.  For
        // a, a2 above: Hd = thr / (s_a s_a2 (s_a + s_a2)), s = sqrt(l), exact
        // also at ties.  A pair (a above, b below) gives h_a / (l_a - l_b), so
        // the sum over all b is h_a (l_a I - G)^+ restricted to the complement
        // of range(V): y_a solves (l_a I - T) y'' = c'' in the real tridiagonal
        // basis (LU with partial pivoting), c_a = (I - V V^H) Msym v_a.
        //   P2 = 2 [V K V^H + sum_a h_a (v_a y_a^H + y_a v_a^H)],
        //   K = Hd o sym(V^H Msym V),  Msym = (C + C^H) / 2.
        // Also d Z_A / d thr contracted with Zbar: -sum_a Re(v_a^H C v_a) / s_a.
        const double2* C = vj.C + (int64_t)blockIdx.x * vj.c_stride;
        double2* Mv = reinterpret_cast<double2*>(vj.scr + (int64_t)blockIdx.x * vj.scr_stride);
        double2* Yv = Mv + (int64_t)s * r;
        double2* Mp = Yv + (int64_t)s * r;     // r x r, [a * r + a2] = v_a^H m_a2
        double2* Kc = Mp + (int64_t)r * r;     // r x r
        double2* Ev = Kc + (int64_t)r * r;     // s x r
        double* lu = reinterpret_cast<double*>(Ev + (int64_t)s * r);   // 4 s r, [i * r + a]
        double* u0 = lu;
        double* du1 = lu + (int64_t)s * r;
        double* du2 = du1 + (int64_t)s * r;
        double* lmul = du2 + (int64_t)s * r;
        // (i) m_a = Msym v_a
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int a = e / s, i = e - a * s;
            double mr = 0, mi = 0;
            for (int j = 0; j < s; ++j) {
                const double2 v = X[(int64_t)a * s + j];
                const double2 c1 = C[(int64_t)i * s + j];
                const double2 c2 = C[(int64_t)j * s + i];
                mr += (c1.x + c2.x) * v.x - (c1.y - c2.y) * v.y;
                mi += (c1.x + c2.x) * v.y + (c1.y - c2.y) * v.x;
            }
            Mv[(int64_t)a * s + i] = make_double2(0.5 * mr, 0.5 * mi);
        }
        __syncthreads();
        // (ii) M' = V^H Msym V
        for (int e = tid; e < r * r; e += EIG_THREADS) {
            const int a = e / r, a2 = e - a * r;
            double pr = 0, pi = 0;
            for (int i = 0; i < s; ++i) {
                const double2 v = X[(int64_t)a * s + i], m = Mv[(int64_t)a2 * s + i];
                pr += v.x * m.x + v.y * m.y;
                pi += v.x * m.y - v.y * m.x;
            }
            Mp[e] = make_double2(pr, pi);
        }
        __syncthreads();
        // (iii) c_a = m_a - V M'[:, a], then conj(phase) Q^H c_a
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int a = e / s, i = e - a * s;
            double2 c = Mv[(int64_t)a * s + i];
            for (int a2 = 0; a2 < r; ++a2) {
                const double2 v = X[(int64_t)a2 * s + i], pm = Mp[a2 * r + a];
                c.x -= v.x * pm.x - v.y * pm.y;
                c.y -= v.x * pm.y + v.y * pm.x;
            }
            Yv[(int64_t)a * s + i] = c;
        }
        apply_reflectors<SL>(Yv, r, s, smax, A, shv, stage, true);
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int i = e % s;
            const double2 c = Yv[e];
            Yv[e] = make_double2(sdre[i] * c.x + sdim[i] * c.y, sdre[i] * c.y - sdim[i] * c.x);
        }
        __syncthreads();
        // (iv) (T - l_a I) y'' = -c'', one thread per eigenvalue
        const double tiny = DBL_EPSILON * tnorm + pivmin;
        for (int a = tid; a < r; a += EIG_THREADS) {
            const double lk = slam[a];
            double dcur = sdd[0] - lk;
            double ucur = s > 1 ? see[0] : 0.0;
            for (int i = 0; i + 1 < s; ++i) {
                const double c = see[i];
                const double a1 = sdd[i + 1] - lk;
                const double b1 = (i + 2 < s) ? see[i + 1] : 0.0;
                const int64_t o = (int64_t)i * r + a;
                if (fabs(dcur) >= fabs(c)) {
                    const double piv = dcur == 0.0 ? tiny : dcur;
                    const double f = c / piv;
                    u0[o] = piv;
                    du1[o] = ucur;
                    du2[o] = 0.0;
                    lmul[o] = f;                 // no row swap, |f| <= 1
                    dcur = a1 - f * ucur;
                    ucur = b1;
                } else {
                    const double f = dcur / c;
                    u0[o] = c;
                    du1[o] = a1;
                    du2[o] = b1;
                    lmul[o] = -(f + 4.0);        // a swap, encoded below -3
                    dcur = ucur - f * a1;
                    ucur = -f * b1;
                }
            }
            u0[(int64_t)(s - 1) * r + a] = dcur == 0.0 ? tiny : dcur;
            double2* y = Yv + (int64_t)a * s;
            for (int i = 0; i < s; ++i) y[i] = make_double2(-y[i].x, -y[i].y);
            for (int i = 0; i + 1 < s; ++i) {
                const double lm = lmul[(int64_t)i * r + a];
                double2 yi = y[i], yi1 = y[i + 1];
                if (lm <= -3.0) {
                    const double f = -lm - 4.0;
                    const double2 t = yi;
                    yi = yi1;
                    yi1 = make_double2(t.x - f * yi.x, t.y - f * yi.y);
                } else {
                    yi1 = make_double2(yi1.x - lm * yi.x, yi1.y - lm * yi.y);
                }
                y[i] = yi;
                y[i + 1] = yi1;
            }
            double2 x1 = make_double2(0.0, 0.0), x2 = x1;
            for (int i = s - 1; i >= 0; --i) {
                const int64_t o = (int64_t)i * r + a;
                double2 v = y[i];
                if (i + 1 < s) {
                    v.x -= du1[o] * x1.x;
                    v.y -= du1[o] * x1.y;
                }
                if (i + 2 < s) {
                    v.x -= du2[o] * x2.x;
                    v.y -= du2[o] * x2.y;
                }
                v.x /= u0[o];
                v.y /= u0[o];
                y[i] = v;
                x2 = x1;
                x1 = v;
            }
        }
        __syncthreads();
        // (v) back to the Gram basis: y = Q diag(phase) y''
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int i = e % s;
            const double2 c = Yv[e];
            Yv[e] = make_double2(sdre[i] * c.x - sdim[i] * c.y, sdre[i] * c.y + sdim[i] * c.x);
        }
        apply_reflectors<SL>(Yv, r, s, smax, A, shv, stage, false);
        // (vi) y_a -= V (V^H y_a): coefficients into Kc, then the update
        for (int e = tid; e < r * r; e += EIG_THREADS) {
            const int a2 = e / r, a = e - a2 * r;
            double pr = 0, pi = 0;
            for (int i = 0; i < s; ++i) {
                const double2 v = X[(int64_t)a2 * s + i], y = Yv[(int64_t)a * s + i];
                pr += v.x * y.x + v.y * y.y;
                pi += v.x * y.y - v.y * y.x;
            }
            Kc[e] = make_double2(pr, pi);   // [a2 * r + a] = v_a2^H y_a
        }
        __syncthreads();
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int a = e / s, i = e - a * s;
            double2 y = Yv[e];
            for (int a2 = 0; a2 < r; ++a2) {
                const double2 v = X[(int64_t)a2 * s + i], cf = Kc[a2 * r + a];
                y.x -= v.x * cf.x - v.y * cf.y;
                y.y -= v.x * cf.y + v.y * cf.x;
            }
            Yv[e] = y;
        }
        __syncthreads();
        // (vii) K = Hd o sym(M'), the threshold contraction
        for (int e = tid; e < r * r; e += EIG_THREADS) {
            const int a = e / r, a2 = e - a * r;
            const double sa = sqrt(slam[a]), sb = sqrt(slam[a2]);
            const double hd = thr / (sa * sb * (sa + sb));
            const double2 m1 = Mp[a * r + a2], m2 = Mp[a2 * r + a];
            Kc[e] = make_double2(0.5 * hd * (m1.x + m2.x), 0.5 * hd * (m1.y - m2.y));
        }
        if (tid == 0 && vj.tbar) {
            double tb = 0;
            for (int a = 0; a < r; ++a) tb -= Mp[a * r + a].x / sqrt(slam[a]);
            vj.tbar[m0 + blockIdx.x] = tb;
        }
        __syncthreads();
        // (viii) E = V K
        for (int e = tid; e < s * r; e += EIG_THREADS) {
            const int a2 = e / s, i = e - a2 * s;
            double er = 0, ei = 0;
            for (int a = 0; a < r; ++a) {
                const double2 v = X[(int64_t)a * s + i], kk = Kc[a * r + a2];
                er += v.x * kk.x - v.y * kk.y;
                ei += v.x * kk.y + v.y * kk.x;
            }
            Ev[e] = make_double2(er, ei);
        }
        __syncthreads();
        // (ix) P2[i][j] = 2 sum_a (E_ia conj(V_ja) + h_a (V_ia conj(Y_ja) + Y_ia conj(V_ja)))
        OC* P2 = vj.P2 + (int64_t)blockIdx.x * vj.p2_stride;
        for (int e = tid; e < s * s; e += EIG_THREADS) {
            const int i = e / s, j = e - i * s;
            double pr = 0, pi = 0;
            for (int a = 0; a < r; ++a) {
                const double ha = 1.0 - thr / sqrt(slam[a]);
                const double2 ei_ = Ev[(int64_t)a * s + i], vj_ = X[(int64_t)a * s + j];
                const double2 vi_ = X[(int64_t)a * s + i], yj_ = Yv[(int64_t)a * s + j];
                const double2 yi_ = Yv[(int64_t)a * s + i];
                // E_ia conj(V_ja)
                pr += ei_.x * vj_.x + ei_.y * vj_.y;
                pi += ei_.y * vj_.x - ei_.x * vj_.y;
                // h_a (V_ia conj(Y_ja) + Y_ia conj(V_ja))
                pr += ha * (vi_.x * yj_.x + vi_.y * yj_.y + yi_.x * vj_.x + yi_.y * vj_.y);
                pi += ha * (vi_.y * yj_.x - vi_.x * yj_.y + yi_.y * vj_.x - yi_.x * vj_.y);
            }
            OC o;
            o.x = 2.0 * pr;
            o.y = 2.0 * pi;
            P2[e] = o;
        }
        __syncthreads();
    }
    // ---- 6. S = X X^H (row-major, ld = s) on the matrix cores ------------------
    // 16 x 16 tiles of the lower block triangle, one wave per tile; each
    // off-diagonal tile is also written conjugate-transposed.  With the
    // derivative X holds the unscaled eigenvectors and sqrt(f) scales both
    // operands.
    {
        double* sgf = se2;   // sqrt(f_k) or 1 (se2 is not needed after the bisection)
        for (int k = tid; k < r; k += EIG_THREADS) {
            double g = 1.0;
            if (vjp) {
                const double sig = sqrt(fmax(slam[k], 0.0));
                g = sqrt(sig > 0 ? fmax(1.0 - thr / sig, 0.0) : 0.0);
            }
            sgf[k] = g;
        }
        __syncthreads();
        const int lr = lane & 15, lk = lane >> 4;
        const int nrt = (s + 15) / 16, ntile = nrt * (nrt + 1) / 2;
        for (int t = wave; t < ntile; t += nw) {
            int tb = 0, rem = t;
            while (rem >= nrt - tb) {
                rem -= nrt - tb;
                ++tb;
            }
            const int ta = tb + rem;
            const int ra = ta * 16 + lr, rb = tb * 16 + lr;
            doublex4 sr = {0.0, 0.0, 0.0, 0.0}, si = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < r; k0 += 4) {
                const int k = k0 + lk;
                double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
                if (k < r) {
                    const double g = sgf[k];
                    if (ra < s) a = cscale(X[(int64_t)k * s + ra], g);
                    if (rb < s) b = cscale(X[(int64_t)k * s + rb], g);
                }
                // S[ra][rb] += a conj(b)
                sr = mfma16(a.x, b.x, sr);
                sr = mfma16(a.y, b.y, sr);
                si = mfma16(a.y, b.x, si);
                si = mfma16(-a.x, b.y, si);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ia = ta * 16 + lk + 4 * q, jb = tb * 16 + lr;
                if (ia < s && jb < s) {
                    OC o;
                    o.x = sr[q];
                    o.y = si[q];
                    S[(int64_t)ia * s + jb] = o;
                    if (ta != tb) {
                        o.y = -si[q];
                        S[(int64_t)jb * s + ia] = o;
                    }
                }
            }
        }
    }
    if (tid == 0) {
        int pos = 0;
        for (int k = 0; k < r; ++k) pos += sqrt(fmax(slam[k], 0.0)) > thr;
        if (ranks) ranks[m0 + blockIdx.x] = pos;
        if (bad && flags) atomicOr(flags, 1u);
    }
}

// dynamic LDS bytes of k_heig_svt for matrices of order <= smax
static size_t heig_lds_bytes(int smax) {
    const int nw = EIG_THREADS / 64;
    return (size_t)heig_region_a(smax) * sizeof(double2) + (size_t)9 * smax * sizeof(double) +
           (2 * nw + 8) * sizeof(double);
}

bool tridiag_rr_supported(int smax, bool fp32) { return smax >= 2 && smax <= (fp32 ? RR32_MAXS_WIDE : RR_MAXS); }

hipError_t launch_tridiag_rr(hipStream_t st, const LRDesc* descs, int m0, int count, double2* Gs, int64_t g_stride,
                             double* scr, int64_t scr_stride, int smax, bool fp32) {
    if (!tridiag_rr_supported(smax, fp32)) return hipErrorInvalidValue;
    const int nb = (smax + 15) / 16;
    // blocks per wave: ceil(nb (nb + 1) / 2 / waves)
    const void* fn;
    int nthr = RR_THREADS;
    if (fp32 && smax <= RR_MAXS) {
        nthr = 512;
        fn = nb <= 6 ? (const void*)k_tridiag_rr32<3, 512, RR_MAXS>
           : nb <= 8 ? (const void*)k_tridiag_rr32<5, 512, RR_MAXS>
           : nb <= 10 ? (const void*)k_tridiag_rr32<7, 512, RR_MAXS>
           : nb <= 12 ? (const void*)k_tridiag_rr32<10, 512, RR_MAXS>
                      : (const void*)k_tridiag_rr32<12, 512, RR_MAXS>;
    } else if (fp32) {
        nthr = 1024;
        fn = nb <= 14 ? (const void*)k_tridiag_rr32<7, 1024, RR32_MAXS_WIDE>
           : nb <= 15 ? (const void*)k_tridiag_rr32<8, 1024, RR32_MAXS_WIDE>
                      : (const void*)k_tridiag_rr32<9, 1024, RR32_MAXS_WIDE>;
    } else
        fn = nb <= 6 ? (const void*)k_tridiag_rr<2>
           : nb <= 8 ? (const void*)k_tridiag_rr<3>
           : nb <= 10 ? (const void*)k_tridiag_rr<5>
           : nb <= 12 ? (const void*)k_tridiag_rr<7>
                      : (const void*)k_tridiag_rr<8>;
    void* args[] = {(void*)&descs, (void*)&m0, (void*)&Gs, (void*)&g_stride, (void*)&scr, (void*)&scr_stride};
    hipError_t e = hipLaunchKernel(fn, dim3(count), dim3(nthr), args, 0, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename OC>
hipError_t launch_heig_svt(hipStream_t st, const LRDesc* descs, int m0, int count, double2* Gs, int64_t g_stride,
                           OC* Ss, int64_t s_stride, double* scr, int64_t scr_stride, int32_t* ranks,
                           double ortol_rel, uint32_t* flags, int smax, const VjpArgs<OC>& vj, int tri_in,
                           double resid_lim) {
    const size_t lds = heig_lds_bytes(smax);
    const int sl = (smax + 63) / 64;
    const void* fn = sl <= 1 ? (const void*)k_heig_svt<OC, 1>
                   : sl == 2 ? (const void*)k_heig_svt<OC, 2>
                   : sl == 3 ? (const void*)k_heig_svt<OC, 3>
                   : sl == 4 ? (const void*)k_heig_svt<OC, 4>
                             : (const void*)k_heig_svt<OC, 5>;
    if (sl > 5) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&descs, (void*)&m0, (void*)&Gs, (void*)&g_stride, (void*)&Ss, (void*)&s_stride, (void*)&scr,
                    (void*)&scr_stride, (void*)&ranks, (void*)&ortol_rel, (void*)&flags, (void*)&smax,
                    (void*)&vj, (void*)&tri_in, (void*)&resid_lim};
    e = hipLaunchKernel(fn, dim3(count), dim3(EIG_THREADS), args, lds, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template hipError_t launch_heig_svt<float2>(hipStream_t, const LRDesc*, int, int, double2*, int64_t, float2*, int64_t,
                                            double*, int64_t, int32_t*, double, uint32_t*, int,
                                            const VjpArgs<float2>&, int, double);
template hipError_t launch_heig_svt<double2>(hipStream_t, const LRDesc*, int, int, double2*, int64_t, double2*,
                                             int64_t, double*, int64_t, int32_t*, double, uint32_t*, int,
                                             const VjpArgs<double2>&, int, double);

}  // namespace shlr
