// Lift + Gram and reprojection + multiplier + adjoint-lift kernels (gfx950).
//
// One lifted matrix per line (Eq. 2 / Eq. 4 of the paper):
//   T[a][c] = w[a+b] * u_{v,j}[a+b] + D[a][c] / beta,  c = (v*J + j)*k + b,
//   u_{0,j} = h_j (the line of coil j) and u_{1,j} = h_j^dagger (virtual coils).
// T is never stored in HBM: chunks of it are rebuilt in LDS from the line
// (kept in LDS) and the multiplier D (streamed from HBM).
//
// The SVT of Eq. 16 is computed on the smaller side s of T through its Gram
// matrix G = A^H A, with A = T (q <= p) or A = T^H (p < q), A of size l x s:
//   k_lift_gram : G = A^H A on the matrix cores (FP32 or FP64 MFMA 16x16x4),
//   (k_heig_svt in eig.hip: S = V f(Lambda) V^H in FP64),
//   k_reproj    : Y = A S; Z = Y (side 0) or Y^H (side 1); then
//                 D' = D + tau (lift - Z)   (Eq. 13)
//                 b  = lift^*(Z - D'/beta)  (Eq. 15 right-hand-side term)
// The adjoint lift sums anti-diagonals in a fixed order (no atomics), so the
// results are bitwise reproducible.
#include "common.h"

namespace shlr {

constexpr int LR_THREADS = 512;     // 8 waves
constexpr int LR_WAVES = LR_THREADS / 64;

// Build the lifted line table u[v][j][i] = w[i] * (v == 0 ? h_j[i] : conj(h_j[flip(i)]))
// from lines at hb + off + j * cs + i * es.
template <typename R>
__device__ inline void load_line_table_at(cplx_t<R>* U, const cplx_t<R>* hb, int64_t off, int cs, int es,
                                          const cplx_t<R>* wtab, const LRDesc& d, int tid, int nth) {
    using C = cplx_t<R>;
    const int n = d.n, J = d.J, V = d.V;
    const int c = n / 2;
    for (int e = tid; e < V * J * n; e += nth) {
        int i = e % n;
        int blk = e / n;
        int v = blk / J, j = blk % J;
        C h;
        if (v == 0) {
            h = hb[off + (int64_t)j * cs + (int64_t)i * es];
        } else {
            int fi = (2 * c - i) % n;
            if (fi < 0) fi += n;
            h = cconj(hb[off + (int64_t)j * cs + (int64_t)fi * es]);
        }
        if (d.use_w) h = cmul(wtab[d.w_off + i], h);
        U[e] = h;
    }
}

template <typename R>
__device__ inline void load_line_table(cplx_t<R>* U, const cplx_t<R>* hb, const cplx_t<R>* wtab,
                                       const LRDesc& d, int tid, int nth) {
    load_line_table_at<R>(U, hb, d.h_off, d.h_cs, d.h_es, wtab, d, tid, nth);
}

// Value of T (without the D term) at (a, col).
template <typename C>
__device__ inline C lift_val(const C* U, int n, int k, int a, int col) {
    int blk = div_small(col, k);
    int b = col - blk * k;
    return U[blk * n + a + b];
}

// ---------------------------------------------------------------------------
// Stage a chunk of A rows [r0, r0 + KC) into LDS as split real/imag planes,
// zero padded to s_pad columns and KC rows.
// ---------------------------------------------------------------------------
// General form: rows of (cu * lift(U) + cd * Dm) (side 0) or of its conjugate
// transpose (side 1).
template <typename R>
__device__ inline void stage_chunk(R* Ar, R* Ai, int ldA, const cplx_t<R>* U, R cu, const cplx_t<R>* Dm, R cd,
                                   const LRDesc& d, int r0, int KC, int s_pad, int tid, int nth) {
    using C = cplx_t<R>;
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int total = KC * s_pad;
    if (side == 0) {
        for (int e = tid; e < total; e += nth) {
            int r = div_small(e, s_pad), cidx = e - r * s_pad;
            int a = r0 + r;
            R re = 0, im = 0;
            if (a < l && cidx < s) {
                C dv = Dm[(int64_t)a * q + cidx];
                C lv = lift_val(U, d.n, d.k, a, cidx);
                re = cu * lv.x + cd * dv.x;
                im = cu * lv.y + cd * dv.y;
            }
            Ar[r * ldA + cidx] = re;
            Ai[r * ldA + cidx] = im;
        }
    } else {
        for (int e = tid; e < total; e += nth) {
            int cidx = div_small(e, KC), r = e - cidx * KC;
            int col = r0 + r;
            R re = 0, im = 0;
            if (col < l && cidx < s) {
                C dv = Dm[(int64_t)cidx * q + col];
                C lv = lift_val(U, d.n, d.k, cidx, col);
                re = cu * lv.x + cd * dv.x;
                im = -(cu * lv.y + cd * dv.y);
            }
            Ar[r * ldA + cidx] = re;
            Ai[r * ldA + cidx] = im;
        }
    }
}

// UB entries per thread at a time: their multiplier reads are all issued before the first is
// used, so that a chunk waits for HBM once per UB entries rather than once per entry (UB = 1
// where the registers are needed elsewhere)
template <typename R, int UB = 1>
__device__ inline void stage_A_chunk(R* Ar, R* Ai, int ldA, const cplx_t<R>* U, const cplx_t<R>* Dm,
                                     const LRDesc& d, R inv_beta, int r0, int KC, int s_pad, int tid, int nth) {
    using C = cplx_t<R>;
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int total = KC * s_pad;
    for (int e0 = tid; e0 < total; e0 += UB * nth) {
        C dv[UB];
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int e = e0 + j * nth;
            dv[j] = C{0, 0};
            if (e < total) {
                if (side == 0) {
                    const int r = div_small(e, s_pad), cidx = e - r * s_pad, a = r0 + r;
                    if (a < l && cidx < s) dv[j] = Dm[(int64_t)a * q + cidx];
                } else {
                    // A[r][c] = conj(T[c][r]): rows of A are columns of T; read D with r fastest
                    const int cidx = div_small(e, KC), r = e - cidx * KC, col = r0 + r;
                    if (col < l && cidx < s) dv[j] = Dm[(int64_t)cidx * q + col];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int e = e0 + j * nth;
            if (e < total) {
                R re = 0, im = 0;
                int r, cidx;
                if (side == 0) {
                    r = div_small(e, s_pad);
                    cidx = e - r * s_pad;
                    if (r0 + r < l && cidx < s) {
                        const C lv = lift_val(U, d.n, d.k, r0 + r, cidx);
                        re = lv.x + dv[j].x * inv_beta;
                        im = lv.y + dv[j].y * inv_beta;
                    }
                } else {
                    cidx = div_small(e, KC);
                    r = e - cidx * KC;
                    if (r0 + r < l && cidx < s) {
                        const C lv = lift_val(U, d.n, d.k, cidx, r0 + r);
                        re = lv.x + dv[j].x * inv_beta;
                        im = -(lv.y + dv[j].y * inv_beta);
                    }
                }
                Ar[r * ldA + cidx] = re;
                Ai[r * ldA + cidx] = im;
            }
        }
    }
}

// Multiplier entries per thread that the Gram kernel keeps in flight for the next chunk, and
// whether a launch does (FP32, tiles up to 16 per wave: the registers allow it there).
constexpr int GRAM_NPF = 4;
__host__ __device__ inline bool gram_prefetches(int rsize, int maxt, int KC, int s_pad) {
    return rsize == 4 && maxt <= 16 && KC * s_pad <= GRAM_NPF * LR_THREADS;
}

// The same staging in two halves, so that the multiplier reads of the next chunk are in flight
// while the current one is multiplied: prefetch_D_chunk loads this thread's D entries of a chunk
// (at most NPF of them) into registers, stage_A_prefetched forms A from them.  Callers check
// KC * s_pad <= NPF * nth.
template <typename R, int NPF>
__device__ inline void prefetch_D_chunk(cplx_t<R> (&dv)[NPF], const cplx_t<R>* Dm, const LRDesc& d, int r0, int KC,
                                        int s_pad, int tid, int nth) {
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int total = KC * s_pad;
#pragma unroll
    for (int j = 0; j < NPF; ++j) {
        const int e = tid + j * nth;
        dv[j] = cplx_t<R>{0, 0};
        if (e < total) {
            if (side == 0) {
                const int r = div_small(e, s_pad), cidx = e - r * s_pad, a = r0 + r;
                if (a < l && cidx < s) dv[j] = Dm[(int64_t)a * q + cidx];
            } else {
                const int cidx = div_small(e, KC), r = e - cidx * KC, col = r0 + r;
                if (col < l && cidx < s) dv[j] = Dm[(int64_t)cidx * q + col];
            }
        }
    }
}

template <typename R, int NPF>
__device__ inline void stage_A_prefetched(R* Ar, R* Ai, int ldA, const cplx_t<R>* U, const cplx_t<R> (&dv)[NPF],
                                          const LRDesc& d, R inv_beta, int r0, int KC, int s_pad, int tid,
                                          int nth) {
    using C = cplx_t<R>;
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int total = KC * s_pad;
    // the element indices are recomputed here rather than kept from the prefetch (registers)
    int t0 = tid;
    asm volatile("" : "+v"(t0));
#pragma unroll
    for (int j = 0; j < NPF; ++j) {
        const int e = t0 + j * nth;
        if (e < total) {
            R re = 0, im = 0;
            int r, cidx;
            if (side == 0) {
                r = div_small(e, s_pad);
                cidx = e - r * s_pad;
                if (r0 + r < l && cidx < s) {
                    const C lv = lift_val(U, d.n, d.k, r0 + r, cidx);
                    re = lv.x + dv[j].x * inv_beta;
                    im = lv.y + dv[j].y * inv_beta;
                }
            } else {
                cidx = div_small(e, KC);
                r = e - cidx * KC;
                if (r0 + r < l && cidx < s) {
                    const C lv = lift_val(U, d.n, d.k, cidx, r0 + r);
                    re = lv.x + dv[j].x * inv_beta;
                    im = -(lv.y + dv[j].y * inv_beta);
                }
            }
            Ar[r * ldA + cidx] = re;
            Ai[r * ldA + cidx] = im;
        }
    }
}

// Tile g of the upper-triangular tiles of an nt x nt tile grid listed row by row in the order
// 0, nt-1, 1, nt-2, ...: pair m = g / (nt + 1) holds row m (nt - m tiles) then row nt - 1 - m.
// Returns (block row, block column).
__device__ inline int2 gram_tile_at(int nt, int g) {
    const int m = g / (nt + 1), rem = g - m * (nt + 1);
    const bool lo = rem < nt - m;
    const int I = lo ? m : nt - 1 - m;
    return int2{I, lo ? m + rem : I + (rem - (nt - m))};
}

// ---------------------------------------------------------------------------
// k_lift_gram
//   grid.x: matrices of the chunk; grid.y: groups of 8 "units".
//   The upper-triangular 16x16 tiles of G are grouped into units: the pair of
//   tile rows (I, nt-1-I), or the middle row alone, which balances the waves.
//   Each wave owns one unit (<= nt + 1 tiles) for the whole l loop.
// ---------------------------------------------------------------------------
template <typename R, int MAXT>
__global__ __launch_bounds__(LR_THREADS) void k_lift_gram(const cplx_t<R>* __restrict__ hb,
                                                          const cplx_t<R>* __restrict__ db,
                                                          const cplx_t<R>* __restrict__ wtab,
                                                          const LRDesc* __restrict__ descs, int m0,
                                                          double2* __restrict__ Gs, int64_t g_stride,
                                                          R inv_beta, int KC) {
    using C = cplx_t<R>;
    using A4 = acc4_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const LRDesc d = descs[m0 + blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s = lr_s(d), l = lr_l(d);
    const int nt = (s + 15) / 16;
    const int s_pad = nt * 16;
    const int ldA = s_pad + 4;
    C* U = reinterpret_cast<C*>(smem_raw);
    const int utab = d.V * d.J * d.n;
    R* Ar = reinterpret_cast<R*>(U + utab);
    R* Ai = Ar + KC * ldA;

    // Tiles of this wave: the nt (nt + 1) / 2 upper-triangular tiles listed row by row in the
    // order 0, nt-1, 1, nt-2, ... and cut into LR_WAVES * gridDim.y contiguous segments of equal
    // size (every SIMD gets the same share).  A launch over matrices of several orders sizes
    // grid.y for the largest: blocks past this matrix's tiles return at once (block-uniform,
    // before any barrier).
    const int n_tiles = nt * (nt + 1) / 2;
    const int nseg = LR_WAVES * (int)gridDim.y;
    const int per = (n_tiles + nseg - 1) / nseg;
    if ((int)blockIdx.y * LR_WAVES * per >= n_tiles) return;
    const int t_begin = min(((int)blockIdx.y * LR_WAVES + wave) * per, n_tiles);
    const int count = min(per, n_tiles - t_begin);
    const bool active = count > 0;
    // The segment covers at most three pieces of tile rows: piece p is row Ip, tiles Jp, Jp + 1,
    // ... for the wave's tiles E(p-1) .. Ep - 1 (E(-1) = 0; unused pieces repeat the last row).
    // Tile g of the list: pair m = g / (nt + 1) holds row m (nt - m tiles) then row nt - 1 - m.
    const int2 p0 = gram_tile_at(nt, min(t_begin, n_tiles - 1));
    const int I0 = p0.x, J0 = p0.y;
    const int E0 = min(count, nt - J0);                 // rest of row I0
    const int2 p1 = gram_tile_at(nt, min(t_begin + E0, n_tiles - 1));
    const int I1 = p1.x, J1 = p1.y;
    const int E1 = E0 + min(count - E0, nt - J1);
    const int2 p2 = gram_tile_at(nt, min(t_begin + E1, n_tiles - 1));
    const int I2 = p2.x, J2 = p2.y;
    // block row and column of tile t of the wave (wave-uniform)
#define tile_I(t) ((t) < E0 ? I0 : ((t) < E1 ? I1 : I2))
#define tile_J(t) ((t) < E0 ? J0 + (t) : ((t) < E1 ? J1 + ((t) - E0) : J2 + ((t) - E1)))

    // Entries of conj(a) b with three real products (Gauss) in FP32 where the registers allow the
    // third accumulator: P1 = ar br, P2 = ai bi, P3 = (ar - ai)(br + bi), Re = P1 + P2,
    // Im = P3 - P1 + P2.  Otherwise (and in FP64) four: acc1 = Re, acc2 = Im.
    constexpr bool G3 = sizeof(R) == 4 && MAXT <= 12;
    A4 acc1[MAXT], acc2[MAXT], acc3[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        acc1[t] = A4{0, 0, 0, 0};
        acc2[t] = A4{0, 0, 0, 0};
        if constexpr (G3) acc3[t] = A4{0, 0, 0, 0};
    }

    load_line_table<R>(U, hb, wtab, d, tid, LR_THREADS);
    const C* Dm = db + d.d_off;
    const int li = lane & 15, lk = lane >> 4;

    // the multiplier entries of the next chunk are loaded while the current one is multiplied
    constexpr int NPF = GRAM_NPF;
    const bool pf = gram_prefetches(sizeof(R), MAXT, KC, s_pad);   // uniform
    C dv[NPF];
    if (pf) prefetch_D_chunk<R, NPF>(dv, Dm, d, 0, KC, s_pad, tid, LR_THREADS);
    for (int r0 = 0; r0 < l; r0 += KC) {
        __syncthreads();
        if (pf) {
            stage_A_prefetched<R, NPF>(Ar, Ai, ldA, U, dv, d, inv_beta, r0, KC, s_pad, tid, LR_THREADS);
            __syncthreads();
            if (r0 + KC < l) prefetch_D_chunk<R, NPF>(dv, Dm, d, r0 + KC, KC, s_pad, tid, LR_THREADS);
        } else {
            stage_A_chunk<R>(Ar, Ai, ldA, U, Dm, d, inv_beta, r0, KC, s_pad, tid, LR_THREADS);
            __syncthreads();
        }
        if (active) {
            for (int kk = 0; kk < KC; kk += 4) {
                const int row = (kk + lk) * ldA + li;
                if constexpr (sizeof(R) == 4 && MAXT <= 16) {
                    // every operand of the step is read before the products (one wait per step);
                    // wider tiles or FP64 operands would not fit in registers beside them
                    const R pr0 = Ar[row + I0 * 16], pm0 = Ai[row + I0 * 16];
                    const R pr1 = Ar[row + I1 * 16], pm1 = Ai[row + I1 * 16];
                    const R pr2 = Ar[row + I2 * 16], pm2 = Ai[row + I2 * 16];
                    R br[MAXT], bi[MAXT];
#pragma unroll
                    for (int t = 0; t < MAXT; ++t) {
                        if (t < count) {
                            br[t] = Ar[row + tile_J(t) * 16];
                            bi[t] = Ai[row + tile_J(t) * 16];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < MAXT; ++t) {
                        if (t < count) {
                            const R ar = t < E0 ? pr0 : (t < E1 ? pr1 : pr2);
                            const R ai = t < E0 ? pm0 : (t < E1 ? pm1 : pm2);
                            if constexpr (G3) {
                                acc1[t] = mfma16(ar, br[t], acc1[t]);
                                acc2[t] = mfma16(ai, bi[t], acc2[t]);
                                acc3[t] = mfma16(ar - ai, br[t] + bi[t], acc3[t]);
                            } else {
                                acc1[t] = mfma16(ar, br[t], acc1[t]);
                                acc1[t] = mfma16(ai, bi[t], acc1[t]);
                                acc2[t] = mfma16(ar, bi[t], acc2[t]);
                                acc2[t] = mfma16(-ai, br[t], acc2[t]);
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < MAXT; ++t) {
                        if (t < count) {
                            const int Ib = tile_I(t), Jb = tile_J(t);
                            const R ar = Ar[row + Ib * 16], ai = Ai[row + Ib * 16];
                            const R br = Ar[row + Jb * 16], bi = Ai[row + Jb * 16];
                            if constexpr (G3) {
                                acc1[t] = mfma16(ar, br, acc1[t]);
                                acc2[t] = mfma16(ai, bi, acc2[t]);
                                acc3[t] = mfma16(ar - ai, br + bi, acc3[t]);
                            } else {
                                acc1[t] = mfma16(ar, br, acc1[t]);
                                acc1[t] = mfma16(ai, bi, acc1[t]);
                                acc2[t] = mfma16(ar, bi, acc2[t]);
                                acc2[t] = mfma16(-ai, br, acc2[t]);
                            }
                        }
                    }
                }
            }
        }
    }
    if (!active) return;
    // write G: packed lower triangle
    double2* G = Gs + (int64_t)blockIdx.x * g_stride;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        if (t < count) {
            const int Ib = tile_I(t), Jb = tile_J(t);
            const int col = Jb * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = Ib * 16 + acc_row<R>(lk, r);
                if (row < s && col < s) {
                    const R gr = G3 ? acc1[t][r] + acc2[t][r] : acc1[t][r];
                    const R gi = G3 ? acc3[t][r] - acc1[t][r] + acc2[t][r] : acc2[t][r];
                    // packed lower triangle; the diagonal tiles hold both halves
                    if (row >= col) G[pk(row, col, s)] = make_double2((double)gr, (double)gi);
                    else if (Ib != Jb) G[pk(col, row, s)] = make_double2((double)gr, -(double)gi);
                }
            }
        }
    }
}
#undef tile_I
#undef tile_J

// ---------------------------------------------------------------------------
// k_reproj
//   One workgroup per matrix.  Loop over chunks of KC rows of A:
//     Y_chunk = A_chunk (KC x s) * S (s x s)   on the matrix cores,
//   then per element the multiplier update and R = Z - D'/beta staged in LDS,
//   then fixed-order anti-diagonal sums into the LDS accumulator Bacc.
// ---------------------------------------------------------------------------
template <typename R, int MAXT>
__global__ __launch_bounds__(LR_THREADS) void k_reproj(const cplx_t<R>* __restrict__ hb,
                                                       cplx_t<R>* __restrict__ db,
                                                       cplx_t<R>* __restrict__ bb,
                                                       const cplx_t<R>* __restrict__ wtab,
                                                       const LRDesc* __restrict__ descs, int m0,
                                                       const cplx_t<R>* __restrict__ Ss, int64_t s_stride,
                                                       R inv_beta, R tau, int KC, int stage_s) {
    using C = cplx_t<R>;
    using A4 = acc4_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const LRDesc d = descs[m0 + blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int n = d.n, k = d.k, J = d.J, V = d.V;
    const int nt = (s + 15) / 16;
    const int s_pad = nt * 16;
    const int ldA = s_pad + 4;
    const int utab = V * J * n;
    C* U = reinterpret_cast<C*>(smem_raw);
    C* Bacc = U + utab;
    R* Ar = reinterpret_cast<R*>(Bacc + utab);
    R* Ai = Ar + KC * ldA;
    C* Rst = reinterpret_cast<C*>(Ar);  // R staging reuses the A planes: KC x s_pad complex fits in 2*KC*ldA reals
    C* Sst = reinterpret_cast<C*>(Ai + KC * ldA);   // two staged steps of S: 2 x 4 x s_pad

    load_line_table<R>(U, hb, wtab, d, tid, LR_THREADS);
    for (int e = tid; e < utab; e += LR_THREADS) Bacc[e] = cmk<C>(0, 0);

    C* Dm = db + d.d_off;
    const C* S = Ss + (int64_t)blockIdx.x * s_stride;
    const int li = lane & 15, lk = lane >> 4;
    const int rt = KC / 16;               // row tiles per chunk
    // tiles of this wave: one row tile It_w and the column tiles kw, kw + nwi, ... (the waves that
    // share a row tile split its column tiles), so the A operand of a step is read once per wave
    const int It_w = wave % rt, kw = wave / rt;
    const int nwi = (LR_WAVES - It_w + rt - 1) / rt;

    for (int r0 = 0; r0 < l; r0 += KC) {
        __syncthreads();
        stage_A_chunk<R, 8>(Ar, Ai, ldA, U, Dm, d, inv_beta, r0, KC, s_pad, tid, LR_THREADS);
        __syncthreads();
        // Complex products with three real ones (Gauss) in FP32 where the registers allow the third
        // accumulator: P1 = Ar Sr, P2 = Ai Si, P3 = (Ar + Ai)(Sr + Si), Re Y = P1 - P2,
        // Im Y = P3 - P1 - P2.  Otherwise (and in FP64) four: acc1 = Re Y, acc2 = Im Y.
        constexpr bool G3 = sizeof(R) == 4 && MAXT <= 8;
        A4 acc1[MAXT], acc2[MAXT], acc3[MAXT];
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            acc1[t] = A4{0, 0, 0, 0};
            acc2[t] = A4{0, 0, 0, 0};
            if constexpr (G3) acc3[t] = A4{0, 0, 0, 0};
        }
        // tiles of this wave: t-th tile = wave + t * LR_WAVES.  The four rows of S that step kk
        // needs are staged in LDS (two buffers); the rows of step kk + 4 are loaded from L2 into
        // registers while the products of step kk run, and written to the other buffer after them.
        const int srow = 4 * s_pad;   // entries per staged step (s_pad <= 320: at most 3 per thread)
        constexpr int SVN = 3;
        C sv[SVN];
        auto load_rows = [&](int kk) {
#pragma unroll
            for (int u = 0; u < SVN; ++u) {
                const int e = tid + u * LR_THREADS;
                const int eq = div_small(e, s_pad), row = kk + eq, col = e - eq * s_pad;
                sv[u] = (e < srow && row < s && col < s) ? S[(int64_t)row * s + col] : cmk<C>(0, 0);
            }
        };
        auto store_rows = [&](C* dst) {
#pragma unroll
            for (int u = 0; u < SVN; ++u) {
                const int e = tid + u * LR_THREADS;
                if (e < srow) dst[e] = sv[u];
            }
        };
        if (!stage_s) {
            // LDS too small for the staged rows: B operands straight from L2
            for (int kk = 0; kk < s_pad; kk += 4) {
                const int kidx = kk + lk;
                const int arow = (It_w * 16 + li) * ldA + kidx;
                const R ar = Ar[arow], ai = Ai[arow];
#pragma unroll
                for (int t = 0; t < MAXT; ++t) {
                    const int Jt = kw + nwi * t;
                    if (Jt < nt) {
                        const int col = Jt * 16 + li;
                        R sr = 0, si = 0;
                        if (kidx < s && col < s) {
                            const C svv = S[(int64_t)kidx * s + col];
                            sr = svv.x;
                            si = svv.y;
                        }
                        if constexpr (G3) {
                            acc1[t] = mfma16(ar, sr, acc1[t]);
                            acc2[t] = mfma16(ai, si, acc2[t]);
                            acc3[t] = mfma16(ar + ai, sr + si, acc3[t]);
                        } else {
                            acc1[t] = mfma16(ar, sr, acc1[t]);
                            acc1[t] = mfma16(-ai, si, acc1[t]);
                            acc2[t] = mfma16(ar, si, acc2[t]);
                            acc2[t] = mfma16(ai, sr, acc2[t]);
                        }
                    }
                }
            }
        } else {
        load_rows(0);
        store_rows(Sst);
        __syncthreads();
        for (int kk = 0; kk < s_pad; kk += 4) {
            const int kidx = kk + lk;
            const C* cur = Sst + ((kk >> 2) & 1) * srow;
            C* nxt = Sst + (((kk >> 2) & 1) ^ 1) * srow;
            if (kk + 4 < s_pad) load_rows(kk + 4);
            // every operand of the step is read before the products (one wait per step)
            const int arow = (It_w * 16 + li) * ldA + kidx;
            const R ar = Ar[arow], ai = Ai[arow], as = ar + ai;
            C sb[MAXT];
#pragma unroll
            for (int t = 0; t < MAXT; ++t) sb[t] = cur[lk * s_pad + min(kw + nwi * t, nt - 1) * 16 + li];
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                if (kw + nwi * t < nt) {   // uniform over the wave
                    if constexpr (G3) {
                        acc1[t] = mfma16(ar, sb[t].x, acc1[t]);
                        acc2[t] = mfma16(ai, sb[t].y, acc2[t]);
                        acc3[t] = mfma16(as, sb[t].x + sb[t].y, acc3[t]);
                    } else {
                        acc1[t] = mfma16(ar, sb[t].x, acc1[t]);
                        acc1[t] = mfma16(-ai, sb[t].y, acc1[t]);
                        acc2[t] = mfma16(ar, sb[t].y, acc2[t]);
                        acc2[t] = mfma16(ai, sb[t].x, acc2[t]);
                    }
                }
            }
            if (kk + 4 < s_pad) store_rows(nxt);
            __syncthreads();
        }
        }
        __syncthreads();  // A planes are dead from here on; reuse them for R
        // epilogue: multiplier update and R staging
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int Jt = kw + nwi * t;
            if (Jt < nt) {
                const int It = It_w;
                const int col = Jt * 16 + li;
                // FP32 with up to 8 tiles per wave: the tile's four multiplier reads are issued
                // before any of its writes (the registers allow it there); otherwise one at a time
                constexpr bool BATCH = sizeof(R) == 4 && MAXT <= 8;
                C dv[4];
                if constexpr (BATCH) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = r0 + It * 16 + acc_row<R>(lk, r);
                        dv[r] = cmk<C>(0, 0);
                        if (row < l && col < s)
                            dv[r] = side == 0 ? Dm[(int64_t)row * q + col] : Dm[(int64_t)col * q + row];
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rloc = It * 16 + acc_row<R>(lk, r);
                    const int row = r0 + rloc;
                    C rv = cmk<C>(0, 0);
                    if (row < l && col < s) {
                        int a, c;
                        C z;
                        const R yr = G3 ? acc1[t][r] - acc2[t][r] : acc1[t][r];
                        const R yi = G3 ? acc3[t][r] - acc1[t][r] - acc2[t][r] : acc2[t][r];
                        if (side == 0) { a = row; c = col; z = cmk<C>(yr, yi); }
                        else { a = col; c = row; z = cmk<C>(yr, -yi); }
                        const C lv = lift_val(U, n, k, a, c);
                        const int64_t di = (int64_t)a * q + c;
                        if constexpr (!BATCH) dv[r] = Dm[di];
                        C dn;
                        dn.x = dv[r].x + tau * (lv.x - z.x);
                        dn.y = dv[r].y + tau * (lv.y - z.y);
                        Dm[di] = dn;
                        rv.x = z.x - dn.x * inv_beta;
                        rv.y = z.y - dn.y * inv_beta;
                    }
                    Rst[rloc * s_pad + col] = rv;
                }
            }
        }
        __syncthreads();
        // anti-diagonal sums of this chunk, fixed order, one owner per entry
        const int rows_here = min(KC, l - r0);
        for (int e = tid; e < utab; e += LR_THREADS) {
            const int blk = div_small(e, n), i = e - blk * n;
            C acc = Bacc[e];
            if (side == 0) {
                // chunk rows are a in [r0, r0 + rows_here): b = i - a in [0, k)
                int a_lo = max(r0, i - k + 1), a_hi = min(r0 + rows_here - 1, min(i, p - 1));
                for (int a = a_lo; a <= a_hi; ++a) {
                    const C v = Rst[(a - r0) * s_pad + blk * k + (i - a)];
                    acc.x += v.x;
                    acc.y += v.y;
                }
            } else {
                // chunk rows are columns c of T: c = blk*k + b, a = i - b in [0, p)
                int c_lo = max(r0, blk * k + max(0, i - p + 1));
                int c_hi = min(r0 + rows_here - 1, blk * k + min(k - 1, i));
                for (int c = c_lo; c <= c_hi; ++c) {
                    const int b = c - blk * k;
                    const C v = Rst[(c - r0) * s_pad + (i - b)];
                    acc.x += v.x;
                    acc.y += v.y;
                }
            }
            Bacc[e] = acc;
        }
    }
    __syncthreads();
    // b_j[i] = conj(w[i]) Bacc[0][j][i] + (virtual coils) conj(conj(w[f]) Bacc[1][j][f]), f = flip(i)
    const int cc = n / 2;
    for (int e = tid; e < J * n; e += LR_THREADS) {
        const int i = e % n, j = e / n;
        C w = d.use_w ? wtab[d.w_off + i] : cmk<C>(1, 0);
        C out = cmulc(w, Bacc[j * n + i]);
        if (V == 2) {
            int fi = (2 * cc - i) % n;
            if (fi < 0) fi += n;
            C wf = d.use_w ? wtab[d.w_off + fi] : cmk<C>(1, 0);
            C g = cmulc(wf, Bacc[(J + j) * n + fi]);
            out.x += g.x;
            out.y -= g.y;
        }
        bb[d.b_off + (int64_t)j * d.b_cs + (int64_t)i * d.b_es] = out;
    }
}

// ---------------------------------------------------------------------------
// Reverse mode of one low-rank step (lift, SVT, multiplier update, adjoint
// lift).  Per matrix, with A the side-s form of T = lift(h) + D / beta and
//   Zbar = (1 + tau/beta) lift(gb) - tau Dbar
// (gb: cotangent of the adjoint-lift output line, Dbar: cotangent of the
// updated multiplier):
//   k_cross_gram : C = A^H Zbar_A (full s x s, FP64) for the eigen kernel;
//   k_reproj_vjp : Tbar_A = Zbar_A S + A P2, then
//                  Dbar' = Dbar - lift(gb) / beta,
//                  Dbar <- Dbar' + Tbar / beta        (cotangent of D),
//                  ghb  = lift^*(tau Dbar' + Tbar)     (cotangent of the line).
// ---------------------------------------------------------------------------
template <typename R, int MAXT>
__global__ __launch_bounds__(LR_THREADS) void k_cross_gram(const cplx_t<R>* __restrict__ hb,
                                                           const cplx_t<R>* __restrict__ db,
                                                           const cplx_t<R>* __restrict__ gb,
                                                           const cplx_t<R>* __restrict__ gdb,
                                                           const cplx_t<R>* __restrict__ wtab,
                                                           const LRDesc* __restrict__ descs, int m0,
                                                           double2* __restrict__ Cs, int64_t c_stride,
                                                           R inv_beta, R cz, R cdz, int KC) {
    using C = cplx_t<R>;
    using A4 = acc4_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const LRDesc d = descs[m0 + blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s = lr_s(d), l = lr_l(d);
    const int nt = (s + 15) / 16;
    const int s_pad = nt * 16;
    const int ldA = s_pad + 4;
    const int utab = d.V * d.J * d.n;
    C* Uh = reinterpret_cast<C*>(smem_raw);
    C* Ub = Uh + utab;
    R* Ar = reinterpret_cast<R*>(Ub + utab);
    R* Ai = Ar + KC * ldA;
    R* Zr = Ai + KC * ldA;
    R* Zi = Zr + KC * ldA;

    const int nseg = (nt + MAXT - 1) / MAXT;
    const int unit = blockIdx.y * LR_WAVES + wave;
    const bool active = unit < nt * nseg;
    const int I = active ? unit / nseg : 0;
    const int J0 = active ? (unit % nseg) * MAXT : 0;
    const int cnt = active ? min(MAXT, nt - J0) : 0;

    A4 accR[MAXT], accI[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        accR[t] = A4{0, 0, 0, 0};
        accI[t] = A4{0, 0, 0, 0};
    }
    load_line_table<R>(Uh, hb, wtab, d, tid, LR_THREADS);
    load_line_table_at<R>(Ub, gb, d.b_off, d.b_cs, d.b_es, wtab, d, tid, LR_THREADS);
    const C* Dm = db + d.d_off;
    const C* Gm = gdb + d.d_off;
    const int li = lane & 15, lk = lane >> 4;
    for (int r0 = 0; r0 < l; r0 += KC) {
        __syncthreads();
        stage_chunk<R>(Ar, Ai, ldA, Uh, (R)1, Dm, inv_beta, d, r0, KC, s_pad, tid, LR_THREADS);
        stage_chunk<R>(Zr, Zi, ldA, Ub, cz, Gm, cdz, d, r0, KC, s_pad, tid, LR_THREADS);
        __syncthreads();
        if (!active) continue;
        for (int kk = 0; kk < KC; kk += 4) {
            const int row = (kk + lk) * ldA + li;
            const R ar = Ar[row + I * 16], ai = Ai[row + I * 16];
#pragma unroll
            for (int t = 0; t < MAXT; ++t) {
                if (t < cnt) {
                    const int Jb = J0 + t;
                    const R zr = Zr[row + Jb * 16], zi = Zi[row + Jb * 16];
                    accR[t] = mfma16(ar, zr, accR[t]);
                    accR[t] = mfma16(ai, zi, accR[t]);
                    accI[t] = mfma16(ar, zi, accI[t]);
                    accI[t] = mfma16(-ai, zr, accI[t]);
                }
            }
        }
    }
    if (!active) return;
    double2* Cm = Cs + (int64_t)blockIdx.x * c_stride;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        if (t < cnt) {
            const int col = (J0 + t) * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = I * 16 + acc_row<R>(lk, r);
                if (row < s && col < s) Cm[(int64_t)row * s + col] = make_double2((double)accR[t][r], (double)accI[t][r]);
            }
        }
    }
}

template <typename R, int MAXT>
__global__ __launch_bounds__(LR_THREADS) void k_reproj_vjp(const cplx_t<R>* __restrict__ hb,
                                                           const cplx_t<R>* __restrict__ db,
                                                           const cplx_t<R>* __restrict__ gb,
                                                           cplx_t<R>* __restrict__ gdb,
                                                           cplx_t<R>* __restrict__ ghb,
                                                           const cplx_t<R>* __restrict__ wtab,
                                                           const LRDesc* __restrict__ descs, int m0,
                                                           const cplx_t<R>* __restrict__ Ss,
                                                           const cplx_t<R>* __restrict__ P2s, int64_t s_stride,
                                                           R inv_beta, R tau, R cz, R cdz, int KC) {
    using C = cplx_t<R>;
    using A4 = acc4_t<R>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const LRDesc d = descs[m0 + blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = lr_p(d), q = lr_q(d), side = lr_side(d);
    const int s = side == 0 ? q : p;
    const int l = side == 0 ? p : q;
    const int n = d.n, k = d.k, J = d.J, V = d.V;
    const int nt = (s + 15) / 16;
    const int s_pad = nt * 16;
    const int ldA = s_pad + 4;
    const int utab = V * J * n;
    C* Uh = reinterpret_cast<C*>(smem_raw);
    C* Ub = Uh + utab;
    C* Bacc = Ub + utab;
    R* Ar = reinterpret_cast<R*>(Bacc + utab);   // one pair of planes: the Zbar chunk, then the A chunk
    R* Ai = Ar + KC * ldA;
    C* Rst = reinterpret_cast<C*>(Ar);   // KC x s_pad complex fits in the two planes

    load_line_table<R>(Uh, hb, wtab, d, tid, LR_THREADS);
    load_line_table_at<R>(Ub, gb, d.b_off, d.b_cs, d.b_es, wtab, d, tid, LR_THREADS);
    for (int e = tid; e < utab; e += LR_THREADS) Bacc[e] = cmk<C>(0, 0);

    const C* Dm = db + d.d_off;
    C* Gm = gdb + d.d_off;
    const C* S = Ss + (int64_t)blockIdx.x * s_stride;
    const C* P2 = P2s + (int64_t)blockIdx.x * s_stride;
    const int li = lane & 15, lk = lane >> 4;
    const int rt = KC / 16;
    const int ntile = rt * nt;

    for (int r0 = 0; r0 < l; r0 += KC) {
        A4 accR[MAXT], accI[MAXT];
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            accR[t] = A4{0, 0, 0, 0};
            accI[t] = A4{0, 0, 0, 0};
        }
        // pass 0: Zbar_A chunk x S; pass 1: A chunk x P2
        for (int pass = 0; pass < 2; ++pass) {
            __syncthreads();
            if (pass == 0) stage_chunk<R>(Ar, Ai, ldA, Ub, cz, Gm, cdz, d, r0, KC, s_pad, tid, LR_THREADS);
            else stage_chunk<R>(Ar, Ai, ldA, Uh, (R)1, Dm, inv_beta, d, r0, KC, s_pad, tid, LR_THREADS);
            __syncthreads();
            const C* B = pass == 0 ? S : P2;
            for (int kk = 0; kk < s_pad; kk += 4) {
                const int kidx = kk + lk;
#pragma unroll
                for (int t = 0; t < MAXT; ++t) {
                    const int tile = wave + t * LR_WAVES;
                    if (tile < ntile) {
                        const int It = tile / nt, Jt = tile - It * nt;
                        const int arow = (It * 16 + li) * ldA + kidx;
                        const int col = Jt * 16 + li;
                        R br = 0, bi = 0;
                        if (kidx < s && col < s) {
                            const C bv = B[(int64_t)kidx * s + col];
                            br = bv.x;
                            bi = bv.y;
                        }
                        const R ar = Ar[arow], ai = Ai[arow];
                        accR[t] = mfma16(ar, br, accR[t]);
                        accR[t] = mfma16(-ai, bi, accR[t]);
                        accI[t] = mfma16(ar, bi, accI[t]);
                        accI[t] = mfma16(ai, br, accI[t]);
                    }
                }
            }
        }
        __syncthreads();   // the A planes are dead from here on; reuse them for the line cotangent terms
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            const int tile = wave + t * LR_WAVES;
            if (tile < ntile) {
                const int It = tile / nt, Jt = tile - It * nt;
                const int col = Jt * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rloc = It * 16 + acc_row<R>(lk, r);
                    const int row = r0 + rloc;
                    C lb = cmk<C>(0, 0);
                    if (row < l && col < s) {
                        int a, c;
                        C tb;
                        if (side == 0) { a = row; c = col; tb = cmk<C>(accR[t][r], accI[t][r]); }
                        else { a = col; c = row; tb = cmk<C>(accR[t][r], -accI[t][r]); }
                        const C rb = lift_val(Ub, n, k, a, c);
                        const int64_t di = (int64_t)a * q + c;
                        const C go = Gm[di];
                        C gp, gn;
                        gp.x = go.x - rb.x * inv_beta;
                        gp.y = go.y - rb.y * inv_beta;
                        gn.x = gp.x + tb.x * inv_beta;
                        gn.y = gp.y + tb.y * inv_beta;
                        Gm[di] = gn;
                        lb.x = tau * gp.x + tb.x;
                        lb.y = tau * gp.y + tb.y;
                    }
                    Rst[rloc * s_pad + col] = lb;
                }
            }
        }
        __syncthreads();
        const int rows_here = min(KC, l - r0);
        for (int e = tid; e < utab; e += LR_THREADS) {
            const int i = e % n, blk = e / n;
            C acc = Bacc[e];
            if (side == 0) {
                int a_lo = max(r0, i - k + 1), a_hi = min(r0 + rows_here - 1, min(i, p - 1));
                for (int a = a_lo; a <= a_hi; ++a) {
                    const C v = Rst[(a - r0) * s_pad + blk * k + (i - a)];
                    acc.x += v.x;
                    acc.y += v.y;
                }
            } else {
                int c_lo = max(r0, blk * k + max(0, i - p + 1));
                int c_hi = min(r0 + rows_here - 1, blk * k + min(k - 1, i));
                for (int c = c_lo; c <= c_hi; ++c) {
                    const int b = c - blk * k;
                    const C v = Rst[(c - r0) * s_pad + (i - b)];
                    acc.x += v.x;
                    acc.y += v.y;
                }
            }
            Bacc[e] = acc;
        }
    }
    __syncthreads();
    const int cc = n / 2;
    for (int e = tid; e < J * n; e += LR_THREADS) {
        const int i = e % n, j = e / n;
        C w = d.use_w ? wtab[d.w_off + i] : cmk<C>(1, 0);
        C out = cmulc(w, Bacc[j * n + i]);
        if (V == 2) {
            int fi = (2 * cc - i) % n;
            if (fi < 0) fi += n;
            C wf = d.use_w ? wtab[d.w_off + fi] : cmk<C>(1, 0);
            C g = cmulc(wf, Bacc[(J + j) * n + fi]);
            out.x += g.x;
            out.y -= g.y;
        }
        ghb[d.h_off + (int64_t)j * d.h_cs + (int64_t)i * d.h_es] = out;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename R>
static size_t gram_lds_bytes(int V, int J, int n, int s, int KC) {
    int s_pad = ((s + 15) / 16) * 16;
    return (size_t)V * J * n * sizeof(cplx_t<R>) + 2 * (size_t)KC * (s_pad + 4) * sizeof(R);
}
// stage: with the two staged steps of S (8 s_pad complex) after the A planes
template <typename R>
static size_t reproj_lds_bytes(int V, int J, int n, int s, int KC, bool stage = false) {
    int s_pad = ((s + 15) / 16) * 16;
    return 2 * (size_t)V * J * n * sizeof(cplx_t<R>) + 2 * (size_t)KC * (s_pad + 4) * sizeof(R) +
           (stage ? 8 * (size_t)s_pad * sizeof(cplx_t<R>) : 0);
}

constexpr size_t LDS_LIMIT = 160 * 1024;

bool lowrank_lds_fits(int csize, int V, int J, int n, int k) {
    LRDesc d{};
    d.n = n;
    d.k = k;
    d.J = J;
    d.V = V;
    const int s = lr_s(d);
    if (csize == 8)
        return gram_lds_bytes<float>(V, J, n, s, 4) <= LDS_LIMIT && reproj_lds_bytes<float>(V, J, n, s, 16) <= LDS_LIMIT;
    return gram_lds_bytes<double>(V, J, n, s, 4) <= LDS_LIMIT && reproj_lds_bytes<double>(V, J, n, s, 16) <= LDS_LIMIT;
}

template <typename R, int MAXT>
static hipError_t launch_gram_t(dim3 grid, size_t lds, hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db,
                                const cplx_t<R>* wtab, const LRDesc* descs, int m0, double2* Gs, int64_t gst,
                                R inv_beta, int KC) {
    hipError_t e = hipFuncSetAttribute((const void*)k_lift_gram<R, MAXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lift_gram<R, MAXT>), grid, dim3(LR_THREADS), lds, st, hb, db, wtab, descs, m0, Gs, gst,
                       inv_beta, KC);
    return hipGetLastError();
}

// LDS of the Gram kernel over several shapes: the largest
template <typename R>
static size_t gram_lds_max(const LRDesc* protos, int n_protos, int KC) {
    size_t b = 0;
    for (int i = 0; i < n_protos; ++i)
        b = std::max(b, gram_lds_bytes<R>(protos[i].V, protos[i].J, protos[i].n, lr_s(protos[i]), KC));
    return b;
}

// Launch the Gram kernel for matrices [m0, m0 + count) whose shapes are among the prototypes
// `protos`: one launch, sized for the largest (each block reads its own descriptor).
template <typename R>
hipError_t launch_lift_gram_multi(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* wtab,
                                  const LRDesc* descs_dev, const LRDesc* protos, int n_protos, int m0, int count,
                                  double2* Gs, int64_t g_stride, double beta, int kc) {
    if (n_protos < 1) return hipErrorInvalidValue;
    int s = 0;
    for (int i = 0; i < n_protos; ++i) s = std::max(s, lr_s(protos[i]));
    const int nt = (s + 15) / 16;
    // tiles per wave: the upper triangle's tiles over LR_WAVES * groups waves, at most 16 each
    const int n_tiles = nt * (nt + 1) / 2;
    int groups = 1;
    while ((n_tiles + LR_WAVES * groups - 1) / (LR_WAVES * groups) > 16) ++groups;
    const int need = (n_tiles + LR_WAVES * groups - 1) / (LR_WAVES * groups);
    // rows of A staged per chunk; by default 16, or 8 where that lets the kernel prefetch
    const int s_pad = nt * 16;
    int KC = 16;
    if (!gram_prefetches(sizeof(R), need, 16, s_pad) && gram_prefetches(sizeof(R), need, 8, s_pad)) KC = 8;
    if (kc == 4 || kc == 8 || kc == 16 || kc == 32) KC = kc;
    while (KC > 4 && gram_lds_max<R>(protos, n_protos, KC) > LDS_LIMIT) KC /= 2;
    const size_t lds = gram_lds_max<R>(protos, n_protos, KC);
    if (lds > LDS_LIMIT) return hipErrorInvalidValue;
    dim3 grid(count, groups);
    const R ib = (R)(1.0 / beta);
    if (need <= 4) return launch_gram_t<R, 4>(grid, lds, st, hb, db, wtab, descs_dev, m0, Gs, g_stride, ib, KC);
    if (need <= 8) return launch_gram_t<R, 8>(grid, lds, st, hb, db, wtab, descs_dev, m0, Gs, g_stride, ib, KC);
    if (need <= 12)
        return launch_gram_t<R, 12>(grid, lds, st, hb, db, wtab, descs_dev, m0, Gs, g_stride, ib, KC);
    if (need <= 16)
        return launch_gram_t<R, 16>(grid, lds, st, hb, db, wtab, descs_dev, m0, Gs, g_stride, ib, KC);
    return hipErrorInvalidValue;
}

// Launch the Gram kernel for matrices [m0, m0 + count) that share (V, J, n, k).
template <typename R>
hipError_t launch_lift_gram(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* wtab,
                            const LRDesc* descs_dev, const LRDesc& proto, int m0, int count, double2* Gs,
                            int64_t g_stride, double beta, int kc) {
    return launch_lift_gram_multi<R>(st, hb, db, wtab, descs_dev, &proto, 1, m0, count, Gs, g_stride, beta, kc);
}

template <typename R, int MAXT>
static hipError_t launch_reproj_t(dim3 grid, size_t lds, hipStream_t st, const cplx_t<R>* hb, cplx_t<R>* db,
                                  cplx_t<R>* bb, const cplx_t<R>* wtab, const LRDesc* descs, int m0,
                                  const cplx_t<R>* Ss, int64_t sst, R inv_beta, R tau, int KC, int stage) {
    hipError_t e = hipFuncSetAttribute((const void*)k_reproj<R, MAXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reproj<R, MAXT>), grid, dim3(LR_THREADS), lds, st, hb, db, bb, wtab, descs, m0, Ss, sst,
                       inv_beta, tau, KC, stage);
    return hipGetLastError();
}

// LDS of the reprojection kernel over several shapes: the largest
template <typename R>
static size_t reproj_lds_max(const LRDesc* protos, int n_protos, int KC, bool stage) {
    size_t b = 0;
    for (int i = 0; i < n_protos; ++i)
        b = std::max(b, reproj_lds_bytes<R>(protos[i].V, protos[i].J, protos[i].n, lr_s(protos[i]), KC, stage));
    return b;
}

// Launch the reprojection kernel for matrices [m0, m0 + count) whose shapes are among the
// prototypes `protos`: one launch with the chunk size every shape can take.
template <typename R>
hipError_t launch_reproj_multi(hipStream_t st, const cplx_t<R>* hb, cplx_t<R>* db, cplx_t<R>* bb,
                               const cplx_t<R>* wtab, const LRDesc* descs_dev, const LRDesc* protos, int n_protos,
                               int m0, int count, const cplx_t<R>* Ss, int64_t s_stride, double beta, double tau,
                               int kc) {
    if (n_protos < 1) return hipErrorInvalidValue;
    int s = 0, l_min = 1 << 30;
    for (int i = 0; i < n_protos; ++i) {
        s = std::max(s, lr_s(protos[i]));
        l_min = std::min(l_min, lr_l(protos[i]));
    }
    const int nt = (s + 15) / 16;
    int KC = (kc >= 16 && kc <= 64 && kc % 16 == 0) ? kc : 64;   // rows of A per chunk
    while (KC > 16 && (reproj_lds_max<R>(protos, n_protos, KC, false) > LDS_LIMIT || KC > ((l_min + 15) / 16) * 16))
        KC -= 16;
    size_t lds = reproj_lds_max<R>(protos, n_protos, KC, false);
    if (lds > LDS_LIMIT) return hipErrorInvalidValue;
    // rows of S staged through LDS where the space allows
    const int stage = reproj_lds_max<R>(protos, n_protos, KC, true) <= LDS_LIMIT ? 1 : 0;
    if (stage) lds = reproj_lds_max<R>(protos, n_protos, KC, true);
    // column tiles per wave: the fewest waves that share a row tile take ceil(nt / that) each
    const int need = (nt + LR_WAVES / (KC / 16) - 1) / (LR_WAVES / (KC / 16));
    dim3 grid(count);
    const R ib = (R)(1.0 / beta), tt = (R)tau;
    if (need <= 2)
        return launch_reproj_t<R, 2>(grid, lds, st, hb, db, bb, wtab, descs_dev, m0, Ss, s_stride, ib, tt, KC, stage);
    if (need <= 4)
        return launch_reproj_t<R, 4>(grid, lds, st, hb, db, bb, wtab, descs_dev, m0, Ss, s_stride, ib, tt, KC, stage);
    if (need <= 8)
        return launch_reproj_t<R, 8>(grid, lds, st, hb, db, bb, wtab, descs_dev, m0, Ss, s_stride, ib, tt, KC, stage);
    if (need <= 12)
        return launch_reproj_t<R, 12>(grid, lds, st, hb, db, bb, wtab, descs_dev, m0, Ss, s_stride, ib, tt, KC, stage);
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_reproj(hipStream_t st, const cplx_t<R>* hb, cplx_t<R>* db, cplx_t<R>* bb, const cplx_t<R>* wtab,
                         const LRDesc* descs_dev, const LRDesc& proto, int m0, int count, const cplx_t<R>* Ss,
                         int64_t s_stride, double beta, double tau, int kc) {
    return launch_reproj_multi<R>(st, hb, db, bb, wtab, descs_dev, &proto, 1, m0, count, Ss, s_stride, beta, tau, kc);
}

template hipError_t launch_lift_gram_multi<float>(hipStream_t, const float2*, const float2*, const float2*,
                                                  const LRDesc*, const LRDesc*, int, int, int, double2*, int64_t,
                                                  double, int);
template hipError_t launch_lift_gram_multi<double>(hipStream_t, const double2*, const double2*, const double2*,
                                                   const LRDesc*, const LRDesc*, int, int, int, double2*, int64_t,
                                                   double, int);
template hipError_t launch_reproj_multi<float>(hipStream_t, const float2*, float2*, float2*, const float2*,
                                               const LRDesc*, const LRDesc*, int, int, int, const float2*, int64_t,
                                               double, double, int);
template hipError_t launch_reproj_multi<double>(hipStream_t, const double2*, double2*, double2*, const double2*,
                                                const LRDesc*, const LRDesc*, int, int, int, const double2*, int64_t,
                                                double, double, int);
template hipError_t launch_lift_gram<float>(hipStream_t, const float2*, const float2*, const float2*, const LRDesc*,
                                            const LRDesc&, int, int, double2*, int64_t, double, int);
template hipError_t launch_lift_gram<double>(hipStream_t, const double2*, const double2*, const double2*,
                                             const LRDesc*, const LRDesc&, int, int, double2*, int64_t, double, int);
template hipError_t launch_reproj<float>(hipStream_t, const float2*, float2*, float2*, const float2*, const LRDesc*,
                                         const LRDesc&, int, int, const float2*, int64_t, double, double, int);
template hipError_t launch_reproj<double>(hipStream_t, const double2*, double2*, double2*, const double2*,
                                          const LRDesc*, const LRDesc&, int, int, const double2*, int64_t, double,
                                          double, int);

template <typename R>
static size_t cross_lds_bytes(int V, int J, int n, int s, int KC) {
    int s_pad = ((s + 15) / 16) * 16;
    return 2 * (size_t)V * J * n * sizeof(cplx_t<R>) + 4 * (size_t)KC * (s_pad + 4) * sizeof(R);
}
template <typename R>
static size_t reproj_vjp_lds_bytes(int V, int J, int n, int s, int KC) {
    int s_pad = ((s + 15) / 16) * 16;
    return 3 * (size_t)V * J * n * sizeof(cplx_t<R>) + 2 * (size_t)KC * (s_pad + 4) * sizeof(R);
}

bool lowrank_vjp_lds_fits(int csize, int V, int J, int n, int k) {
    LRDesc d{};
    d.n = n;
    d.k = k;
    d.J = J;
    d.V = V;
    const int s = lr_s(d);
    if (csize == 8)
        return cross_lds_bytes<float>(V, J, n, s, 4) <= LDS_LIMIT && reproj_vjp_lds_bytes<float>(V, J, n, s, 16) <= LDS_LIMIT;
    return cross_lds_bytes<double>(V, J, n, s, 4) <= LDS_LIMIT && reproj_vjp_lds_bytes<double>(V, J, n, s, 16) <= LDS_LIMIT;
}

template <typename R, int MAXT>
static hipError_t launch_cross_t(dim3 grid, size_t lds, hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db,
                                 const cplx_t<R>* gb, const cplx_t<R>* gdb, const cplx_t<R>* wtab,
                                 const LRDesc* descs, int m0, double2* Cs, int64_t c_stride, R ib, R cz, R cdz,
                                 int KC) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cross_gram<R, MAXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cross_gram<R, MAXT>), grid, dim3(LR_THREADS), lds, st, hb, db, gb, gdb, wtab, descs, m0,
                       Cs, c_stride, ib, cz, cdz, KC);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_cross_gram(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* gb,
                             const cplx_t<R>* gdb, const cplx_t<R>* wtab, const LRDesc* descs_dev,
                             const LRDesc& proto, int m0, int count, double2* Cs, int64_t c_stride, double beta,
                             double tau) {
    const int s = lr_s(proto);
    const int nt = (s + 15) / 16;
    constexpr int MAXT = sizeof(R) == 4 ? 8 : 4;
    const int nseg = (nt + MAXT - 1) / MAXT;
    const int groups = (nt * nseg + LR_WAVES - 1) / LR_WAVES;
    int KC = 16;
    while (KC > 4 && cross_lds_bytes<R>(proto.V, proto.J, proto.n, s, KC) > LDS_LIMIT) KC /= 2;
    const size_t lds = cross_lds_bytes<R>(proto.V, proto.J, proto.n, s, KC);
    if (lds > LDS_LIMIT) return hipErrorInvalidValue;
    return launch_cross_t<R, MAXT>(dim3(count, groups), lds, st, hb, db, gb, gdb, wtab, descs_dev, m0, Cs, c_stride,
                                   (R)(1.0 / beta), (R)(1.0 + tau / beta), (R)(-tau), KC);
}

template <typename R, int MAXT>
static hipError_t launch_reproj_vjp_t(dim3 grid, size_t lds, hipStream_t st, const cplx_t<R>* hb,
                                      const cplx_t<R>* db, const cplx_t<R>* gb, cplx_t<R>* gdb, cplx_t<R>* ghb,
                                      const cplx_t<R>* wtab, const LRDesc* descs, int m0, const cplx_t<R>* Ss,
                                      const cplx_t<R>* P2s, int64_t sst, R ib, R tau, R cz, R cdz, int KC) {
    hipError_t e = hipFuncSetAttribute((const void*)k_reproj_vjp<R, MAXT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reproj_vjp<R, MAXT>), grid, dim3(LR_THREADS), lds, st, hb, db, gb, gdb, ghb, wtab, descs,
                       m0, Ss, P2s, sst, ib, tau, cz, cdz, KC);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_reproj_vjp(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* gb,
                             cplx_t<R>* gdb, cplx_t<R>* ghb, const cplx_t<R>* wtab, const LRDesc* descs_dev,
                             const LRDesc& proto, int m0, int count, const cplx_t<R>* Ss, const cplx_t<R>* P2s,
                             int64_t s_stride, double beta, double tau) {
    const int s = lr_s(proto), l = lr_l(proto);
    const int nt = (s + 15) / 16;
    int KC = sizeof(R) == 4 ? 32 : 16;
    while (KC > 16 && (reproj_vjp_lds_bytes<R>(proto.V, proto.J, proto.n, s, KC) > LDS_LIMIT ||
                       KC > ((l + 15) / 16) * 16))
        KC -= 16;
    const size_t lds = reproj_vjp_lds_bytes<R>(proto.V, proto.J, proto.n, s, KC);
    if (lds > LDS_LIMIT) return hipErrorInvalidValue;
    const int tiles = (KC / 16) * nt;
    const int need = (tiles + LR_WAVES - 1) / LR_WAVES;
    const R ib = (R)(1.0 / beta), tt = (R)tau, cz = (R)(1.0 + tau / beta), cdz = (R)(-tau);
    dim3 grid(count);
    if (need <= 2)
        return launch_reproj_vjp_t<R, 2>(grid, lds, st, hb, db, gb, gdb, ghb, wtab, descs_dev, m0, Ss, P2s, s_stride,
                                         ib, tt, cz, cdz, KC);
    if (need <= 4)
        return launch_reproj_vjp_t<R, 4>(grid, lds, st, hb, db, gb, gdb, ghb, wtab, descs_dev, m0, Ss, P2s, s_stride,
                                         ib, tt, cz, cdz, KC);
    if (need <= 6)
        return launch_reproj_vjp_t<R, 6>(grid, lds, st, hb, db, gb, gdb, ghb, wtab, descs_dev, m0, Ss, P2s, s_stride,
                                         ib, tt, cz, cdz, KC);
    return hipErrorInvalidValue;
}

template hipError_t launch_cross_gram<float>(hipStream_t, const float2*, const float2*, const float2*, const float2*,
                                             const float2*, const LRDesc*, const LRDesc&, int, int, double2*, int64_t,
                                             double, double);
template hipError_t launch_cross_gram<double>(hipStream_t, const double2*, const double2*, const double2*,
                                              const double2*, const double2*, const LRDesc*, const LRDesc&, int, int,
                                              double2*, int64_t, double, double);
template hipError_t launch_reproj_vjp<float>(hipStream_t, const float2*, const float2*, const float2*, float2*, float2*,
                                             const float2*, const LRDesc*, const LRDesc&, int, int, const float2*,
                                             const float2*, int64_t, double, double);
template hipError_t launch_reproj_vjp<double>(hipStream_t, const double2*, const double2*, const double2*, double2*,
                                              double2*, const double2*, const LRDesc*, const LRDesc&, int, int,
                                              const double2*, const double2*, int64_t, double, double);

}  // namespace shlr
