// Shared device helpers for the SHLR kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shlr {

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename R> using cplx_t = typename cplx_of<R>::type;

template <typename C> __host__ __device__ inline C cmk(double re, double im) { C c; c.x = re; c.y = im; return c; }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// conj(a) * b
__device__ inline double2 cmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ inline float2 cmulc(float2 a, float2 b) { return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
// e / d without an integer division, for 0 <= e < 2^21 and 1 <= d < 2^24, from a reciprocal of d
// good to an ulp (v_rcp_f32): (e + 1/2) / d lies at least 1/(2d) from an integer, while the
// product's relative error (under 2^-22) moves it by less than (e + 1/2) 2^-22 / d < 1/(2d), so
// truncation gives the exact quotient.
__device__ inline int div_small(int e, int d) {
    return (int)(((float)e + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// acc + a b as four fused multiply-adds
__device__ inline double2 cfma(double2 a, double2 b, double2 acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// conj(a) b
__device__ inline double2 cconj_mul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -(a.y * b.x)));
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R> struct acc4_of;
template <> struct acc4_of<float> { using type = floatx4; };
template <> struct acc4_of<double> { using type = doublex4; };
template <typename R> using acc4_t = typename acc4_of<R>::type;

// 16x16x4 matrix-core step: D[i][j] += sum_k A[i][k] B[k][j].
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Element r of the
// accumulator of lane l holds D[acc_row<R>(l / 16, r)][l % 16]: row
// 4 * (l / 16) + r for the FP32 instruction, (l / 16) + 4 * r for FP64
// (both checked on gfx950).
__device__ inline floatx4 mfma16(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 mfma16(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename R> __device__ inline int acc_row(int lk, int r);
template <> __device__ inline int acc_row<float>(int lk, int r) { return 4 * lk + r; }
template <> __device__ inline int acc_row<double>(int lk, int r) { return lk + 4 * r; }

// Sum of a double over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (no LDS traffic).  The total is valid in lane 63 only.
__device__ inline double dpp_shift_d(double v, int ctrl_sel) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int rlo, rhi;
    switch (ctrl_sel) {
        case 1: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, true);
                rhi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, true); break;   // row_shr:1
        case 2: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x112, 0xf, 0xf, true);
                rhi = __builtin_amdgcn_update_dpp(0, hi, 0x112, 0xf, 0xf, true); break;   // row_shr:2
        case 4: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x114, 0xf, 0xf, true);
                rhi = __builtin_amdgcn_update_dpp(0, hi, 0x114, 0xf, 0xf, true); break;   // row_shr:4
        case 8: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x118, 0xf, 0xf, true);
                rhi = __builtin_amdgcn_update_dpp(0, hi, 0x118, 0xf, 0xf, true); break;   // row_shr:8
        case 15: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xa, 0xf, false);
                 rhi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xa, 0xf, false); break;  // row_bcast:15
        default: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xc, 0xf, false);
                 rhi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xc, 0xf, false); break;  // row_bcast:31
    }
    return __hiloint2double(rhi, rlo);
}
// sum over each row of 16 lanes, valid in the row's lane 15
__device__ inline double row16_sum_to15(double v) {
    v += dpp_shift_d(v, 1);
    v += dpp_shift_d(v, 2);
    v += dpp_shift_d(v, 4);
    v += dpp_shift_d(v, 8);
    return v;
}
// a double moved between lanes by a DPP control that reads a valid lane for every lane
template <int CTRL>
__device__ inline double dpp_move_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// the sum of a complex value over each quad of lanes, in every lane of the quad
__device__ inline double2 quad_sum_z(double2 v) {
    v.x += dpp_move_d<0xB1>(v.x);   // quad_perm [1,0,3,2]
    v.y += dpp_move_d<0xB1>(v.y);
    v.x += dpp_move_d<0x4E>(v.x);   // quad_perm [2,3,0,1]
    v.y += dpp_move_d<0x4E>(v.y);
    return v;
}
// Sums of x and of y over the four rows of 16 lanes (lanes l, l ^ 16, l ^ 32, l ^ 48), with
// the gfx950 lane-swap instructions.  permlane16_swap(a, b) exchanges the odd rows of a with
// the even rows of b, so swapping x with y leaves rows (x0, y0, x2, y2) and (x1, y1, x3, y3),
// whose sum pairs the rows; permlane32_swap(c, c) exchanges the halves of c.  On return lanes
// of rows 0 and 2 hold the sum of x, lanes of rows 1 and 3 the sum of y.
__device__ inline double colsum4_pair(double x, double y) {
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y),
                                                    false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y),
                                                    false, false);
    const double c = __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    const unsigned clo = (unsigned)__double2loint(c), chi = (unsigned)__double2hiint(c);
    const auto l2 = __builtin_amdgcn_permlane32_swap(clo, clo, false, false);
    const auto h2 = __builtin_amdgcn_permlane32_swap(chi, chi, false, false);
    return __hiloint2double((int)h2[0], (int)l2[0]) + __hiloint2double((int)h2[1], (int)l2[1]);
}
// the maximum over the 64 lanes, in every lane
__device__ inline double wave_max_all(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline double wave_sum_to63(double v) {
    v += dpp_shift_d(v, 1);
    v += dpp_shift_d(v, 2);
    v += dpp_shift_d(v, 4);
    v += dpp_shift_d(v, 8);
    v += dpp_shift_d(v, 15);
    v += dpp_shift_d(v, 31);
    return v;
}
// the same total broadcast to every lane
__device__ inline double wave_sum_all(double v) {
    v = wave_sum_to63(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Raw buffer access (gfx9 descriptor): 32-bit byte offsets from a wave-uniform
// base; an offset past the end reads 0 and a store there is dropped, which
// gives branch-free masked memory operations.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr unsigned BUF_OOB = 0x7ffffff0u;   // an offset beyond any buffer used here
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline double2 buf_load_d2(__amdgpu_buffer_rsrc_t r, unsigned off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return __builtin_bit_cast(double2, v);
}
__device__ inline void buf_store_d2(__amdgpu_buffer_rsrc_t r, unsigned off, double2 x) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), r, (int)off, 0, 0);
}

// Geometry and addressing of one lifted matrix (one line of J coils).
// Offsets count complex elements from the base pointers given to the kernels.
struct LRDesc {
    int64_t h_off;    // input line: coil 0, element 0
    int64_t b_off;    // output adjoint line: coil 0, element 0
    int64_t d_off;    // multiplier D, p x q row-major
    int32_t h_cs, h_es;  // input coil stride, element stride
    int32_t b_cs, b_es;  // output coil stride, element stride
    int32_t n, k, J, V;  // line length, window, coils, 1 + virtual coils
    int32_t use_w;       // 1: weights W applied
    int32_t w_off;       // offset of the n weights in the weight table
    double thr;          // singular-value threshold
};

__host__ __device__ inline int lr_p(const LRDesc& d) { return d.n - d.k + 1; }
__host__ __device__ inline int lr_q(const LRDesc& d) { return d.k * d.J * d.V; }
// side 0: A = T (l = p rows, s = q columns); side 1: A = T^H (l = q, s = p)
__host__ __device__ inline int lr_side(const LRDesc& d) { return lr_q(d) <= lr_p(d) ? 0 : 1; }
__host__ __device__ inline int lr_s(const LRDesc& d) { return lr_side(d) == 0 ? lr_q(d) : lr_p(d); }
__host__ __device__ inline int lr_l(const LRDesc& d) { return lr_side(d) == 0 ? lr_p(d) : lr_q(d); }

// Packed lower triangle of an s x s Hermitian matrix, column-major: entry (r, c), r >= c.
__host__ __device__ inline int64_t pk(int r, int c, int s) { return (int64_t)c * (2 * s - c - 1) / 2 + r; }
__host__ __device__ inline int64_t packed_size(int s) { return (int64_t)s * (s + 1) / 2; }

// Groups of 16 consecutive Householder reflectors (0 .. s-2) in the blocked back-transform.
__host__ __device__ inline int wy_groups(int s) { return (s + 14) / 16; }
// Per-slot scratch of the eigen-solver, in doubles, for matrices of order s: small vectors, the
// tridiagonal eigenvectors (s^2), the back-transformed vectors (2 s^2) and one 16 x 16 complex
// factor per reflector group.
__host__ __device__ inline int64_t eig_scratch_doubles(int s) {
    return 3LL * s * s + 16LL * s + 64 + 512LL * wy_groups(s);
}

// Reverse-mode arguments of the eigen-SVT kernel (all null in the forward).
template <typename OC>
struct VjpArgs {
    const double2* C = nullptr;   // per matrix s x s, row-major: A^H Zbar_A
    int64_t c_stride = 0;
    OC* P2 = nullptr;             // per matrix s x s output: 2 x (cotangent of G, Hermitian part)
    int64_t p2_stride = 0;
    double* scr = nullptr;        // per matrix scratch of eig_vjp_scratch_doubles(s)
    int64_t scr_stride = 0;
    double* tbar = nullptr;       // per descriptor: Re <Zbar, dZ/dthr> (may be null)
};
__host__ __device__ inline int64_t eig_vjp_scratch_doubles(int s) { return 14LL * s * s + 64; }

}  // namespace shlr
