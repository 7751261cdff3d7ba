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
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

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

// Per-slot scratch of the eigen-solver, in doubles, for matrices of order s.
__host__ __device__ inline int64_t eig_scratch_doubles(int s) { return 7LL * s * s + 16LL * s + 64; }

}  // namespace shlr
