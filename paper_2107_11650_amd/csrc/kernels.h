// Launchers of the SHLR kernels (host side) and the structs they take.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace shlr {

constexpr int FFT_MAX_STAGES = 24;

// n: line length; f: size of the FFT actually run (n, or for Bluestein's chirp-z
// transform a power of two >= 2n - 1); radix: the Stockham stages of size f.
struct FftPlan {
    int n;
    int f;
    int blue;
    int nst;
    int radix[FFT_MAX_STAGES];
};

// line g -> g1 = g / n0, g0 = g % n0; element t at base + g1*s1 + g0*s0 + t*es
struct LineAddr {
    int64_t base, s1, s0;
    int32_t n0, es;
};

// row g -> digits (d2, d1, d0); element i at d2*s2 + d1*s1 + d0*s0 + i*es
struct RowAddr {
    int64_t s2, s1, s0;
    int32_t es;
};

struct XupdRows {
    int n, n1, n0, n_rows;
    int rc_digit;                   // which digit indexes the rc table
    int unit_digit = -1;            // stop-test unit of a row: digit d2 when 2, else unit 0
    RowAddr bo, a, y, k, out, msk;  // msk counts bytes
    int64_t rr_off, rc_off;         // offsets into the real table
};

FftPlan make_fft_plan(int n);

// Segmented launches: the lines of several slices (each its own length and plan) in one launch.
// Segments are sorted by their first block; a block finds its segment by binary search.
struct FftSeg {
    FftPlan pl;
    LineAddr ia, oa;   // bases are offsets from the kernel's in / out pointers
    int n_lines, NL, block0, inverse;
    double scale;
};
struct XupdSeg {
    FftPlan pl;
    XupdRows x;
    int NL, block0, unit;                 // unit: stop-test unit (slice) of the rows
    int64_t bo, a, y, k, out, m;          // array offsets from the arena bases (m in bytes)
};
template <typename R>
FftSeg make_fft_seg(int n, int n_lines, int inverse, double scale, const LineAddr& ia, const LineAddr& oa, int block0,
                    size_t* lds);
template <typename R>
XupdSeg make_xupd_seg(const XupdRows& x, int block0, int unit, int64_t bo, int64_t a, int64_t y, int64_t k,
                      int64_t out, int64_t m, size_t* lds);
int fft_seg_blocks(const FftSeg& g);
int xupd_seg_blocks(const XupdSeg& g);
template <typename R>
hipError_t launch_fft_lines_seg(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, const FftSeg* segs_dev,
                                int n_seg, int blocks, size_t lds);
template <typename R>
hipError_t launch_xupd_rows_seg(hipStream_t st, cplx_t<R>* cbase, const uint8_t* mbase, const R* rtab,
                                const XupdSeg* segs_dev, int n_seg, int blocks, size_t lds, double lam, double beta,
                                int hard_dc, double* change, const int32_t* active);

template <typename R>
hipError_t launch_fft_lines(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, const LineAddr& ia,
                            const LineAddr& oa, int n, int n_lines, int inverse, double scale);
template <typename R>
hipError_t launch_xupd_rows(hipStream_t st, const cplx_t<R>* bo, const cplx_t<R>* a, const cplx_t<R>* y,
                            cplx_t<R>* k, cplx_t<R>* out, const uint8_t* m, const R* rtab, const XupdRows& x,
                            double lam, double beta, int hard_dc, double* change_acc,
                            const int32_t* active = nullptr);
template <typename R>
hipError_t launch_xupd_rows_rhs(hipStream_t st, const cplx_t<R>* bo, const cplx_t<R>* a, const cplx_t<R>* y,
                                cplx_t<R>* rhs, const uint8_t* m, const R* rtab, const XupdRows& x, double lam,
                                double beta);
// SPIRiT operator in three passes: number of partial sums of the fused row pass, 0 when the column
// pass does not fit the LDS
template <typename R>
int spirit_fused_blocks(int J, int M, int N);
template <typename R>
hipError_t launch_spirit_cols(hipStream_t st, const cplx_t<R>* t, cplx_t<R>* y, const cplx_t<R>* A, int J, int M,
                              int N);
// One step of the Chronopoulos-Gear form of preconditioned CG: partial-sum sets and scalar slots.
// gamma = <r, u>, delta = <u, A u>, u = r / den; slots = {gamma, gamma, alpha, alpha} by step parity.
struct CgStep {
    const double* gam0;       // gamma_0 (read by the first step)
    const double* gpart_in;   // partials of the gamma the kernel needs
    double* gpart_out;        // partials of gamma written by the first row pass
    const double* dpart_in;   // partials of delta_i (first row pass, final update)
    double* dpart_out;        // partials of delta written by the second row pass
    double* slots;
    int np;                   // partials per set (blocks of the row passes)
    int step;
    int setup;                // second row pass of the set-up: beta = 0
};
template <typename R>
hipError_t launch_fft_rows_cg1(hipStream_t st, cplx_t<R>* x, cplx_t<R>* r, const cplx_t<R>* p, const cplx_t<R>* s,
                               cplx_t<R>* t, int J, int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off,
                               int64_t rc_off, double lam, double beta, const CgStep& cs);
template <typename R>
hipError_t launch_fft_rows_cg3(hipStream_t st, const cplx_t<R>* y, const cplx_t<R>* r, cplx_t<R>* p, cplx_t<R>* s,
                               int J, int M, int N, const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off,
                               double lam, double beta, double lam1, const CgStep& cs);
template <typename R>
hipError_t launch_cg_final(hipStream_t st, cplx_t<R>* x, const cplx_t<R>* p, int64_t count, const CgStep& cs);
template <typename R>
hipError_t launch_fft_rows_apply(hipStream_t st, cplx_t<R>* io, const cplx_t<R>* p, int J, int M, int N,
                                 const uint8_t* mask, const R* rtab, int64_t rr_off, int64_t rc_off, double lam,
                                 double beta, double lam1, double* partials);
template <typename R>
hipError_t launch_scale_copy(hipStream_t st, const cplx_t<R>* in, cplx_t<R>* out, int64_t count,
                             const double* scale_ptr, int invert);
template <typename R>
hipError_t launch_fill_pattern(hipStream_t st, cplx_t<R>* out, int64_t count, const cplx_t<R>* table, int64_t div,
                               int64_t mod);
template <typename R>
hipError_t launch_fill_const(hipStream_t st, cplx_t<R>* out, int64_t count, double re, double im);
template <typename R>
hipError_t launch_fill_hash(hipStream_t st, cplx_t<R>* out, int64_t count, uint64_t seed, double scale);
template <typename R>
hipError_t launch_maxabs(hipStream_t st, const cplx_t<R>* in, int64_t count, unsigned long long* out, uint32_t* flags);
hipError_t launch_zero_doubles(hipStream_t st, double* p, int count);
// change[0] += sum |a - b|^2, change[1] += sum |b|^2 over count elements, and commit[i] = a[i] when commit is
// not null (it may be b); nothing happens when gate is not null and *gate == 0
template <typename R>
hipError_t launch_change_pair(hipStream_t st, const cplx_t<R>* a, const cplx_t<R>* b, int64_t count, double* change,
                              const int32_t* gate, cplx_t<R>* commit = nullptr);
// Relative-change stop of Algorithms S1 / S2 for n_units independent units: for every active unit,
// iters += 1, rel = change[2u] / change[2u + 1] and the unit stops (active = 0) when rel < tol; the
// number of units still active goes to *n_active.
hipError_t launch_stop_test(hipStream_t st, const double* change, int32_t* active, int32_t* iters, double* rel,
                            int n_units, double tol, int32_t* n_active);

// one launch over matrices of several shapes (the prototypes): sized for the largest
template <typename R>
hipError_t launch_lift_gram_multi(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* wtab,
                                  const LRDesc* descs_dev, const LRDesc* protos, int n_protos, int m0, int count,
                                  double2* Gs, int64_t g_stride, double beta, int kc);
template <typename R>
hipError_t launch_reproj_multi(hipStream_t st, const cplx_t<R>* hb, cplx_t<R>* db, cplx_t<R>* bb,
                               const cplx_t<R>* wtab, const LRDesc* descs_dev, const LRDesc* protos, int n_protos,
                               int m0, int count, const cplx_t<R>* Ss, int64_t s_stride, double beta, double tau,
                               int kc);
template <typename R>
hipError_t launch_lift_gram(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* wtab,
                            const LRDesc* descs_dev, const LRDesc& proto, int m0, int count, double2* Gs,
                            int64_t g_stride, double beta, int kc = 0);
template <typename R>
hipError_t launch_reproj(hipStream_t st, const cplx_t<R>* hb, cplx_t<R>* db, cplx_t<R>* bb, const cplx_t<R>* wtab,
                         const LRDesc* descs_dev, const LRDesc& proto, int m0, int count, const cplx_t<R>* Ss,
                         int64_t s_stride, double beta, double tau, int kc = 0);
template <typename R>
hipError_t launch_cross_gram(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* gb,
                             const cplx_t<R>* gdb, const cplx_t<R>* wtab, const LRDesc* descs_dev,
                             const LRDesc& proto, int m0, int count, double2* Cs, int64_t c_stride, double beta,
                             double tau);
template <typename R>
hipError_t launch_reproj_vjp(hipStream_t st, const cplx_t<R>* hb, const cplx_t<R>* db, const cplx_t<R>* gb,
                             cplx_t<R>* gdb, cplx_t<R>* ghb, const cplx_t<R>* wtab, const LRDesc* descs_dev,
                             const LRDesc& proto, int m0, int count, const cplx_t<R>* Ss, const cplx_t<R>* P2s,
                             int64_t s_stride, double beta, double tau);
constexpr int DC_VJP_BLOCKS = 512;   // partial sums per slice of the data-consistency backward
template <typename R>
hipError_t launch_dc_vjp(hipStream_t st, const cplx_t<R>* gk, const cplx_t<R>* K, const cplx_t<R>* Y,
                         const uint8_t* mask, const R* rr, const R* rc, int J, int M, int N, double lam, double beta,
                         cplx_t<R>* rbar, cplx_t<R>* gy, double* partials);
template <typename R>
hipError_t launch_add(hipStream_t st, cplx_t<R>* a, const cplx_t<R>* b, int64_t n);
// True when the reverse-mode kernels' LDS staging fits for this shape.
bool lowrank_vjp_lds_fits(int csize, int V, int J, int n, int k);
// True when the Gram and reprojection kernels' LDS staging for lifted matrices
// of this shape fits a compute unit (csize = 8 for complex64, 16 for complex128).
bool lowrank_lds_fits(int csize, int V, int J, int n, int k);
template <typename OC>
hipError_t launch_heig_svt(hipStream_t st, const LRDesc* descs, int m0, int count, double2* Gs, int64_t g_stride,
                           OC* Ss, int64_t s_stride, double* scr, int64_t scr_stride, int32_t* ranks,
                           double ortol_rel, uint32_t* flags, int smax, const VjpArgs<OC>& vj = VjpArgs<OC>(),
                           int tri_in = 0, double resid_lim = 1e-6);
// residual bound of the eigenpair check (relative to ||T|| ||z||) unless the caller sets another
constexpr double EIG_RESID_LIM_DEFAULT = 1e-6;
// Register-resident Householder reduction of the packed Gram matrices (orders 2..208): reflectors in
// place, diagonal / off-diagonal / h in the first 4 s doubles of each slot's scratch (then tri_in = 1).
// fp32: the matrix held in FP32 (the mixed form's forward iterations), orders up to 256; FP64 up to 208.
bool tridiag_rr_supported(int smax, bool fp32);
hipError_t launch_tridiag_rr(hipStream_t st, const LRDesc* descs, int m0, int count, double2* Gs, int64_t g_stride,
                             double* scr, int64_t scr_stride, int smax, bool fp32);

// ---- evaluation step (eval.hip) ----
constexpr int EVAL_MAX_PARTIALS = 8190;   // per-block partials a 64 KiB work buffer holds, with 2 result slots
constexpr int T2_MAX_ECHOES = 32;
struct TeList {
    int L;
    double te[T2_MAX_ECHOES];
};
template <typename R>
hipError_t launch_ssos(hipStream_t st, const cplx_t<R>* x, R* out, int n_img, int J, int64_t MN);
template <typename R>
hipError_t launch_rlne(hipStream_t st, const R* a, const R* b, const uint8_t* roi, int64_t count, double* work,
                       int* n_partials);
template <typename R>
hipError_t launch_mssim(hipStream_t st, const R* a, const R* b, int M, int N, double c1, double c2, double sigma,
                        double* work, int* n_partials);
// fixed-order sum (mode 0) or max (mode 1) of n partials (stride apart) into out[0]
hipError_t launch_reduce_partials(hipStream_t st, const double* partials, int n, int stride, int mode, double* out);
template <typename R>
hipError_t launch_max_real(hipStream_t st, const R* a, int64_t count, double* work, double* out);
template <typename R>
hipError_t launch_t2_fit(hipStream_t st, const R* img, int64_t npix, const TeList& te, double roi_frac, double t2_min,
                         double t2_max, R* t2, R* rho, uint8_t* roi, double* work);

}  // namespace shlr
