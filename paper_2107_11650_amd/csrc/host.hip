// C ABI of the SHLR library: plans, workspace layout and the orchestration of
// one ADMM iteration on one HIP stream.  All arithmetic runs in the kernels of
// fft.hip, lowrank.hip, eig.hip and spirit.hip; this file only validates,
// lays out memory and enqueues launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/shlr.h"
#include "common.h"
#include "kernels.h"

using namespace shlr;

static thread_local std::string g_last_error;

static shlr_status fail(shlr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(SHLR_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(_e));      \
    } while (0)

#define STCHK(call)                          \
    do {                                     \
        shlr_status _s = (call);             \
        if (_s != SHLR_OK) return _s;        \
    } while (0)

extern "C" const char* shlr_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* shlr_version(void) { return "shlr-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// host-side tables (FP64), shared by the two precisions
// ---------------------------------------------------------------------------

// W of Eq. 2: DFT of the circular first difference at the centred frequency
static void weights_host(int n, std::vector<double>& re, std::vector<double>& im) {
    re.resize(n);
    im.resize(n);
    for (int i = 0; i < n; ++i) {
        const double f = (double)(i - n / 2);
        re[i] = 1.0 - cos(2.0 * M_PI * f / n);
        im[i] = sin(2.0 * M_PI * f / n);
    }
}

static int flip_idx(int n, int i) { return ((2 * (n / 2) - i) % n + n) % n; }
static double hankel_count(int n, int k, int i) {
    return (double)std::min(std::min(i + 1, k), std::min(n - k + 1, n - i));
}

// Diagonal of (lift)^*(lift) on one line (the Eq. 15 / S7 Hankel terms) for the weights (wr, wi)
static std::vector<double> gram_diag_host(int n, int k, bool use_w, bool vc, const std::vector<double>& wr,
                                          const std::vector<double>& wi) {
    std::vector<double> r(n);
    for (int i = 0; i < n; ++i) {
        const double a = use_w ? wr[i] * wr[i] + wi[i] * wi[i] : 1.0;
        r[i] = hankel_count(n, k, i) * a;
        if (vc) {
            const int f = flip_idx(n, i);
            const double af = use_w ? wr[f] * wr[f] + wi[f] * wi[f] : 1.0;
            r[i] += hankel_count(n, k, f) * af;
        }
    }
    return r;
}

static std::vector<double> gram_diag_host(int n, int k, bool use_w, bool vc) {
    std::vector<double> wr, wi;
    weights_host(n, wr, wi);
    return gram_diag_host(n, k, use_w, vc, wr, wi);
}

// lift^*(const * ones): the initial adjoint term for D = d0, Z = 0 (same on every line), weights (wr, wi)
static void init_adjoint_host(int n, int k, bool use_w, bool vc, double cst, const std::vector<double>& wr,
                              const std::vector<double>& wi, std::vector<double>& re, std::vector<double>& im) {
    re.assign(n, 0.0);
    im.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        const double c = hankel_count(n, k, i) * cst;
        const double ar = use_w ? wr[i] : 1.0, ai = use_w ? wi[i] : 0.0;
        re[i] += ar * c;  // conj(w) * c
        im[i] += -ai * c;
        if (vc) {
            const int f = flip_idx(n, i);
            const double cf = hankel_count(n, k, f) * cst;
            const double fr = use_w ? wr[f] : 1.0, fi = use_w ? wi[f] : 0.0;
            // conj(conj(w_f) * cf) = w_f * cf
            re[i] += fr * cf;
            im[i] += fi * cf;
        }
    }
}
static void init_adjoint_host(int n, int k, bool use_w, bool vc, double cst, std::vector<double>& re,
                              std::vector<double>& im) {
    std::vector<double> wr, wi;
    weights_host(n, wr, wi);
    init_adjoint_host(n, k, use_w, vc, cst, wr, wi, re, im);
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------

struct LRGroup {
    int first, count;  // descriptors [first, first + count)
    LRDesc proto;
    int gram_kc = 0, reproj_kc = 0;   // rows of A per chunk (0: the launchers' default)
};

// Consecutive groups of one eigen-solver class whose matrix orders are within a
// factor 2 share the eigen-solver slots: chunks of up to `slots` matrices,
// strides for order smax.
struct LRRun {
    int first, count;      // descriptors [first, first + count)
    int g0, g1;            // groups [g0, g1)
    int smax, slots;
    int64_t g_stride, s_stride, scr_stride;
    int rr = -1;           // Householder reduction: 1 registers, 0 memory, -1 registers when supported
};

// complex64 data (the two mixed forms) or complex128 (the FP64 form)
static bool prec_c64(int prec) { return prec == SHLR_PREC_MIXED || prec == SHLR_PREC_MIXED_R32; }
static bool prec_valid(int prec) { return prec == SHLR_PREC_MIXED || prec == SHLR_PREC_FP64 || prec == SHLR_PREC_MIXED_R32; }
// the Householder reduction in FP32 (opt-in form only)
static bool prec_r32(int prec) { return prec == SHLR_PREC_MIXED_R32; }

static int run_uses_rr(const LRRun& r, bool fp32) {
    return r.rr >= 0 ? r.rr : (tridiag_rr_supported(r.smax, fp32) ? 1 : 0);
}

struct SliceLayout {
    int M, N;
    // complex offsets (elements of the working complex type)
    int64_t yn, k, a, hr, hct, br, bct, dr, dc;
    // PARAM
    int64_t bp, be, xe, dp, de;
    int64_t mask_b;        // byte offset of the mask copy
    int64_t rr, rc;        // real-table offsets (elements of the working real type)
    int64_t wr, wc;        // complex weight-table offsets (elements)
    int64_t vr, vc;        // complex init-pattern offsets
};

struct shlr_plan {
    shlr_params p;
    std::vector<int32_t> Ms, Ns;
    int csize;   // bytes per complex
    int rsize;   // bytes per real
    std::vector<SliceLayout> sl;
    std::vector<LRDesc> descs;
    std::vector<LRGroup> groups;
    int s_max = 0;
    std::vector<LRRun> runs;
    size_t bytes_g = 0, bytes_s = 0, bytes_scr = 0;   // slot regions (max over runs)
    // byte offsets in the workspace
    size_t off_c = 0, bytes_c = 0;      // complex arena
    size_t off_r = 0, bytes_r = 0;      // real arena
    size_t off_m = 0, bytes_m = 0;      // mask arena
    size_t off_desc = 0, off_g = 0, off_s = 0, off_scr = 0, off_ranks = 0, off_scal = 0;
    size_t off_spirit = 0, bytes_spirit = 0;
    // segmented launches of the X-update phase (PI): every slice's lines in one launch per step
    std::vector<FftSeg> seg_fwd, seg_inv;   // column transforms B_row -> A and K -> H_row
    std::vector<XupdSeg> seg_x;             // fused row transform, Eq. 15 division, inverse (no SPIRiT)
    int blk_fwd = 0, blk_inv = 0, blk_x = 0;
    size_t lds_fwd = 0, lds_inv = 0, lds_x = 0;
    size_t off_seg = 0, bytes_seg = 0;
    size_t total = 0;
    // host tables uploaded at bind
    std::vector<double> rtab;                      // real table (FP64, converted at upload)
    std::vector<double> ctab;                      // complex table interleaved (FP64)
    // device state
    unsigned char* ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false, initialised = false;
    std::vector<double> scales;
    int64_t total_elems = 0;  // complex elements of Y
    int n_units = 1;          // units of the relative-change stop: slices (PI) or FE positions (PARAM)
    int64_t d_block_off = 0, d_block_elems = 0;   // PI: the multipliers of all slices (complex elements)
    // reverse mode: the forward with checkpoints that the backward may follow
    int unrolled_n = 0;
    const void* unrolled_ckpt = nullptr;
    // spirit
    bool spirit_ready = false;
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int iters_total = 0;
    bool tuned = false;   // shlr_autotune chose the launch parameters
    double eig_resid_lim = EIG_RESID_LIM_DEFAULT;   // eigenpair check of the eigen-solver (shlr_set_eig_check)
    // per-phase HIP-event timing (phase: 0 transforms + X-update, 1 Gram, 2 eigen-SVT, 3 reprojection, 4 SPIRiT,
    // 5 register-resident Householder reduction)
    bool timing = false;
    uint32_t timing_mask = 0x3f;   // phases timed while timing is on
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, std::pair<size_t, size_t>>> ev_marks;  // (phase, (start, stop))
    double t_ms[8] = {0};
    int t_cnt[8] = {0};
};

// event helpers: a phase is bracketed by two events on the plan's stream
static shlr_status ev_get(shlr_plan* P, size_t* idx) {
    if (P->ev_used == P->ev_pool.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        P->ev_pool.push_back(e);
    }
    *idx = P->ev_used++;
    return SHLR_OK;
}
static bool phase_timed(const shlr_plan* P, int phase) { return P->timing && ((P->timing_mask >> phase) & 1u); }
static shlr_status phase_begin(shlr_plan* P, int phase, size_t* start) {
    if (!phase_timed(P, phase)) return SHLR_OK;
    STCHK(ev_get(P, start));
    HIPCHK(hipEventRecord(P->ev_pool[*start], P->stream));
    return SHLR_OK;
}
static shlr_status phase_end(shlr_plan* P, int phase, size_t start) {
    if (!phase_timed(P, phase)) return SHLR_OK;
    size_t stop;
    STCHK(ev_get(P, &stop));
    HIPCHK(hipEventRecord(P->ev_pool[stop], P->stream));
    P->ev_marks.push_back({phase, {start, stop}});
    return SHLR_OK;
}
static shlr_status timing_collect(shlr_plan* P) {
    if (P->ev_marks.empty()) return SHLR_OK;
    HIPCHK(hipStreamSynchronize(P->stream));
    for (auto& m : P->ev_marks) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, P->ev_pool[m.second.first], P->ev_pool[m.second.second]));
        P->t_ms[m.first] += ms;
        P->t_cnt[m.first] += 1;
    }
    P->ev_marks.clear();
    P->ev_used = 0;
    return SHLR_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static size_t scal_bytes(int n_slices, int n_units) { return (size_t)n_slices * 16 + 64 + (size_t)n_units * 32 + 64; }

static size_t spirit_bytes(const shlr_plan* P);

static shlr_status validate(const shlr_params* p) {
    if (!p) return fail(SHLR_E_INVALID_ARG, "params is NULL");
    if (p->model != SHLR_MODEL_PI && p->model != SHLR_MODEL_PARAM)
        return fail(SHLR_E_INVALID_ARG, "model must be SHLR_MODEL_PI or SHLR_MODEL_PARAM");
    if (!prec_valid(p->precision))
        return fail(SHLR_E_INVALID_ARG, "precision must be SHLR_PREC_MIXED, SHLR_PREC_FP64 or SHLR_PREC_MIXED_R32");
    if (p->n_slices < 1 || p->n_slices > SHLR_MAX_SLICES)
        return fail(SHLR_E_INVALID_ARG, "n_slices must be in [1, %d]", SHLR_MAX_SLICES);
    if (p->model == SHLR_MODEL_PARAM && p->n_slices != 1)
        return fail(SHLR_E_INVALID_ARG, "the parameter-imaging model takes one series (n_slices = 1)");
    if (!p->M || !p->N) return fail(SHLR_E_INVALID_ARG, "M and N must be host arrays");
    if (p->J < 1 || p->J > 64) return fail(SHLR_E_INVALID_ARG, "J must be in [1, 64]");
    if (!(p->beta > 0) || !isfinite(p->beta)) return fail(SHLR_E_INVALID_ARG, "beta must be positive and finite");
    if (!(p->tau > 0) || !isfinite(p->tau)) return fail(SHLR_E_INVALID_ARG, "tau must be positive and finite");
    if (!p->hard_dc && (!(p->lambda > 0) || !isfinite(p->lambda)))
        return fail(SHLR_E_INVALID_ARG, "lambda must be positive and finite (or set hard_dc)");
    if (!(p->lambda1 >= 0) || !isfinite(p->lambda1)) return fail(SHLR_E_INVALID_ARG, "lambda1 must be >= 0");
    if (!isfinite(p->d0)) return fail(SHLR_E_INVALID_ARG, "d0 must be finite");
    if (p->slot_budget < 0) return fail(SHLR_E_INVALID_ARG, "slot_budget must be >= 0 (0: the default)");
    if (p->max_iter < 0) return fail(SHLR_E_INVALID_ARG, "max_iter must be >= 0");
    if (p->model == SHLR_MODEL_PARAM) {
        if (p->L < 2 || p->L > 512) return fail(SHLR_E_INVALID_ARG, "L must be in [2, 512]");
        if (!(p->lambda2 > 0) || !isfinite(p->lambda2)) return fail(SHLR_E_INVALID_ARG, "lambda2 must be positive");
        if (p->spirit_ksize != 0) return fail(SHLR_E_UNSUPPORTED, "the SPIRiT term is defined for the PI model only");
    }
    if (p->spirit_ksize < 0 || (p->spirit_ksize > 0 && (p->spirit_ksize % 2 == 0 || p->spirit_ksize > 9)))
        return fail(SHLR_E_INVALID_ARG, "spirit_ksize must be 0 or odd in [1, 9]");
    if (p->spirit_ksize > 0 && p->hard_dc) return fail(SHLR_E_UNSUPPORTED, "SPIRiT with hard data consistency");
    if (p->spirit_ksize > 0 && p->n_cg < 1) return fail(SHLR_E_INVALID_ARG, "n_cg must be >= 1 with SPIRiT");
    for (int s = 0; s < p->n_slices; ++s) {
        const int M = p->M[s], N = p->N[s];
        if (M < 1 || N < 1 || M > 4096 || N > 4096) return fail(SHLR_E_INVALID_ARG, "slice %d: bad size %dx%d", s, M, N);
        const int nr = N, nc = (p->model == SHLR_MODEL_PI) ? M : p->L;
        if (p->k_row < 1 || p->k_row > nr) return fail(SHLR_E_INVALID_ARG, "k_row must be in [1, %d]", nr);
        if (p->k_col < 1 || p->k_col > nc) return fail(SHLR_E_INVALID_ARG, "k_col must be in [1, %d]", nc);
        const int V = p->use_vc ? 2 : 1;
        const int pr = nr - p->k_row + 1, qr = p->k_row * p->J * V;
        const int Vc = (p->model == SHLR_MODEL_PI) ? V : 1;
        const int pc = nc - p->k_col + 1, qc = p->k_col * p->J * Vc;
        if (std::min(pr, qr) > 320 || std::min(pc, qc) > 320)
            return fail(SHLR_E_UNSUPPORTED, "lifted matrices with min(p, q) > 320 are not supported");
        if (std::max(pr, qr) > 4096 || std::max(pc, qc) > 4096)
            return fail(SHLR_E_UNSUPPORTED, "lifted matrices with max(p, q) > 4096 are not supported");
        const int cs = prec_c64(p->precision) ? 8 : 16;
        if (!lowrank_lds_fits(cs, V, p->J, nr, p->k_row) || !lowrank_lds_fits(cs, Vc, p->J, nc, p->k_col))
            return fail(SHLR_E_UNSUPPORTED, "slice %d: the line table of a lifted matrix (V*J*n = %d) exceeds the "
                        "LDS staging of this precision", s, V * p->J * std::max(nr, nc));
    }
    return SHLR_OK;
}

static LRDesc make_desc(int64_t h_off, int h_cs, int h_es, int64_t b_off, int b_cs, int b_es, int64_t d_off, int n,
                        int k, int J, int V, int use_w, int64_t w_off, double thr) {
    LRDesc d;
    d.h_off = h_off;
    d.b_off = b_off;
    d.d_off = d_off;
    d.h_cs = h_cs;
    d.h_es = h_es;
    d.b_cs = b_cs;
    d.b_es = b_es;
    d.n = n;
    d.k = k;
    d.J = J;
    d.V = V;
    d.use_w = use_w;
    d.w_off = (int32_t)w_off;
    d.thr = thr;
    return d;
}

static const size_t SLOT_BUDGET = (size_t)16 << 30;   // eigen-solver scratch for one chunk (of 288 GB HBM)

// Eigen-solver class of a matrix order: register-resident reductions (order <= 208, or <= 256
// in FP32) apart from in-memory ones, then by the number of 64-row tiles the eigen kernel is
// built for.
static int order_class(int s, bool fp32) { return (tridiag_rr_supported(s, fp32) ? 0 : 16) + (s + 63) / 64; }

// Groups sorted by class (stable), the descriptors laid out again in that order, so that the
// runs formed below hold matrices of one class.
static void order_groups(shlr_plan* P) {
    const bool fp32 = prec_r32(P->p.precision);
    std::vector<int> idx(P->groups.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return order_class(lr_s(P->groups[a].proto), fp32) < order_class(lr_s(P->groups[b].proto), fp32);
    });
    std::vector<LRDesc> d;
    std::vector<LRGroup> g;
    d.reserve(P->descs.size());
    for (int i : idx) {
        LRGroup x = P->groups[i];
        const int first = (int)d.size();
        for (int k = 0; k < x.count; ++k) d.push_back(P->descs[x.first + k]);
        x.first = first;
        g.push_back(x);
    }
    P->descs.swap(d);
    P->groups.swap(g);
}

static void layout_slots(shlr_plan* P) {
    const bool fp32 = prec_r32(P->p.precision);
    P->runs.clear();
    P->bytes_g = P->bytes_s = P->bytes_scr = 0;
    for (int gi = 0; gi < (int)P->groups.size(); ++gi) {
        const LRGroup& g = P->groups[gi];
        const int sg = lr_s(g.proto);
        if (!P->runs.empty()) {
            LRRun& r = P->runs.back();
            int lo = sg, hi = sg;
            for (int gj = r.g0; gj < r.g1; ++gj) {
                lo = std::min(lo, lr_s(P->groups[gj].proto));
                hi = std::max(hi, lr_s(P->groups[gj].proto));
            }
            if (hi <= 2 * lo && order_class(sg, fp32) == order_class(r.smax, fp32)) {
                r.g1 = gi + 1;
                r.count += g.count;
                r.smax = hi;
                continue;
            }
        }
        LRRun r{};
        r.first = g.first;
        r.count = g.count;
        r.g0 = gi;
        r.g1 = gi + 1;
        r.smax = sg;
        P->runs.push_back(r);
    }
    for (LRRun& r : P->runs) {
        r.g_stride = packed_size(r.smax);                    // double2, packed lower triangle
        r.s_stride = (int64_t)r.smax * r.smax;                // working complex
        r.scr_stride = eig_scratch_doubles(r.smax);           // doubles
        const size_t per = r.g_stride * 16 + r.s_stride * P->csize + r.scr_stride * 8 + 3 * 256;
        const size_t budget = P->p.slot_budget > 0 ? (size_t)P->p.slot_budget : SLOT_BUDGET;
        r.slots = (int)std::min<size_t>((size_t)r.count, std::max<size_t>(1, budget / per));
        P->bytes_g = std::max(P->bytes_g, (size_t)r.slots * r.g_stride * 16);
        P->bytes_s = std::max(P->bytes_s, (size_t)r.slots * r.s_stride * P->csize);
        P->bytes_scr = std::max(P->bytes_scr, (size_t)r.slots * r.scr_stride * 8);
    }
}

extern "C" shlr_status shlr_params_default(int32_t model, shlr_params* p) {
    if (!p) return fail(SHLR_E_INVALID_ARG, "p is NULL");
    if (model != SHLR_MODEL_PI && model != SHLR_MODEL_PARAM)
        return fail(SHLR_E_INVALID_ARG, "model must be SHLR_MODEL_PI or SHLR_MODEL_PARAM");
    memset(p, 0, sizeof(*p));
    p->model = model;
    p->precision = SHLR_PREC_MIXED;
    p->n_slices = 1;
    p->use_w = 1;
    p->normalize = 1;
    p->max_iter = model == SHLR_MODEL_PI ? 50 : 100;   // Algorithm S1 / Algorithm S2 caps
    p->tol = 1e-6;                                     // their relative-change tolerance
    p->d0 = 1.0;                                       // their initial multipliers
    p->n_cg = 10;
    return SHLR_OK;
}

// Segment tables of the X-update phase of the PI model: one entry per slice, blocks numbered
// consecutively over the slices, so that each step of the phase is one launch for the whole batch.
template <typename R>
static void build_segments(shlr_plan* P) {
    const int J = P->p.J;
    P->seg_fwd.clear();
    P->seg_inv.clear();
    P->seg_x.clear();
    P->blk_fwd = P->blk_inv = P->blk_x = 0;
    P->lds_fwd = P->lds_inv = P->lds_x = 0;
    for (int si = 0; si < (int)P->sl.size(); ++si) {
        const SliceLayout& L = P->sl[si];
        const int M = L.M, N = L.N;
        const int64_t MN = (int64_t)M * N;
        size_t lds = 0;
        // lines (j, n) along m
        FftSeg f = make_fft_seg<R>(M, J * N, 0, 1.0 / sqrt((double)M), LineAddr{L.br, MN, 1, N, N},
                                   LineAddr{L.a, MN, 1, N, N}, P->blk_fwd, &lds);
        P->lds_fwd = std::max(P->lds_fwd, lds);
        P->blk_fwd += fft_seg_blocks(f);
        P->seg_fwd.push_back(f);
        FftSeg g = make_fft_seg<R>(M, J * N, 1, 1.0 / sqrt((double)M), LineAddr{L.k, MN, 1, N, N},
                                   LineAddr{L.hr, MN, 1, N, N}, P->blk_inv, &lds);
        P->lds_inv = std::max(P->lds_inv, lds);
        P->blk_inv += fft_seg_blocks(g);
        P->seg_inv.push_back(g);
        XupdRows x;
        x.n = N;
        x.n1 = J;
        x.n0 = M;
        x.n_rows = J * M;
        x.rc_digit = 0;
        x.bo = RowAddr{0, MN, 1, M};
        x.a = RowAddr{0, MN, N, 1};
        x.y = x.a;
        x.k = x.a;
        x.out = RowAddr{0, MN, 1, M};
        x.msk = RowAddr{0, 0, N, 1};
        x.rr_off = L.rr;
        x.rc_off = L.rc;
        XupdSeg xs = make_xupd_seg<R>(x, P->blk_x, si, L.bct, L.a, L.yn, L.k, L.hct, L.mask_b, &lds);
        P->lds_x = std::max(P->lds_x, lds);
        P->blk_x += xupd_seg_blocks(xs);
        P->seg_x.push_back(xs);
    }
    P->bytes_seg = align256(P->seg_fwd.size() * sizeof(FftSeg)) + align256(P->seg_inv.size() * sizeof(FftSeg)) +
                   align256(P->seg_x.size() * sizeof(XupdSeg));
}

extern "C" shlr_status shlr_plan_create(const shlr_params* p, shlr_plan** out) {
    if (!out) return fail(SHLR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    STCHK(validate(p));
    shlr_plan* P = new shlr_plan();
    P->p = *p;
    P->Ms.assign(p->M, p->M + p->n_slices);
    P->Ns.assign(p->N, p->N + p->n_slices);
    P->p.M = nullptr;
    P->p.N = nullptr;
    P->csize = prec_c64(p->precision) ? 8 : 16;
    P->rsize = prec_c64(p->precision) ? 4 : 8;
    const int J = p->J, V = p->use_vc ? 2 : 1;
    int64_t c = 0, r = 0, m = 0;
    auto cal = [&](int64_t n) { int64_t o = c; c += n; c = (c + 31) & ~(int64_t)31; return o; };
    auto ral = [&](int64_t n) { int64_t o = r; r += n; r = (r + 63) & ~(int64_t)63; return o; };
    auto mal = [&](int64_t n) { int64_t o = m; m += n; m = (m + 255) & ~(int64_t)255; return o; };
    std::vector<double>& rt = P->rtab;
    std::vector<double>& ct = P->ctab;
    auto put_real = [&](int64_t off, const std::vector<double>& v) {
        if ((int64_t)rt.size() < off + (int64_t)v.size()) rt.resize(off + v.size(), 0.0);
        for (size_t i = 0; i < v.size(); ++i) rt[off + i] = v[i];
    };
    std::vector<double> ctmp;
    // complex host table (weights + init patterns): stored densely, copied into the complex arena
    auto put_cplx = [&](const std::vector<double>& re, const std::vector<double>& im) {
        int64_t o = (int64_t)ct.size() / 2;
        for (size_t i = 0; i < re.size(); ++i) {
            ct.push_back(re[i]);
            ct.push_back(im[i]);
        }
        return o;
    };
    std::vector<double> wr, wi, vr, vi;
    const double thr_rc = 1.0 / p->beta;
    if (p->model == SHLR_MODEL_PI) {
        for (int s = 0; s < p->n_slices; ++s) {
            SliceLayout L{};
            const int M = P->Ms[s], N = P->Ns[s];
            L.M = M;
            L.N = N;
            const int64_t e = (int64_t)J * M * N;
            L.yn = cal(e);
            L.k = cal(e);
            L.a = cal(e);
            L.hr = cal(e);
            L.hct = cal(e);
            L.br = cal(e);
            L.bct = cal(e);
            L.mask_b = mal((int64_t)M * N);
            L.rr = ral(N);
            L.rc = ral(M);
            put_real(L.rr, gram_diag_host(N, p->k_row, p->use_w, p->use_vc));
            put_real(L.rc, gram_diag_host(M, p->k_col, p->use_w, p->use_vc));
            P->total_elems += e;
            P->sl.push_back(L);
        }
        // the multipliers of all slices form one contiguous block (checkpoints copy it whole)
        P->d_block_off = c;
        for (int s = 0; s < p->n_slices; ++s) {
            SliceLayout& L = P->sl[s];
            const int M = L.M, N = L.N;
            const int pr = N - p->k_row + 1, qr = p->k_row * J * V;
            const int pc = M - p->k_col + 1, qc = p->k_col * J * V;
            L.dr = cal((int64_t)M * pr * qr);
            L.dc = cal((int64_t)N * pc * qc);
        }
        P->d_block_elems = c - P->d_block_off;
        // complex tables after the per-slice arrays
        for (int s = 0; s < p->n_slices; ++s) {
            SliceLayout& L = P->sl[s];
            weights_host(L.N, wr, wi);
            L.wr = put_cplx(wr, wi);
            weights_host(L.M, wr, wi);
            L.wc = put_cplx(wr, wi);
            init_adjoint_host(L.N, p->k_row, p->use_w, p->use_vc, -p->d0 / p->beta, vr, vi);
            L.vr = put_cplx(vr, vi);
            init_adjoint_host(L.M, p->k_col, p->use_w, p->use_vc, -p->d0 / p->beta, vr, vi);
            L.vc = put_cplx(vr, vi);
        }
    } else {
        SliceLayout L{};
        const int M = P->Ms[0], N = P->Ns[0], Lh = p->L;
        L.M = M;
        L.N = N;
        const int64_t e = (int64_t)Lh * J * M * N;
        L.yn = cal(e);
        L.k = cal(e);
        L.bp = cal(e);
        L.be = cal(e);
        L.xe = cal(e);
        const int pp = N - p->k_row + 1, qp = p->k_row * J * V;
        const int pe = Lh - p->k_col + 1, qe = p->k_col * J;
        L.dp = cal((int64_t)M * Lh * pp * qp);
        L.de = cal((int64_t)M * N * pe * qe);
        L.mask_b = mal((int64_t)Lh * N);
        L.rr = ral(N);
        L.rc = ral(Lh);
        put_real(L.rr, gram_diag_host(N, p->k_row, p->use_w, p->use_vc));
        put_real(L.rc, gram_diag_host(Lh, p->k_col, false, false));
        weights_host(N, wr, wi);
        L.wr = put_cplx(wr, wi);
        L.wc = L.wr;
        init_adjoint_host(N, p->k_row, p->use_w, p->use_vc, -p->d0 / p->beta, vr, vi);
        L.vr = put_cplx(vr, vi);
        init_adjoint_host(Lh, p->k_col, false, false, -p->d0 / p->beta, vr, vi);
        L.vc = put_cplx(vr, vi);
        P->total_elems = e;
        P->sl.push_back(L);
    }
    // the complex table lives at the end of the complex arena
    const int64_t ctab_off = cal((int64_t)P->ctab.size() / 2 + 1);
    for (auto& L : P->sl) {
        L.wr += ctab_off;
        L.wc += ctab_off;
        L.vr += ctab_off;
        L.vc += ctab_off;
    }
    // descriptors
    if (p->model == SHLR_MODEL_PI) {
        for (int s = 0; s < p->n_slices; ++s) {
            const SliceLayout& L = P->sl[s];
            const int M = L.M, N = L.N;
            const int pr = N - p->k_row + 1, qr = p->k_row * J * V;
            const int pc = M - p->k_col + 1, qc = p->k_col * J * V;
            LRGroup g;
            g.first = (int)P->descs.size();
            g.count = M;
            for (int mm = 0; mm < M; ++mm)
                P->descs.push_back(make_desc(L.hr + (int64_t)mm * N, M * N, 1, L.br + (int64_t)mm * N, M * N, 1,
                                             L.dr + (int64_t)mm * pr * qr, N, p->k_row, J, V, p->use_w, L.wr, thr_rc));
            g.proto = P->descs[g.first];
            P->groups.push_back(g);
            g.first = (int)P->descs.size();
            g.count = N;
            for (int nn = 0; nn < N; ++nn)
                P->descs.push_back(make_desc(L.hct + (int64_t)nn * M, N * M, 1, L.bct + (int64_t)nn * M, N * M, 1,
                                             L.dc + (int64_t)nn * pc * qc, M, p->k_col, J, V, p->use_w, L.wc, thr_rc));
            g.proto = P->descs[g.first];
            P->groups.push_back(g);
        }
    } else {
        const SliceLayout& L = P->sl[0];
        const int M = L.M, N = L.N, Lh = p->L;
        const int pp = N - p->k_row + 1, qp = p->k_row * J * V;
        const int pe = Lh - p->k_col + 1, qe = p->k_col * J;
        const int64_t LJN = (int64_t)Lh * J * N;
        LRGroup g;
        g.first = (int)P->descs.size();
        g.count = M * Lh;
        for (int mm = 0; mm < M; ++mm)
            for (int l = 0; l < Lh; ++l) {
                const int64_t o = mm * LJN + (int64_t)l * J * N;
                P->descs.push_back(make_desc(L.k + o, N, 1, L.bp + o, N, 1,
                                             L.dp + ((int64_t)mm * Lh + l) * pp * qp, N, p->k_row, J, V, p->use_w,
                                             L.wr, thr_rc));
            }
        g.proto = P->descs[g.first];
        P->groups.push_back(g);
        g.first = (int)P->descs.size();
        g.count = M * N;
        for (int mm = 0; mm < M; ++mm)
            for (int nn = 0; nn < N; ++nn) {
                const int64_t o = mm * LJN + nn;
                P->descs.push_back(make_desc(L.xe + o, N, J * N, L.be + o, N, J * N,
                                             L.de + ((int64_t)mm * N + nn) * pe * qe, Lh, p->k_col, J, 1, 0, L.wr,
                                             p->lambda2 / p->beta));
            }
        g.proto = P->descs[g.first];
        P->groups.push_back(g);
    }
    for (auto& d : P->descs) P->s_max = std::max(P->s_max, lr_s(d));
    order_groups(P);
    layout_slots(P);
    // workspace
    size_t off = 0;
    P->off_c = off;
    P->bytes_c = (size_t)c * P->csize;
    off = align256(off + P->bytes_c);
    P->off_r = off;
    P->bytes_r = (size_t)std::max<int64_t>(r, (int64_t)P->rtab.size()) * P->rsize;
    off = align256(off + P->bytes_r);
    P->off_m = off;
    P->bytes_m = (size_t)m;
    off = align256(off + P->bytes_m);
    P->off_desc = off;
    off = align256(off + P->descs.size() * sizeof(LRDesc));
    P->off_g = off;
    off = align256(off + P->bytes_g);
    P->off_s = off;
    off = align256(off + P->bytes_s);
    P->off_scr = off;
    off = align256(off + P->bytes_scr);
    P->off_ranks = off;
    off = align256(off + P->descs.size() * 4);
    // scale (n_slices doubles), maxabs (n_slices u64), flags (u32, 64 bytes), then per stop unit: the change
    // pair (2 doubles), active flag and iteration count (int32 each), last relative change (double), and the
    // count of active units
    P->n_units = p->model == SHLR_MODEL_PI ? p->n_slices : P->Ms[0];
    P->off_scal = off;
    off = align256(off + scal_bytes(p->n_slices, P->n_units));
    P->off_spirit = off;
    P->bytes_spirit = spirit_bytes(P);
    off = align256(off + P->bytes_spirit);
    if (p->model == SHLR_MODEL_PI) {
        if (prec_c64(p->precision)) build_segments<float>(P);
        else build_segments<double>(P);
    }
    P->off_seg = off;
    off = align256(off + P->bytes_seg);
    P->total = off;
    P->scales.assign(p->n_slices, 1.0);
    *out = P;
    return SHLR_OK;
}

extern "C" void shlr_plan_destroy(shlr_plan* plan) {
    if (!plan) return;
    for (auto e : plan->ev_pool) (void)hipEventDestroy(e);
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

extern "C" shlr_status shlr_workspace_size(const shlr_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(SHLR_E_INVALID_ARG, "NULL argument");
    *bytes = plan->total;
    return SHLR_OK;
}

template <typename R>
static shlr_status upload_tables(shlr_plan* P) {
    using C = cplx_t<R>;
    std::vector<R> rt(P->rtab.begin(), P->rtab.end());
    if (!rt.empty())
        HIPCHK(hipMemcpyAsync(P->ws + P->off_r, rt.data(), rt.size() * sizeof(R), hipMemcpyHostToDevice, P->stream));
    std::vector<C> ct(P->ctab.size() / 2);
    for (size_t i = 0; i < ct.size(); ++i) {
        ct[i].x = (R)P->ctab[2 * i];
        ct[i].y = (R)P->ctab[2 * i + 1];
    }
    if (!ct.empty()) {
        const int64_t off = P->sl[0].wr;  // first complex-table entry
        HIPCHK(hipMemcpyAsync(P->ws + P->off_c + off * sizeof(C), ct.data(), ct.size() * sizeof(C),
                              hipMemcpyHostToDevice, P->stream));
    }
    HIPCHK(hipMemcpyAsync(P->ws + P->off_desc, P->descs.data(), P->descs.size() * sizeof(LRDesc),
                          hipMemcpyHostToDevice, P->stream));
    if (P->bytes_seg) {
        unsigned char* d = P->ws + P->off_seg;
        HIPCHK(hipMemcpyAsync(d, P->seg_fwd.data(), P->seg_fwd.size() * sizeof(FftSeg), hipMemcpyHostToDevice,
                              P->stream));
        d += align256(P->seg_fwd.size() * sizeof(FftSeg));
        HIPCHK(hipMemcpyAsync(d, P->seg_inv.data(), P->seg_inv.size() * sizeof(FftSeg), hipMemcpyHostToDevice,
                              P->stream));
        d += align256(P->seg_inv.size() * sizeof(FftSeg));
        HIPCHK(hipMemcpyAsync(d, P->seg_x.data(), P->seg_x.size() * sizeof(XupdSeg), hipMemcpyHostToDevice,
                              P->stream));
    }
    HIPCHK(hipStreamSynchronize(P->stream));   // host vectors go out of scope
    return SHLR_OK;
}

extern "C" shlr_status shlr_bind(shlr_plan* plan, void* ws_dev, size_t bytes, void* stream) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!ws_dev) return fail(SHLR_E_WORKSPACE, "workspace is NULL");
    if (bytes < plan->total) return fail(SHLR_E_WORKSPACE, "workspace has %zu bytes, %zu needed", bytes, plan->total);
    if (((uintptr_t)ws_dev) & 255) return fail(SHLR_E_WORKSPACE, "workspace must be 256-byte aligned");
    plan->ws = (unsigned char*)ws_dev;
    plan->stream = (hipStream_t)stream;
    plan->bound = true;
    plan->initialised = false;
    plan->spirit_ready = false;
    if (plan->graph_exec) {
        (void)hipGraphExecDestroy(plan->graph_exec);
        plan->graph_exec = nullptr;
    }
    if (prec_c64(plan->p.precision)) return upload_tables<float>(plan);
    return upload_tables<double>(plan);
}

extern "C" shlr_status shlr_set_weights(shlr_plan* plan, const void* w_row_dev, const void* w_col_dev) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->bound) return fail(SHLR_E_WORKSPACE, "no workspace bound");
    const shlr_params& p = plan->p;
    if (!p.use_w) return fail(SHLR_E_STATE, "the plan was created with use_w = 0 (no weighting W)");
    if (!w_row_dev) return fail(SHLR_E_INVALID_ARG, "w_row is NULL");
    const bool pi = p.model == SHLR_MODEL_PI;
    if (pi && !w_col_dev) return fail(SHLR_E_INVALID_ARG, "w_col is NULL");
    if (!pi && w_col_dev) return fail(SHLR_E_INVALID_ARG, "the parameter model has no column weights (w_col must be NULL)");
    size_t nr = 0, nc = 0;
    for (const SliceLayout& L : plan->sl) {
        nr += L.N;
        nc += pi ? L.M : 0;
    }
    std::vector<double> wrow(2 * nr), wcol(2 * nc);
    HIPCHK(hipMemcpyAsync(wrow.data(), w_row_dev, 16 * nr, hipMemcpyDeviceToHost, plan->stream));
    if (nc) HIPCHK(hipMemcpyAsync(wcol.data(), w_col_dev, 16 * nc, hipMemcpyDeviceToHost, plan->stream));
    HIPCHK(hipStreamSynchronize(plan->stream));
    for (double v : wrow)
        if (!isfinite(v)) return fail(SHLR_E_NONFINITE, "w_row holds NaN or Inf");
    for (double v : wcol)
        if (!isfinite(v)) return fail(SHLR_E_NONFINITE, "w_col holds NaN or Inf");
    const int64_t c0 = plan->sl[0].wr;   // complex-arena offset of the first complex-table entry
    auto put = [&](int64_t at, const std::vector<double>& re, const std::vector<double>& im) {
        for (size_t i = 0; i < re.size(); ++i) {
            plan->ctab[2 * (at - c0 + (int64_t)i)] = re[i];
            plan->ctab[2 * (at - c0 + (int64_t)i) + 1] = im[i];
        }
    };
    // one direction of one slice: weights, Gram diagonal (Eq. 15 denominator) and the D = d0 pattern
    auto line = [&](const double* w, int n, int k, int64_t w_at, int64_t r_at, int64_t v_at) {
        std::vector<double> re(n), im(n), vr, vi;
        for (int i = 0; i < n; ++i) {
            re[i] = w[2 * i];
            im[i] = w[2 * i + 1];
        }
        put(w_at, re, im);
        const std::vector<double> r = gram_diag_host(n, k, true, p.use_vc != 0, re, im);
        for (int i = 0; i < n; ++i) plan->rtab[r_at + i] = r[i];
        init_adjoint_host(n, k, true, p.use_vc != 0, -p.d0 / p.beta, re, im, vr, vi);
        put(v_at, vr, vi);
    };
    size_t orow = 0, ocol = 0;
    for (SliceLayout& L : plan->sl) {
        line(wrow.data() + 2 * orow, L.N, p.k_row, L.wr, L.rr, L.vr);
        orow += L.N;
        if (pi) {
            line(wcol.data() + 2 * ocol, L.M, p.k_col, L.wc, L.rc, L.vc);
            ocol += L.M;
        }
    }
    // the iterate (and a captured graph) were formed with the old tables
    plan->initialised = false;
    if (plan->graph_exec) {
        (void)hipGraphExecDestroy(plan->graph_exec);
        plan->graph_exec = nullptr;
    }
    if (prec_c64(p.precision)) return upload_tables<float>(plan);
    return upload_tables<double>(plan);
}

// ---------------------------------------------------------------------------
// iteration
// ---------------------------------------------------------------------------

template <typename R>
struct Ptrs {
    using C = cplx_t<R>;
    C* c;
    R* r;
    uint8_t* m;
    LRDesc* desc;
    double2* g;
    C* s;
    double* scr;
    int32_t* ranks;
    double* scale;
    unsigned long long* maxabs;
    uint32_t* flags;
    double* change;     // [n_units][2]: sum |K - K_prev|^2, sum |K_prev|^2
    int32_t* active;    // [n_units]
    int32_t* iters;     // [n_units]
    double* rel;        // [n_units]
    int32_t* n_active;
    explicit Ptrs(const shlr_plan* P) {
        c = (C*)(P->ws + P->off_c);
        r = (R*)(P->ws + P->off_r);
        m = P->ws + P->off_m;
        desc = (LRDesc*)(P->ws + P->off_desc);
        g = (double2*)(P->ws + P->off_g);
        s = (C*)(P->ws + P->off_s);
        scr = (double*)(P->ws + P->off_scr);
        ranks = (int32_t*)(P->ws + P->off_ranks);
        unsigned char* sc = P->ws + P->off_scal;
        const int S = P->p.n_slices;
        const int U = P->n_units;
        scale = (double*)sc;
        maxabs = (unsigned long long*)(sc + 8 * S);
        flags = (uint32_t*)(sc + 16 * S);
        change = (double*)(sc + 16 * S + 64);
        active = (int32_t*)(change + 2 * U);
        iters = active + U;
        rel = (double*)(iters + U);
        n_active = (int32_t*)(rel + U);
    }
};

template <typename R>
static shlr_status spirit_xupdate(shlr_plan* P, int si, bool track_change);

static double ortol_for(const shlr_plan* P) { return prec_c64(P->p.precision) ? 1e-5 : 1e-3; }

template <typename R>
static shlr_status run_lowrank(shlr_plan* P, cplx_t<R>* hb, cplx_t<R>* db, cplx_t<R>* bb, const cplx_t<R>* wtab,
                               LRDesc* desc_dev, double2* G, cplx_t<R>* S, double* scr, int32_t* ranks,
                               uint32_t* flags) {
    // Per run, chunks of up to `slots` matrices: the Gram products of every
    // group segment in the chunk, then one eigen-solver launch over the whole
    // chunk, then the reprojections.
    const double ortol = ortol_for(P);
    std::vector<LRDesc> protos;
    for (const LRRun& run : P->runs) {
        for (int c0 = run.first; c0 < run.first + run.count; c0 += run.slots) {
            const int c1 = std::min(run.first + run.count, c0 + run.slots);
            // the shapes of the groups in the chunk; a launch parameter the autotuner chose is kept
            // where every group of the chunk agrees on it
            protos.clear();
            int gkc = -1, rkc = -1;
            for (int gi = run.g0; gi < run.g1; ++gi) {
                const LRGroup& g = P->groups[gi];
                if (std::max(c0, g.first) >= std::min(c1, g.first + g.count)) continue;
                protos.push_back(g.proto);
                gkc = gkc == -1 || gkc == g.gram_kc ? g.gram_kc : 0;
                rkc = rkc == -1 || rkc == g.reproj_kc ? g.reproj_kc : 0;
            }
            const int np = (int)protos.size();
            size_t e0 = 0;
            STCHK(phase_begin(P, 1, &e0));
            HIPCHK(launch_lift_gram_multi<R>(P->stream, hb, db, wtab, desc_dev, protos.data(), np, c0, c1 - c0, G,
                                             run.g_stride, P->p.beta, gkc));
            STCHK(phase_end(P, 1, e0));
            const bool r32 = prec_r32(P->p.precision);
            const int rr = run_uses_rr(run, r32);
            if (rr) {
                STCHK(phase_begin(P, 5, &e0));
                HIPCHK(launch_tridiag_rr(P->stream, desc_dev, c0, c1 - c0, G, run.g_stride, scr, run.scr_stride,
                                         run.smax, r32));
                STCHK(phase_end(P, 5, e0));
            }
            STCHK(phase_begin(P, 2, &e0));
            HIPCHK(launch_heig_svt<cplx_t<R>>(P->stream, desc_dev, c0, c1 - c0, G, run.g_stride, S, run.s_stride, scr,
                                              run.scr_stride, ranks, ortol, flags, run.smax, VjpArgs<cplx_t<R>>(),
                                              rr, P->eig_resid_lim));
            STCHK(phase_end(P, 2, e0));
            STCHK(phase_begin(P, 3, &e0));
            HIPCHK(launch_reproj_multi<R>(P->stream, hb, db, bb, wtab, desc_dev, protos.data(), np, c0, c1 - c0, S,
                                          run.s_stride, P->p.beta, P->p.tau, rkc));
            STCHK(phase_end(P, 3, e0));
        }
    }
    return SHLR_OK;
}

template <typename R>
static shlr_status x_update_phase(shlr_plan* P, bool track_change) {
    Ptrs<R> Q(P);
    const shlr_params& p = P->p;
    const int J = p.J;
    if (track_change) HIPCHK(launch_zero_doubles(P->stream, Q.change, 2 * P->n_units));
    size_t e0 = 0;
    STCHK(phase_begin(P, 0, &e0));
    if (p.model == SHLR_MODEL_PI) {
        // every slice in one launch per step: A = F_m(B_row), the X-update of Eq. 15 (or SPIRiT's
        // PCG per slice), H_row = F_m^-1(K)
        const FftSeg* sf = (const FftSeg*)(P->ws + P->off_seg);
        const FftSeg* sv = (const FftSeg*)((const unsigned char*)sf + align256(P->seg_fwd.size() * sizeof(FftSeg)));
        const XupdSeg* sx =
            (const XupdSeg*)((const unsigned char*)sv + align256(P->seg_inv.size() * sizeof(FftSeg)));
        const int ns = (int)P->seg_fwd.size();
        HIPCHK(launch_fft_lines_seg<R>(P->stream, Q.c, Q.c, sf, ns, P->blk_fwd, P->lds_fwd));
        if (p.spirit_ksize > 0 && p.lambda1 > 0) {
            for (int si = 0; si < p.n_slices; ++si) STCHK(spirit_xupdate<R>(P, si, track_change));
        } else {
            HIPCHK(launch_xupd_rows_seg<R>(P->stream, Q.c, Q.m, Q.r, sx, ns, P->blk_x, P->lds_x, p.lambda, p.beta,
                                           p.hard_dc, track_change ? Q.change : nullptr,
                                           track_change ? Q.active : nullptr));
        }
        HIPCHK(launch_fft_lines_seg<R>(P->stream, Q.c, Q.c, sv, ns, P->blk_inv, P->lds_inv));
    } else {
        const SliceLayout& L = P->sl[0];
        const int M = L.M, N = L.N, Lh = p.L;
        XupdRows x;
        x.n = N;
        x.n1 = Lh;
        x.n0 = J;
        x.n_rows = M * Lh * J;
        x.rc_digit = 1;
        x.bo = RowAddr{(int64_t)Lh * J * N, (int64_t)J * N, N, 1};
        x.a = x.bo;
        x.y = x.bo;
        x.k = x.bo;
        x.out = x.bo;
        x.msk = RowAddr{0, N, 0, 1};
        x.rr_off = L.rr;
        x.rc_off = L.rc;
        x.unit_digit = 2;   // one stop unit per FE position (Algorithm S2)
        HIPCHK(launch_xupd_rows<R>(P->stream, Q.c + L.be, Q.c + L.bp, Q.c + L.yn, Q.c + L.k, Q.c + L.xe,
                                   Q.m + L.mask_b, Q.r, x, p.lambda, p.beta, p.hard_dc,
                                   track_change ? Q.change : nullptr, track_change ? Q.active : nullptr));
    }
    STCHK(phase_end(P, 0, e0));
    return SHLR_OK;
}

template <typename R>
static shlr_status lowrank_phase(shlr_plan* P) {
    Ptrs<R> Q(P);
    return run_lowrank<R>(P, Q.c, Q.c, Q.c, Q.c, Q.desc, Q.g, Q.s, Q.scr, Q.ranks, Q.flags);
}

// One iteration of Algorithm S1 / S2: X-update, then the Z and multiplier updates.  With the
// relative-change stop on, the X-update of a unit (slice or FE position) that has stopped keeps its
// K, and the stop test after the multiplier updates retires the units whose change fell below tol.
template <typename R>
static shlr_status iterate_once(shlr_plan* P, bool track_change) {
    STCHK(x_update_phase<R>(P, track_change));
    STCHK(lowrank_phase<R>(P));
    if (track_change) {
        Ptrs<R> Q(P);
        HIPCHK(launch_stop_test(P->stream, Q.change, Q.active, Q.iters, Q.rel, P->n_units, P->p.tol, Q.n_active));
    }
    return SHLR_OK;
}

template <typename R>
static shlr_status init_impl(shlr_plan* P, const void* y_dev, const uint8_t* mask_dev) {
    using C = cplx_t<R>;
    Ptrs<R> Q(P);
    const shlr_params& p = P->p;
    const int J = p.J;
    const C* Y = (const C*)y_dev;
    HIPCHK(hipMemsetAsync(P->ws + P->off_scal, 0, scal_bytes(p.n_slices, P->n_units), P->stream));
    {
        // every unit starts active (Algorithm S1 / S2 iterate until their own stop test)
        std::vector<int32_t> ones(P->n_units, 1);
        HIPCHK(hipMemcpyAsync(Q.active, ones.data(), ones.size() * 4, hipMemcpyHostToDevice, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
    }
    if (p.model == SHLR_MODEL_PI) {
        int64_t yoff = 0, moff = 0;
        for (int si = 0; si < p.n_slices; ++si) {
            const SliceLayout& L = P->sl[si];
            const int64_t e = (int64_t)J * L.M * L.N;
            HIPCHK(launch_maxabs<R>(P->stream, Y + yoff, e, Q.maxabs + si, Q.flags));
            yoff += e;
            moff += (int64_t)L.M * L.N;
        }
        std::vector<unsigned long long> mx(p.n_slices);
        HIPCHK(hipMemcpyAsync(mx.data(), Q.maxabs, mx.size() * 8, hipMemcpyDeviceToHost, P->stream));
        uint32_t fl = 0;
        HIPCHK(hipMemcpyAsync(&fl, Q.flags, 4, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
        if (fl & 1u) return fail(SHLR_E_NONFINITE, "Y holds NaN or Inf");
        for (int si = 0; si < p.n_slices; ++si) {
            double v;
            memcpy(&v, &mx[si], 8);
            P->scales[si] = (p.normalize && v > 0) ? v : 1.0;
        }
        HIPCHK(hipMemcpyAsync(Q.scale, P->scales.data(), 8 * p.n_slices, hipMemcpyHostToDevice, P->stream));
        yoff = 0;
        moff = 0;
        for (int si = 0; si < p.n_slices; ++si) {
            const SliceLayout& L = P->sl[si];
            const int M = L.M, N = L.N;
            const int64_t e = (int64_t)J * M * N;
            HIPCHK(launch_scale_copy<R>(P->stream, Y + yoff, Q.c + L.yn, e, Q.scale + si, 1));
            HIPCHK(hipMemcpyAsync(Q.c + L.k, Q.c + L.yn, e * sizeof(C), hipMemcpyDeviceToDevice, P->stream));
            HIPCHK(hipMemcpyAsync(Q.m + L.mask_b, mask_dev + moff, (size_t)M * N, hipMemcpyDeviceToDevice, P->stream));
            const int V = p.use_vc ? 2 : 1;
            const int64_t dr = (int64_t)M * (N - p.k_row + 1) * p.k_row * J * V;
            const int64_t dc = (int64_t)N * (M - p.k_col + 1) * p.k_col * J * V;
            HIPCHK(launch_fill_const<R>(P->stream, Q.c + L.dr, dr, p.d0, 0.0));
            HIPCHK(launch_fill_const<R>(P->stream, Q.c + L.dc, dc, p.d0, 0.0));
            HIPCHK(launch_fill_pattern<R>(P->stream, Q.c + L.br, e, Q.c + L.vr, 1, N));
            HIPCHK(launch_fill_pattern<R>(P->stream, Q.c + L.bct, e, Q.c + L.vc, 1, M));
            // Eq. 15 is singular where both lifted terms vanish (W is zero there: the k-space centre for the
            // first-difference weights) unless the point is sampled
            std::vector<int> zn, zm;
            for (int i = 0; i < N; ++i)
                if (!(P->rtab[L.rr + i] > 0)) zn.push_back(i);
            for (int i = 0; i < M; ++i)
                if (!(P->rtab[L.rc + i] > 0)) zm.push_back(i);
            if (!zn.empty() && !zm.empty()) {
                std::vector<uint8_t> mh((size_t)M * N);
                HIPCHK(hipMemcpyAsync(mh.data(), mask_dev + moff, mh.size(), hipMemcpyDeviceToHost, P->stream));
                HIPCHK(hipStreamSynchronize(P->stream));
                for (int a : zm)
                    for (int b : zn)
                        if (!mh[(size_t)a * N + b])
                            return fail(SHLR_E_SINGULAR, "slice %d: k-space point (%d, %d) is not sampled and the lifted "
                                        "terms vanish there", si, a, b);
            }
            yoff += e;
            moff += (int64_t)M * N;
        }
    } else {
        const SliceLayout& L = P->sl[0];
        const int M = L.M, N = L.N, Lh = p.L;
        const int64_t e = (int64_t)Lh * J * M * N;
        HIPCHK(launch_maxabs<R>(P->stream, Y, e, Q.maxabs, Q.flags));
        unsigned long long mx = 0;
        uint32_t fl = 0;
        HIPCHK(hipMemcpyAsync(&mx, Q.maxabs, 8, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipMemcpyAsync(&fl, Q.flags, 4, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
        if (fl & 1u) return fail(SHLR_E_NONFINITE, "Y holds NaN or Inf");
        double v;
        memcpy(&v, &mx, 8);
        P->scales[0] = (p.normalize && v > 0) ? v : 1.0;
        HIPCHK(hipMemcpyAsync(Q.scale, P->scales.data(), 8, hipMemcpyHostToDevice, P->stream));
        // inverse DFT along FE, into [M][L][J][N], normalised
        LineAddr ia{0, (int64_t)M * N, 1, N, N};
        LineAddr oa{0, N, 1, N, (int32_t)((int64_t)Lh * J * N)};
        HIPCHK(launch_fft_lines<R>(P->stream, Y, Q.c + L.yn, ia, oa, M, Lh * J * N, 1,
                                   1.0 / (sqrt((double)M) * P->scales[0])));
        HIPCHK(hipMemcpyAsync(Q.c + L.k, Q.c + L.yn, e * sizeof(C), hipMemcpyDeviceToDevice, P->stream));
        HIPCHK(hipMemcpyAsync(Q.m + L.mask_b, mask_dev, (size_t)Lh * N, hipMemcpyDeviceToDevice, P->stream));
        const int V = p.use_vc ? 2 : 1;
        const int64_t dp = (int64_t)M * Lh * (N - p.k_row + 1) * p.k_row * J * V;
        const int64_t de = (int64_t)M * N * (Lh - p.k_col + 1) * p.k_col * J;
        HIPCHK(launch_fill_const<R>(P->stream, Q.c + L.dp, dp, p.d0, 0.0));
        HIPCHK(launch_fill_const<R>(P->stream, Q.c + L.de, de, p.d0, 0.0));
        HIPCHK(launch_fill_pattern<R>(P->stream, Q.c + L.bp, e, Q.c + L.vr, 1, N));
        HIPCHK(launch_fill_pattern<R>(P->stream, Q.c + L.be, e, Q.c + L.vc, (int64_t)J * N, Lh));
    }
    HIPCHK(hipStreamSynchronize(P->stream));
    P->initialised = true;
    P->iters_total = 0;
    return SHLR_OK;
}

extern "C" shlr_status shlr_init(shlr_plan* plan, const void* y_dev, const uint8_t* mask_dev) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->bound) return fail(SHLR_E_WORKSPACE, "no workspace bound");
    if (!y_dev || !mask_dev) return fail(SHLR_E_INVALID_ARG, "NULL data pointer");
    if (prec_c64(plan->p.precision)) return init_impl<float>(plan, y_dev, mask_dev);
    return init_impl<double>(plan, y_dev, mask_dev);
}

// Read the per-unit stop state back and fill info (synchronises the stream).
template <typename R>
static shlr_status fill_info(shlr_plan* P, bool track, const std::vector<int32_t>& iters_before, int ran,
                             shlr_info* info) {
    Ptrs<R> Q(P);
    const int U = P->n_units;
    uint32_t fl = 0;
    std::vector<int32_t> it(U), act(U);
    std::vector<double> rel(U);
    HIPCHK(hipMemcpyAsync(&fl, Q.flags, 4, hipMemcpyDeviceToHost, P->stream));
    if (track) {
        HIPCHK(hipMemcpyAsync(it.data(), Q.iters, 4 * U, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipMemcpyAsync(act.data(), Q.active, 4 * U, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipMemcpyAsync(rel.data(), Q.rel, 8 * U, hipMemcpyDeviceToHost, P->stream));
    }
    HIPCHK(hipStreamSynchronize(P->stream));
    info->iters_done = ran;
    info->converged = 0;
    info->rel_change = 0;
    if (track) {
        int most = 0, still = 0;
        double worst = 0;
        for (int u = 0; u < U; ++u) {
            most = std::max(most, it[u] - (iters_before.empty() ? 0 : iters_before[u]));
            still += act[u] != 0;
            worst = std::max(worst, rel[u]);
        }
        info->iters_done = most;
        info->converged = still == 0;
        info->rel_change = worst;
    }
    info->scale = P->scales[0];
    info->device_flags = fl;
    if (fl & 1u) return fail(SHLR_E_NONFINITE, "a non-finite value was met during the iterations");
    if (fl & 2u)
        return fail(SHLR_E_EIG_NOCONV, "an eigenpair of a lifted matrix's Gram matrix missed the residual check "
                    "(||T z - l z|| > %g ||T|| ||z||)", P->eig_resid_lim);
    return SHLR_OK;
}

extern "C" shlr_status shlr_set_eig_check(shlr_plan* plan, double rel_residual_limit) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!(rel_residual_limit >= 0) || !isfinite(rel_residual_limit))
        return fail(SHLR_E_INVALID_ARG, "the residual limit must be finite and >= 0");
    plan->eig_resid_lim = rel_residual_limit;
    if (plan->graph_exec) {   // the captured graph holds the old limit
        (void)hipGraphExecDestroy(plan->graph_exec);
        plan->graph_exec = nullptr;
    }
    return SHLR_OK;
}

template <typename R>
static shlr_status iterate_impl(shlr_plan* P, int n, shlr_info* info) {
    Ptrs<R> Q(P);
    const bool track = P->p.tol > 0;
    std::vector<int32_t> before;
    if (track && info) {
        before.resize(P->n_units);
        HIPCHK(hipMemcpyAsync(before.data(), Q.iters, 4 * before.size(), hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
    }
    // The stop decision stays on the device (units that stopped keep their K); the host looks at the
    // count of active units only every STOP_POLL iterations, to end the loop once all have stopped.
    constexpr int STOP_POLL = 8;
    int done = 0;
    for (int it = 0; it < n; ++it) {
        STCHK(iterate_once<R>(P, track));
        ++done;
        if (track && (done % STOP_POLL == 0) && done < n) {
            int32_t na = 1;
            HIPCHK(hipMemcpyAsync(&na, Q.n_active, 4, hipMemcpyDeviceToHost, P->stream));
            HIPCHK(hipStreamSynchronize(P->stream));
            if (na == 0) break;
        }
    }
    P->iters_total += done;
    if (info) STCHK(fill_info<R>(P, track, before, done, info));
    return SHLR_OK;
}

extern "C" shlr_status shlr_timing_enable_phases(shlr_plan* plan, uint32_t phase_mask) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (phase_mask >> SHLR_TIMING_PHASES) return fail(SHLR_E_INVALID_ARG, "phase mask has bits above phase %d",
                                                       SHLR_TIMING_PHASES - 1);
    STCHK(timing_collect(plan));
    plan->timing = phase_mask != 0;
    plan->timing_mask = phase_mask;
    for (int i = 0; i < 8; ++i) {
        plan->t_ms[i] = 0;
        plan->t_cnt[i] = 0;
    }
    return SHLR_OK;
}

extern "C" shlr_status shlr_timing_enable(shlr_plan* plan, int32_t enable) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    STCHK(timing_collect(plan));
    plan->timing = enable != 0;
    plan->timing_mask = (1u << SHLR_TIMING_PHASES) - 1;
    for (int i = 0; i < 8; ++i) {
        plan->t_ms[i] = 0;
        plan->t_cnt[i] = 0;
    }
    return SHLR_OK;
}

extern "C" shlr_status shlr_timing_read(shlr_plan* plan, double* ms_out, int32_t* launches_out) {
    if (!plan || !ms_out || !launches_out) return fail(SHLR_E_INVALID_ARG, "NULL argument");
    STCHK(timing_collect(plan));
    for (int i = 0; i < SHLR_TIMING_PHASES; ++i) {
        ms_out[i] = plan->t_ms[i];
        launches_out[i] = plan->t_cnt[i];
    }
    return SHLR_OK;
}

extern "C" shlr_status shlr_iterate(shlr_plan* plan, int32_t n, shlr_info* info) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->initialised) return fail(SHLR_E_STATE, "shlr_init must come first");
    if (n < 0) return fail(SHLR_E_INVALID_ARG, "n must be >= 0");
    if (plan->p.spirit_ksize > 0 && plan->p.lambda1 > 0 && !plan->spirit_ready)
        return fail(SHLR_E_STATE, "the SPIRiT kernel is not set (shlr_set_spirit_kernel / shlr_calibrate_spirit)");
    if (prec_c64(plan->p.precision)) return iterate_impl<float>(plan, n, info);
    return iterate_impl<double>(plan, n, info);
}

template <typename R>
static shlr_status build_graph(shlr_plan* P) {
    if (!P->cap_stream) HIPCHK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    hipStream_t user = P->stream;
    P->stream = P->cap_stream;
    hipGraph_t graph = nullptr;
    // no timing events go into the graph: captured events cannot be read back as phase times
    const bool timing = P->timing;
    P->timing = false;
    hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        P->stream = user;
        P->timing = timing;
        return fail(SHLR_E_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    shlr_status st = iterate_once<R>(P, P->p.tol > 0);
    e = hipStreamEndCapture(P->cap_stream, &graph);
    P->stream = user;
    P->timing = timing;
    if (st != SHLR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(SHLR_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&P->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        P->graph_exec = nullptr;
        return fail(SHLR_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return SHLR_OK;
}

extern "C" shlr_status shlr_iterate_graph(shlr_plan* plan, int32_t n, shlr_info* info) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->initialised) return fail(SHLR_E_STATE, "shlr_init must come first");
    if (n < 0) return fail(SHLR_E_INVALID_ARG, "n must be >= 0");
    if (plan->p.spirit_ksize > 0 && plan->p.lambda1 > 0 && !plan->spirit_ready)
        return fail(SHLR_E_STATE, "the SPIRiT kernel is not set");
    if (!plan->graph_exec) {
        if (prec_c64(plan->p.precision)) STCHK(build_graph<float>(plan));
        else STCHK(build_graph<double>(plan));
    }
    const bool track = plan->p.tol > 0;
    std::vector<int32_t> before;
    if (track && info) {
        before.resize(plan->n_units);
        const size_t off = plan->off_scal + 16 * (size_t)plan->p.n_slices + 64 + 16 * (size_t)plan->n_units +
                           4 * (size_t)plan->n_units;   // the iteration counts (layout of Ptrs)
        HIPCHK(hipMemcpyAsync(before.data(), plan->ws + off, 4 * before.size(), hipMemcpyDeviceToHost, plan->stream));
        HIPCHK(hipStreamSynchronize(plan->stream));
    }
    for (int i = 0; i < n; ++i) HIPCHK(hipGraphLaunch(plan->graph_exec, plan->stream));
    plan->iters_total += n;
    if (info) {
        if (prec_c64(plan->p.precision)) STCHK(fill_info<float>(plan, track, before, n, info));
        else STCHK(fill_info<double>(plan, track, before, n, info));
    }
    return SHLR_OK;
}

extern "C" shlr_status shlr_unit_status(const shlr_plan* plan, int32_t n_units, int32_t* iters_host,
                                        double* rel_host, int32_t* active_host) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->initialised) return fail(SHLR_E_STATE, "shlr_init must come first");
    if (n_units != plan->n_units)
        return fail(SHLR_E_INVALID_ARG, "the plan has %d stop units, %d given", plan->n_units, n_units);
    const size_t U = (size_t)plan->n_units;
    const unsigned char* base = plan->ws + plan->off_scal + 16 * (size_t)plan->p.n_slices + 64 + 16 * U;
    if (active_host) HIPCHK(hipMemcpyAsync(active_host, base, 4 * U, hipMemcpyDeviceToHost, plan->stream));
    if (iters_host) HIPCHK(hipMemcpyAsync(iters_host, base + 4 * U, 4 * U, hipMemcpyDeviceToHost, plan->stream));
    if (rel_host) HIPCHK(hipMemcpyAsync(rel_host, base + 8 * U, 8 * U, hipMemcpyDeviceToHost, plan->stream));
    HIPCHK(hipStreamSynchronize(plan->stream));
    return SHLR_OK;
}

template <typename R>
static shlr_status get_impl(const shlr_plan* P, void* out) {
    using C = cplx_t<R>;
    Ptrs<R> Q(P);
    const shlr_params& p = P->p;
    const int J = p.J;
    C* O = (C*)out;
    if (p.model == SHLR_MODEL_PI) {
        int64_t off = 0;
        for (int si = 0; si < p.n_slices; ++si) {
            const SliceLayout& L = P->sl[si];
            const int64_t e = (int64_t)J * L.M * L.N;
            HIPCHK(launch_scale_copy<R>(P->stream, Q.c + L.k, O + off, e, Q.scale + si, 0));
            off += e;
        }
    } else {
        const SliceLayout& L = P->sl[0];
        const int M = L.M, N = L.N, Lh = p.L;
        LineAddr ia{0, N, 1, N, (int32_t)((int64_t)Lh * J * N)};
        LineAddr oa{0, (int64_t)M * N, 1, N, N};
        HIPCHK(launch_fft_lines<R>(P->stream, Q.c + L.k, O, ia, oa, M, Lh * J * N, 0,
                                   P->scales[0] / sqrt((double)M)));
    }
    HIPCHK(hipStreamSynchronize(P->stream));
    return SHLR_OK;
}

extern "C" shlr_status shlr_get_kspace(const shlr_plan* plan, void* k_out_dev) {
    if (!plan) return fail(SHLR_E_INVALID_ARG, "plan is NULL");
    if (!plan->initialised) return fail(SHLR_E_STATE, "shlr_init must come first");
    if (!k_out_dev) return fail(SHLR_E_INVALID_ARG, "k_out is NULL");
    if (prec_c64(plan->p.precision)) return get_impl<float>(plan, k_out_dev);
    return get_impl<double>(plan, k_out_dev);
}

extern "C" shlr_status shlr_reconstruct(shlr_plan* plan, const void* y_dev, const uint8_t* mask_dev, void* k_out_dev,
                                        shlr_info* info) {
    STCHK(shlr_init(plan, y_dev, mask_dev));
    if (plan->p.spirit_ksize > 0 && plan->p.lambda1 > 0 && !plan->spirit_ready)
        return fail(SHLR_E_STATE, "the SPIRiT kernel is not set");
    STCHK(shlr_iterate(plan, plan->p.max_iter, info));
    return shlr_get_kspace(plan, k_out_dev);
}

// ---------------------------------------------------------------------------
// stage entry points
// ---------------------------------------------------------------------------

extern "C" shlr_status shlr_fft_lines(int32_t precision, int32_t n, int32_t n_lines, int32_t inverse,
                                      const void* in_dev, void* out_dev, void* stream) {
    if (!prec_valid(precision)) return fail(SHLR_E_INVALID_ARG, "bad precision");
    if (n < 1 || n > 4096) return fail(SHLR_E_INVALID_ARG, "n must be in [1, 4096]");
    if (n_lines < 0) return fail(SHLR_E_INVALID_ARG, "n_lines must be >= 0");
    if (n_lines == 0) return SHLR_OK;
    if (!in_dev || !out_dev) return fail(SHLR_E_INVALID_ARG, "NULL pointer");
    LineAddr a{0, n, 0, 1, 1};
    const double sc = 1.0 / sqrt((double)n);
    if (prec_c64(precision))
        HIPCHK(launch_fft_lines<float>((hipStream_t)stream, (const float2*)in_dev, (float2*)out_dev, a, a, n, n_lines,
                                       inverse, sc));
    else
        HIPCHK(launch_fft_lines<double>((hipStream_t)stream, (const double2*)in_dev, (double2*)out_dev, a, a, n,
                                        n_lines, inverse, sc));
    return SHLR_OK;
}

struct LRLayout {
    size_t off_desc, off_g, off_s, off_scr, off_w, off_flags, total;
    int slots, s;
    int64_t gst, sst, scst;
};

// cap > 0: the layout must fit cap bytes; the eigen-solver slots (chunk size) shrink to what is left
static shlr_status lr_layout(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k, int32_t use_vc,
                             LRLayout* L, size_t cap = 0) {
    if (!prec_valid(precision)) return fail(SHLR_E_INVALID_ARG, "bad precision");
    if (n_mat < 0 || J < 1 || n < 1 || k < 1 || k > n) return fail(SHLR_E_INVALID_ARG, "bad shape");
    LRDesc d = make_desc(0, 0, 0, 0, 0, 0, 0, n, k, J, use_vc ? 2 : 1, 0, 0, 0.0);
    const int s = lr_s(d);
    if (s > 320) return fail(SHLR_E_UNSUPPORTED, "min(p, q) > 320");
    if (lr_l(d) > 4096) return fail(SHLR_E_UNSUPPORTED, "max(p, q) > 4096");
    const int cs = prec_c64(precision) ? 8 : 16;
    if (!lowrank_lds_fits(cs, use_vc ? 2 : 1, J, n, k))
        return fail(SHLR_E_UNSUPPORTED, "the line table of a lifted matrix (V*J*n) exceeds the LDS staging");
    L->s = s;
    L->gst = packed_size(s);
    L->sst = (int64_t)s * s;
    L->scst = eig_scratch_doubles(s);
    const size_t per = L->gst * 16 + L->sst * cs + L->scst * 8 + 3 * 256;
    size_t budget = SLOT_BUDGET;
    if (cap > 0) {
        const size_t fixed = align256((size_t)std::max(n_mat, 1) * sizeof(LRDesc)) + align256((size_t)n * cs) + 256 +
                             3 * 256;
        if (fixed + per > cap)
            return fail(SHLR_E_WORKSPACE, "n_mat = %d lines of this shape need %zu bytes for one eigen-solver slot "
                        "and the line tables, beyond the %zu-byte fixed scratch", n_mat, fixed + per, cap);
        budget = std::min(budget, cap - fixed);
    }
    L->slots = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(n_mat, 1), budget / per));
    size_t off = 0;
    L->off_desc = off;
    off = align256(off + (size_t)std::max(n_mat, 1) * sizeof(LRDesc));
    L->off_g = off;
    off = align256(off + (size_t)L->slots * L->gst * 16);
    L->off_s = off;
    off = align256(off + (size_t)L->slots * L->sst * cs);
    L->off_scr = off;
    off = align256(off + (size_t)L->slots * L->scst * 8);
    L->off_w = off;
    off = align256(off + (size_t)n * cs);
    L->off_flags = off;
    off = align256(off + 256);
    L->total = off;
    return SHLR_OK;
}

extern "C" shlr_status shlr_lowrank_workspace_size(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k,
                                                   int32_t use_vc, size_t* bytes) {
    if (!bytes) return fail(SHLR_E_INVALID_ARG, "bytes is NULL");
    LRLayout L;
    STCHK(lr_layout(precision, n_mat, J, n, k, use_vc, &L));
    *bytes = L.total;
    return SHLR_OK;
}

template <typename R>
static shlr_status lowrank_impl(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k, int32_t use_vc, int32_t use_w,
                                double beta, double tau, double thr, const void* h_dev, void* d_dev, void* b_dev,
                                int32_t* ranks_dev, unsigned char* ws, const LRLayout& L, hipStream_t st) {
    using C = cplx_t<R>;
    const int V = use_vc ? 2 : 1;
    const int p = n - k + 1, q = k * J * V;
    std::vector<LRDesc> descs(n_mat);
    for (int i = 0; i < n_mat; ++i)
        descs[i] = make_desc((int64_t)i * J * n, n, 1, (int64_t)i * J * n, n, 1, (int64_t)i * p * q, n, k, J, V, use_w,
                             0, thr);
    std::vector<double> wr, wi;
    weights_host(n, wr, wi);
    std::vector<C> w(n);
    for (int i = 0; i < n; ++i) {
        w[i].x = (R)wr[i];
        w[i].y = (R)wi[i];
    }
    HIPCHK(hipMemcpyAsync(ws + L.off_desc, descs.data(), descs.size() * sizeof(LRDesc), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws + L.off_w, w.data(), w.size() * sizeof(C), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(ws + L.off_flags, 0, 4, st));
    LRGroup g;
    g.first = 0;
    g.count = n_mat;
    g.proto = descs[0];
    shlr_plan tmp;
    tmp.p.beta = beta;
    tmp.p.tau = tau;
    tmp.p.precision = precision;
    tmp.stream = st;
    tmp.groups = {g};
    LRRun run{};
    run.first = 0;
    run.count = n_mat;
    run.g0 = 0;
    run.g1 = 1;
    run.smax = L.s;
    run.slots = L.slots;
    run.g_stride = L.gst;
    run.s_stride = L.sst;
    run.scr_stride = L.scst;
    tmp.runs = {run};
    STCHK(run_lowrank<R>(&tmp, (C*)h_dev, (C*)d_dev, (C*)b_dev, (const C*)(ws + L.off_w), (LRDesc*)(ws + L.off_desc),
                         (double2*)(ws + L.off_g), (C*)(ws + L.off_s), (double*)(ws + L.off_scr), ranks_dev,
                         (uint32_t*)(ws + L.off_flags)));
    uint32_t fl = 0;
    HIPCHK(hipMemcpyAsync(&fl, ws + L.off_flags, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));   // host descriptor vectors go out of scope
    if (fl & 1u) return fail(SHLR_E_NONFINITE, "a non-finite value was met in a lifted matrix");
    if (fl & 2u) return fail(SHLR_E_EIG_NOCONV, "an eigenpair of a lifted matrix's Gram matrix missed the residual check");
    return SHLR_OK;
}

extern "C" shlr_status shlr_lowrank_lines(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k,
                                          int32_t use_vc, int32_t use_w, double beta, double tau, double thr,
                                          const void* h_dev, void* d_dev, void* b_dev, int32_t* ranks_dev,
                                          void* ws_dev, size_t ws_bytes, void* stream) {
    LRLayout L;
    STCHK(lr_layout(precision, n_mat, J, n, k, use_vc, &L));
    if (n_mat == 0) return SHLR_OK;
    if (!(beta > 0) || !(tau > 0) || !(thr >= 0)) return fail(SHLR_E_INVALID_ARG, "beta, tau > 0 and thr >= 0 required");
    if (!h_dev || !d_dev || !b_dev) return fail(SHLR_E_INVALID_ARG, "NULL data pointer");
    if (!ws_dev || ws_bytes < L.total) return fail(SHLR_E_WORKSPACE, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    if (((uintptr_t)ws_dev) & 255) return fail(SHLR_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (prec_c64(precision))
        return lowrank_impl<float>(precision, n_mat, J, n, k, use_vc, use_w, beta, tau, thr, h_dev, d_dev, b_dev, ranks_dev,
                                   (unsigned char*)ws_dev, L, (hipStream_t)stream);
    return lowrank_impl<double>(precision, n_mat, J, n, k, use_vc, use_w, beta, tau, thr, h_dev, d_dev, b_dev, ranks_dev,
                                (unsigned char*)ws_dev, L, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// shlr_lowrank_lines without a caller workspace: the eigen-solver slots, descriptors, weights and
// flags live in a fixed device array of this file (one copy per GPU, held until the process ends)
// ---------------------------------------------------------------------------

static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::vector<unsigned char*> g_scratch_ptr;   // per device: the address of that device's copy

// The device address of this device's scratch array, looked up once per device with it current.
static shlr_status scratch_ptr(unsigned char** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SHLR_E_DEVICE, "no device address for the fixed scratch array");
        g_scratch_ptr[dev] = (unsigned char*)p;
    }
    *out = g_scratch_ptr[dev];
    return SHLR_OK;
}

extern "C" shlr_status shlr_lowrank_lines_noalloc(int32_t precision, int32_t n_mat, int32_t J, int32_t n, int32_t k,
                                                  int32_t use_vc, int32_t use_w, double beta, double tau, double thr,
                                                  const void* h_dev, void* d_dev, void* b_dev, int32_t* ranks_dev,
                                                  void* stream) {
    LRLayout L;
    STCHK(lr_layout(precision, n_mat, J, n, k, use_vc, &L, NOALLOC_SCRATCH_BYTES));
    if (n_mat == 0) return SHLR_OK;
    if (!(beta > 0) || !(tau > 0) || !(thr >= 0)) return fail(SHLR_E_INVALID_ARG, "beta, tau > 0 and thr >= 0 required");
    if (!h_dev || !d_dev || !b_dev) return fail(SHLR_E_INVALID_ARG, "NULL data pointer");
    if (L.total > NOALLOC_SCRATCH_BYTES)
        return fail(SHLR_E_WORKSPACE, "the layout needs %zu bytes, beyond the %zu-byte fixed scratch", L.total,
                    NOALLOC_SCRATCH_BYTES);
    unsigned char* ws = nullptr;
    STCHK(scratch_ptr(&ws));
    if (prec_c64(precision))
        return lowrank_impl<float>(precision, n_mat, J, n, k, use_vc, use_w, beta, tau, thr, h_dev, d_dev, b_dev,
                                   ranks_dev, ws, L, (hipStream_t)stream);
    return lowrank_impl<double>(precision, n_mat, J, n, k, use_vc, use_w, beta, tau, thr, h_dev, d_dev, b_dev,
                                ranks_dev, ws, L, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// SPIRiT (Eq. 3): set / calibrate the kernel; X-update by PCG
// ---------------------------------------------------------------------------
#include "spirit_host.inc"
#include "unrolled.inc"
#include "autotune.inc"
#include "eval_host.inc"
