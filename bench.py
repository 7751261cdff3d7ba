#!/usr/bin/env python
"""SHLR throughput on one MI355X: iterations/s of the full ADMM iteration.

Workload (the 8-coil parallel-imaging configuration): 8 coils, 256 x 256
complex64 k-space of the seeded ellipse phantom with smooth quadratic phase
and Gaussian coil maps, 2D Poisson-disc mask at R = 4 with a fully sampled
24 x 24 centre, Hankel window 25 on rows and columns, SPIRiT 5 x 5 kernel
calibrated on the centre, 10 PCG steps per X-update, lambda = 1e4,
lambda1 = 10, beta = tau = 30.  One step = one ADMM iteration (X-update,
Z-updates of all 512 row/column lifts, multiplier updates).

Prints one JSON line with the throughput, the roofline of the dominant kernel
(timed live with HIP events on the plan's stream), the FP64 oracle timed on
the host as a CPU baseline, and the NMSE of the GPU iterate against the
oracle after the same iterations from the same inputs.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SHLR iterations/sec (256² k-space × coils) at NMSE≤1e-5 vs FP64 oracle; % roofline"

PEAK_TFLOPS_FP32_MFMA = 157.3
PEAK_TFLOPS_FP32_VECTOR = 157.3   # published figure (it counts packed FP32 issue)
PEAK_TFLOPS_FP64 = 78.6
PEAK_HBM_GBS = 8000.0


def workload(J=8, M=256, N=256, seed=0):
    import numpy as np
    from paper_2107_11650_amd import inputs
    k = inputs.phantom_kspace(J, M, N, seed=1000 + seed)
    mask = inputs.mask_poisson_disc(M, N, R=4.0, acs=24, seed=2000 + seed)
    return inputs.undersample(k, mask), mask.astype(np.uint8)


def lowrank_work(shapes):
    """Algorithmic work of one iteration's lifted matrices [(p, q, count)] (Gram, eigen, reprojection)."""
    w = {"gram": 0.0, "eig": 0.0, "reproj": 0.0, "tridiag": 0.0}
    for p, q, c in shapes:
        s, l = min(p, q), max(p, q)
        w["gram"] += c * 4.0 * l * s * s      # Hermitian product: complex MAC = 8 flops, half the tiles
        w["reproj"] += c * 8.0 * l * s * s    # full product A S
        w["eig"] += c * 13.3 * s ** 3         # tridiagonalisation + back-transform bookkeeping
        w["tridiag"] += c * 16.0 / 3.0 * s ** 3   # Householder reduction of a complex Hermitian matrix
    return w


def build_workload(name, prec, n_cg, tune=True):
    """(plan, Y, mask, shapes, coil-k-space elements, config dict) of a named workload."""
    import numpy as np
    import torch
    from paper_2107_11650_amd import inputs, shlr
    kw = 25
    if name == "pi256":
        J, M, N = 8, 256, 256
        Y, mask = workload(J, M, N)
        p = shlr.Params(M=(M,), N=(N,), J=J, k_row=kw, k_col=kw, lam=1e4, lambda1=10.0, beta=30.0, tau=30.0,
                        spirit_ksize=5, n_cg=n_cg, precision=prec, max_iter=100)
        shapes = [(N - kw + 1, kw * J, M), (M - kw + 1, kw * J, N)]
        cfg = {"workload": "SHLR-S iteration, 8 coils, 256x256 complex64 ellipse phantom (quadratic phase, Gaussian "
                           "coils), 2D Poisson-disc R=4 + 24x24 centre, Hankel window 25 rows/cols (512 lifts of "
                           "232x200), SPIRiT 5x5, 10 PCG steps, lambda=1e4, lambda1=10, beta=tau=30",
               "coils": J, "M": M, "N": N, "window": kw, "spirit_kernel": 5, "n_cg": n_cg}
        elems = J * M * N
    elif name == "ragged":
        J = 12
        sizes = inputs.ragged_sizes(32, 192, 320, seed=3000)
        ys, ms = [], []
        for i, (M, N, R) in enumerate(sizes):
            k = inputs.phantom_kspace(J, M, N, seed=1000 + i)
            m = inputs.mask_poisson_disc(M, N, R=R, acs=24, seed=2000 + i)
            ys.append(inputs.undersample(k, m).ravel())
            ms.append(m.astype(np.uint8).ravel())
        Y, mask = np.concatenate(ys), np.concatenate(ms)
        p = shlr.Params(M=tuple(s[0] for s in sizes), N=tuple(s[1] for s in sizes), J=J, k_row=kw, k_col=kw,
                        lam=1e4, beta=30.0, tau=30.0, precision=prec, max_iter=100)
        shapes = []
        for M, N, _ in sizes:
            shapes += [(N - kw + 1, kw * J, M), (M - kw + 1, kw * J, N)]
        cfg = {"workload": "SHLR iteration over a ragged batch: 32 slices, sides U{192..320} (seed 3000), 12 coils, "
                           "complex64, Poisson-disc R in {4,5,6} + 24x24 centre, window 25, lambda=1e4, beta=tau=30",
               "slices": 32, "coils": J, "window": kw}
        elems = int(Y.size)
    elif name == "t2":
        L, J, M, N = 8, 12, 256, 256
        k = inputs.t2_kspace(J, M, N, L=L, seed=1004)
        m2 = inputs.mask_t2_cartesian(L, N, R=6, n_center=16)
        Y = inputs.undersample(k, m2[:, None, None, :])
        mask = m2.astype(np.uint8)
        p = shlr.Params(model=shlr.MODEL_PARAM, precision=prec, M=(M,), N=(N,), J=J, L=L, k_row=kw, k_col=4,
                        use_vc=True, lam=1e4, lambda2=2.0, beta=30.0, tau=30.0, max_iter=100)
        shapes = [(N - kw + 1, kw * J * 2, M * L), (L - 4 + 1, 4 * J, M * N)]
        cfg = {"workload": "SHLR-VP iteration, T2 series: 8 echoes (TE 10..80 ms, T2 U[30,150] ms per ellipse), "
                           "12 coils, 256x256 complex64, per-echo shifted R=6 Cartesian + 16 centre lines, PE window 25 "
                           "with virtual coils (2048 lifts of 232x600), echo window 4 (65536 lifts of 5x48), "
                           "lambda=1e4, lambda2=2, beta=tau=30",
               "echoes": L, "coils": J, "M": M, "N": N}
        elems = L * J * M * N
    else:
        raise SystemExit(f"unknown workload {name}")
    plan = shlr.Plan(p)
    if tune:
        cfg["autotune"] = plan.autotune(reps=3).strip().split("\n")
    plan.init(torch.from_numpy(Y).to(plan.cdtype).cuda(), torch.from_numpy(mask).cuda())
    if name == "pi256":
        plan.calibrate_spirit(acs=24, reg=1e-3)
    return plan, Y, mask, shapes, elems, cfg


def measured_traffic(phase, prec_name):
    """HBM bytes per launch of a phase's kernel from the committed rocprofv3 counter runs of this
    precision form, or None when there are none or the kernel's sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_8coil_256_k25_{prec_name.replace('-', '_')}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("precision") != prec_name:
        return None
    rec = d["phases"].get(phase)
    if rec is None:
        return None
    for name, digest in rec["sources"].items():
        with open(os.path.join(ROOT, "paper_2107_11650_amd", "csrc", name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec["bytes_per_launch"]


def diff_leg(batch, steps, kw, lam, beta, reps=2):
    """Reverse mode through `steps` unrolled iterations of a batch of 8-coil 256 x 256 slices."""
    import numpy as np
    import torch
    from paper_2107_11650_amd import inputs, shlr
    J, M, N = 8, 256, 256
    mask = inputs.mask_poisson_disc(M, N, R=4.0, acs=24, seed=2000).astype(np.uint8)
    ys = []
    for b in range(batch):
        k = inputs.phantom_kspace(J, M, N, seed=1000 + b)
        y = inputs.undersample(k, mask.astype(bool))
        ys.append(y / np.abs(y).max())
    p = shlr.Params(M=(M,) * batch, N=(N,) * batch, J=J, k_row=kw, k_col=kw, lam=lam, beta=beta, tau=beta,
                    normalize=False, precision=shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    y = torch.from_numpy(np.concatenate([v.ravel() for v in ys])).to(torch.complex64).cuda()
    m = torch.from_numpy(np.tile(mask.ravel(), batch)).cuda()
    gk = torch.from_numpy(inputs.random_complex(y.shape, seed=77)).to(torch.complex64).cuda()
    tf, tb = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.unrolled_forward(y, m, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.unrolled_backward(gk, steps)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tb.append(t2 - t1)
    ck, wk = plan.unrolled_sizes(steps)
    plan.close()
    fwd, bwd = min(tf), min(tb)
    # accuracy of the timed (mixed) reverse mode on the first slice: the directional derivative
    # <gY, d> against a central difference of L = Re <gk, K_steps> from two FP64 forwards
    y1 = torch.from_numpy(ys[0].ravel()).to(torch.complex128).cuda()
    m1 = torch.from_numpy(mask.ravel()).cuda()
    g1 = gk[:y1.numel()].to(torch.complex128)
    rng = np.random.default_rng(78)
    d = torch.from_numpy(rng.standard_normal(y1.shape) + 1j * rng.standard_normal(y1.shape)).cuda()
    one = dict(M=(M,), N=(N,), J=J, k_row=kw, k_col=kw, lam=lam, beta=beta, tau=beta, normalize=False)

    def loss(yv):
        pl = shlr.Plan(shlr.Params(precision=shlr.PREC_FP64, **one))
        kv = pl.unrolled_forward(yv, m1, steps)
        pl.close()
        return float((torch.conj(g1) * kv.to(torch.complex128)).real.sum().item())

    eps = 1e-6 * float(torch.linalg.vector_norm(y1)) / float(torch.linalg.vector_norm(d))
    fd = (loss(y1 + eps * d) - loss(y1 - eps * d)) / (2 * eps)
    pl = shlr.Plan(shlr.Params(precision=shlr.PREC_MIXED, **one))
    pl.unrolled_forward(y1.to(torch.complex64), m1, steps)
    gy, _ = pl.unrolled_backward(g1.to(torch.complex64), steps)
    pl.close()
    an = float(torch.sum((torch.conj(gy.to(torch.complex128)) * d).real).item())
    return {
        "accuracy": {"what": "first slice: directional derivative <gY, d> of the mixed-precision reverse mode against "
                             "a central difference of two FP64 forwards (step 1e-6 of |Y|, seeded direction)",
                     "vjp": an, "central_difference": fd, "rel_error": abs(an - fd) / abs(fd)},
        "workload": f"reverse mode through {steps} unrolled SHLR iterations, batch {batch} x 8 coils x 256x256 "
                    "complex64 (seeds 1000+b, shared 2D Poisson-disc R=4 mask), window 25, lambda=1e4, beta=tau=30; "
                    "gradient w.r.t. Y and lambda; checkpoints K and D of every iteration",
        "forward_ms": 1e3 * fwd, "backward_ms": 1e3 * bwd,
        "forward_ms_per_step": 1e3 * fwd / steps, "backward_ms_per_step": 1e3 * bwd / steps,
        "backward_over_forward": bwd / fwd,
        "unrolled_steps_per_s": steps / (fwd + bwd),
        "checkpoint_gb": ck / 1e9, "work_gb": wk / 1e9, "reps": reps, "timing": "best of reps, wall clock with syncs",
    }


def quality_leg(t2_iters=30):
    """Synthetic analogues of the paper's comparisons, scored on the GPU (SSOS, RLNE, MSSIM, T2 fit):
    SHLR / -S / -V / -SV at Gaussian Cartesian 0.34 with 22 ACS lines (as in Fig. 4), SHLR-SV over
    8..22 ACS lines at the same rate (Fig. 11), SHLR-SV under the other patterns (Figs. 7, 9, S1,
    S2), and SHLR-P / SHLR-VP T2 maps at R = 6 (Figs. 6, 10) against the map of the fully sampled
    series.  Every PI run uses the paper's Algorithm S1 settings (cap 50, tolerance 1e-6)."""
    import numpy as np
    import torch
    from paper_2107_11650_amd import inputs as I, shlr
    J, M, N = 8, 256, 256
    k = I.phantom_kspace(J, M, N, seed=1000)
    kd = torch.from_numpy(k).to(torch.complex64).cuda()
    truth = shlr.ssos(kd)
    kw = 25

    def run(mask, vc, spirit, acs):
        Y = I.undersample(k, mask)
        p = shlr.Params.paper_defaults(shlr.MODEL_PI, M=(M,), N=(N,), J=J, k_row=kw, k_col=kw, use_vc=vc,
                                       lam=1e4, lambda1=10.0 if spirit else 0.0, beta=30.0, tau=30.0,
                                       spirit_ksize=5 if spirit else 0, n_cg=10)
        plan = shlr.Plan(p)
        plan.init(torch.from_numpy(Y).to(torch.complex64).cuda(), torch.from_numpy(mask.astype(np.uint8)).cuda())
        if spirit:
            plan.calibrate_spirit(acs=acs, reg=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.iterate(p.max_iter)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        img = shlr.ssos(plan.kspace())
        plan.close()
        return {"rlne": shlr.rlne(truth, img), "mssim": shlr.mssim(truth, img), "iterations": info.iters_done,
                "it_per_s": info.iters_done / (t1 - t0), "rate": round(I.sampling_rate(mask), 4)}

    out = {"workload": "8-coil 256x256 phantom (seed 1000), window 25, lambda 1e4, lambda1 10, beta = tau = 30, "
                       "cap 50 iterations, tolerance 1e-6; scored against the fully sampled SSOS image"}
    cart = I.mask_gaussian_cartesian(M, N, rate=0.34, n_acs=22, seed=2000)
    out["models_cartesian_0.34"] = {name: run(cart, vc, sp, 22) for name, vc, sp in
                                    (("SHLR", False, False), ("SHLR-S", False, True), ("SHLR-V", True, False),
                                     ("SHLR-SV", True, True))}
    out["acs_sweep_shlr_sv"] = {str(a): run(I.mask_gaussian_cartesian(M, N, rate=0.34, n_acs=a, seed=2000), True,
                                            True, a) for a in range(8, 23, 2)}
    pats = {"uniform_R6_acs20": (I.mask_uniform_cartesian(M, N, R=6, n_acs=20), 20),
            "cartesian_pf3/4_0.30": (I.mask_gaussian_cartesian(M, N, rate=0.30, n_acs=22, seed=2000, pf=0.75), 22),
            "random2d_0.18": (I.mask_random_2d(M, N, rate=0.18, acs=16, seed=2000), 16),
            "random2d_pf4/5_0.17": (I.mask_random_2d(M, N, rate=0.17, acs=16, seed=2000, pf=0.8), 16),
            "uniform_R6_pf3/4": (I.mask_uniform_cartesian(M, N, R=6, n_acs=20, pf=0.75), 20)}
    out["patterns_shlr_sv"] = {name: run(m, True, True, a) for name, (m, a) in pats.items()}
    # parameter sweeps (Supplement S5): lambda and lambda1 of SHLR-SV at Cartesian 0.34
    def run_prm(lam, lam1):
        Y = I.undersample(k, cart)
        p = shlr.Params.paper_defaults(shlr.MODEL_PI, M=(M,), N=(N,), J=J, k_row=kw, k_col=kw, use_vc=True,
                                       lam=lam, lambda1=lam1, beta=30.0, tau=30.0, spirit_ksize=5, n_cg=10)
        plan = shlr.Plan(p)
        plan.init(torch.from_numpy(Y).to(torch.complex64).cuda(), torch.from_numpy(cart.astype(np.uint8)).cuda())
        plan.calibrate_spirit(acs=22, reg=1e-3)
        info = plan.iterate(p.max_iter)
        img = shlr.ssos(plan.kspace())
        plan.close()
        return {"rlne": shlr.rlne(truth, img), "mssim": shlr.mssim(truth, img), "iterations": info.iters_done}
    out["lambda_sweep_shlr_sv"] = {f"{v:g}": run_prm(v, 10.0) for v in (1e2, 1e3, 1e4, 1e5, 1e6)}
    out["lambda1_sweep_shlr_sv"] = {f"{v:g}": run_prm(1e4, v) for v in (0.1, 1.0, 10.0, 1e2, 1e3, 1e4)}
    # T2 maps (SHLR-P / SHLR-VP)
    L, J2 = 8, 12
    te = 10.0 * (np.arange(L) + 1)
    k2 = I.t2_kspace(J2, M, N, L=L, seed=1004)
    m2 = I.mask_t2_cartesian(L, N, R=6, n_center=16)
    t2_true, _, roi = shlr.t2_fit(shlr.ssos(torch.from_numpy(k2).to(torch.complex64).cuda()), te)
    res = {}
    for name, vc in (("SHLR-P", False), ("SHLR-VP", True)):
        p = shlr.Params(model=shlr.MODEL_PARAM, M=(M,), N=(N,), J=J2, L=L, k_row=kw, k_col=4, use_vc=vc, lam=1e4,
                        lambda2=2.0, beta=30.0, tau=30.0)
        plan = shlr.Plan(p)
        plan.init(torch.from_numpy(I.undersample(k2, m2[:, None, None, :])).to(torch.complex64).cuda(),
                  torch.from_numpy(m2.astype(np.uint8)).cuda())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.iterate(t2_iters)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        img = shlr.ssos(plan.kspace())
        plan.close()
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        t2_rec, _, _ = shlr.t2_fit(img, te)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        res[name] = {"t2_map_rlne": shlr.rlne(t2_true, t2_rec, roi), "iterations": t2_iters,
                     "it_per_s": t2_iters / (t1 - t0), "t2_fit_ms": 1e3 * (f1 - f0)}
    lam2_sweep = {}
    for l2 in (0.5, 1.0, 2.0, 5.0, 10.0):
        p = shlr.Params(model=shlr.MODEL_PARAM, M=(M,), N=(N,), J=J2, L=L, k_row=kw, k_col=4, use_vc=True, lam=1e4,
                        lambda2=l2, beta=30.0, tau=30.0)
        plan = shlr.Plan(p)
        plan.init(torch.from_numpy(I.undersample(k2, m2[:, None, None, :])).to(torch.complex64).cuda(),
                  torch.from_numpy(m2.astype(np.uint8)).cuda())
        plan.iterate(t2_iters)
        t2_rec, _, _ = shlr.t2_fit(shlr.ssos(plan.kspace()), te)
        plan.close()
        lam2_sweep[f"{l2:g}"] = {"t2_map_rlne": shlr.rlne(t2_true, t2_rec, roi)}
    res["lambda2_sweep_shlr_vp"] = lam2_sweep
    out["t2_maps_R6"] = {"workload": "T2 series 8 echoes x 12 coils x 256x256 (seed 1004), per-echo shifted R=6 + 16 "
                                     "centre lines, PE window 25, echo window 4, lambda 1e4, lambda2 2, beta = tau = 30; "
                                     "T2 maps fitted to the SSOS echo images (ROI 0.1, range 5..500 ms), RLNE over the "
                                     "ROI of the fully sampled map", "roi_pixels": int(roi.sum().item()), **res}
    return out


def timed_run(plan, steps, warmup, check_iters):
    """The accuracy-check iterations, the warm-up with every phase timed, then `steps` iterations timed
    with HIP events around the dominant phase only (each timed phase adds an event pair per launch)."""
    import numpy as np
    import torch
    k_check = None
    if check_iters > 0:
        plan.iterate(check_iters)
        k_check = plan.kspace().cpu().numpy().astype(np.complex128)
    names = ("gram", "eig", "reproj", "xupdate", "spirit", "tridiag")
    warm = None
    if warmup > 0:
        plan.timing_enable(True)
        plan.iterate(warmup)
        warm = plan.timing_read()
        plan.timing_enable(False)
        dom = max(names, key=lambda k: warm[k][0])
        plan.timing_enable_phases([dom])
    else:
        plan.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.iterate_async(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = plan.timing_read()
    plan.timing_enable(False)
    if warm is None:
        dom = max(names, key=lambda k: phases[k][0])
        warm, n_warm = phases, steps
    else:
        n_warm = warmup
    return {"k_check": k_check, "warm": warm, "n_warm": n_warm, "phases": phases, "dom": dom,
            "elapsed": t1 - t0}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64", "mixed-r32"], default="mixed",
                    help="mixed: FP32 MFMA products, FP64 eigen-solve (the default); fp64: FP64 throughout; "
                         "mixed-r32: the opt-in form whose Householder reduction runs in FP32")
    ap.add_argument("--quality-only", action="store_true",
                    help="only run the synthetic quality comparisons (models, ACS sweep, patterns, T2 maps) and "
                         "print them as one JSON line")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the comparison runs of the other precision forms on the same workload")
    ap.add_argument("--workload", choices=["pi256", "ragged", "t2"], default="pi256",
                    help="pi256: the headline 8-coil 256x256 SHLR-S iteration; ragged: 32 slices of 12 coils; "
                         "t2: the SHLR-VP T2 series")
    ap.add_argument("--check-iters", type=int, default=2,
                    help="iterations compared with the FP64 oracle (also the CPU-baseline sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-cg", type=int, default=10)
    ap.add_argument("--no-diff", action="store_true", help="skip the reverse-mode (differentiation) leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--diff-batch", type=int, default=8)
    ap.add_argument("--diff-steps", type=int, default=8)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path shards by slice / FE position "
              "with no communication, so N > 1 is not measured here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "copies": 3}))
        return
    from paper_2107_11650_amd import shlr
    if args.quality_only:
        print(json.dumps(quality_leg()))
        return

    kw, lam, lam1, beta = 25, 1e4, 10.0, 30.0
    precs = {"mixed": shlr.PREC_MIXED, "fp64": shlr.PREC_FP64, "mixed-r32": shlr.PREC_MIXED_R32}
    prec = precs[args.precision]
    plan, Y, mask, shapes, elems, cfg = build_workload(args.workload, prec, args.n_cg, tune=not args.no_autotune)
    run = timed_run(plan, args.steps, args.warmup, args.check_iters if args.workload == "pi256" else 0)
    k_check, warm, n_warm, phases, dom = run["k_check"], run["warm"], run["n_warm"], run["phases"], run["dom"]
    elapsed = run["elapsed"]
    value = args.steps / elapsed
    # the same iterations as replays of the captured one-iteration graph (no per-phase events inside)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    plan.iterate_async(args.steps, graph=True)
    torch.cuda.synchronize()
    g1 = time.perf_counter()

    # roofline of the dominant kernel: algorithmic work of one iteration / launches per iteration
    csize = 16 if prec == shlr.PREC_FP64 else 8
    work = lowrank_work(shapes)
    ms_dom, n_dom = phases[dom]
    avg_ms = ms_dom / max(n_dom, 1)
    launches_per_step = n_dom / args.steps
    if dom in ("gram", "reproj"):
        peak = PEAK_TFLOPS_FP64 if prec == shlr.PREC_FP64 else PEAK_TFLOPS_FP32_MFMA
        achieved = work[dom] / launches_per_step / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "unit": "TFLOP/s"}
    elif dom in ("eig", "tridiag"):
        # only the opt-in FP32-reduction form reduces in FP32; every other eigen-solve runs in FP64
        peak = PEAK_TFLOPS_FP32_VECTOR if (dom == "tridiag" and prec == shlr.PREC_MIXED_R32) else PEAK_TFLOPS_FP64
        achieved = work[dom] / launches_per_step / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "unit": "TFLOP/s"}
    else:
        # transform phases: one read and one write of each coil k-space array touched per launch
        peak = PEAK_HBM_GBS
        bytes_launch = 6 * elems * csize / launches_per_step
        achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "unit": "GB/s"}
    traffic = measured_traffic(dom, args.precision) if args.workload == "pi256" else None
    roof.update({"kernel": dom, "achieved": achieved, "peak": peak, "frac": achieved / peak,
                 "traffic": traffic, "avg_launch_ms": avg_ms, "launches": n_dom})

    result = {
        "metric": METRIC if args.workload == "pi256" else f"SHLR iterations/sec ({args.workload} workload)",
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == shlr.PREC_FP64 else "f32",
        "data": "synthetic",
        "config": {**cfg, "precision": args.precision,
                   "tridiag_dtype": "f32" if prec == shlr.PREC_MIXED_R32 else "f64", "eig_dtype": "f64"},
        "phases_ms_per_step": {k: v[0] / n_warm for k, v in warm.items()},
        "phases_timed_over": "warm-up iterations, every phase timed" if n_warm == args.warmup and args.warmup > 0
                             else "timed iterations",
        "roofline": roof,
        "graph_replay": {"value": args.steps / (g1 - g0), "ms_per_step": 1e3 * (g1 - g0) / args.steps,
                         "how": "the same step count right after the timed region, as replays of the hipGraph of one "
                                "iteration (shlr_iterate_graph); value above is the eager path with HIP events on the "
                                "dominant phase"},
    }

    # the low-rank step per iteration, from the phase times of the warm-up: the contraction kernels
    # against max(bytes / HBM, flops / MFMA), and the whole step (Gram, reduction, eigen-solve,
    # reprojection) against flops / MFMA + eigen flops / FP64 (13.3 s^3 per matrix), or bytes / HBM.
    # Bytes: D read by the Gram kernel, read and written by the reprojection.
    mfma_peak = PEAK_TFLOPS_FP64 if prec == shlr.PREC_FP64 else PEAK_TFLOPS_FP32_MFMA
    ms = {k: warm[k][0] / n_warm if k in warm else 0.0 for k in ("gram", "tridiag", "eig", "reproj")}
    d_bytes = sum(c * 3.0 * p * q * csize for p, q, c in shapes)
    t_hbm = d_bytes / (PEAK_HBM_GBS * 1e9) * 1e3
    t_mfma = (work["gram"] + work["reproj"]) / (mfma_peak * 1e12) * 1e3
    t_eig = work["eig"] / (PEAK_TFLOPS_FP64 * 1e12) * 1e3
    ms_contr = ms["gram"] + ms["reproj"]
    ms_whole = ms_contr + ms["tridiag"] + ms["eig"]
    if ms_contr > 0 and ms_whole > 0:
        result["lowrank_step"] = {
            "contraction": {"kernels": "gram + reproj", "ms_per_step": ms_contr, "bound_ms": max(t_hbm, t_mfma),
                            "bound": "mfma" if t_mfma >= t_hbm else "hbm", "frac": max(t_hbm, t_mfma) / ms_contr,
                            "tflops": (work["gram"] + work["reproj"]) / (ms_contr * 1e-3) / 1e12,
                            "peak_tflops": mfma_peak},
            "whole": {"kernels": "gram + tridiag + eig + reproj", "ms_per_step": ms_whole,
                      "bound_ms": max(t_hbm, t_mfma + t_eig), "frac": max(t_hbm, t_mfma + t_eig) / ms_whole,
                      "convention": "contractions at the MFMA peak of the data type; the eigen-solve counted as "
                                    "13.3 s^3 FP64 flops per matrix at the FP64 peak"},
            "d_bytes_per_step": d_bytes,
        }

    if not args.no_diff and args.workload == "pi256":
        result["differentiation"] = diff_leg(args.diff_batch, args.diff_steps, kw, lam, beta)

    if not args.no_cpu_baseline and args.workload == "pi256":
        from threadpoolctl import threadpool_info
        from oracle import shlr_oracle as O
        Yn = Y / np.abs(Y).max()
        g = O.spirit_calibrate(Yn, acs=24, ks=5)
        prm = O.PIParams(k_row=kw, k_col=kw, lam=lam, lam1=lam1, beta=beta, n_cg=args.n_cg,
                         iters=args.check_iters)
        c0 = time.perf_counter()
        k_ref = O.shlr_pi(Y, mask.astype(bool), prm, g=g)
        c1 = time.perf_counter()
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
        result["cpu_baseline"] = {
            "value": args.check_iters / (c1 - c0), "unit": "iterations/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {args.check_iters} iterations of the same workload (NumPy FP64, LAPACK SVD "
                      f"per lift, SPIRiT kernel calibrated beforehand)",
        }
        # the same oracle on one host thread, over its first iteration (a bounded sample)
        from threadpoolctl import threadpool_limits
        prm1 = O.PIParams(k_row=kw, k_col=kw, lam=lam, lam1=lam1, beta=beta, n_cg=args.n_cg, iters=1)
        with threadpool_limits(limits=1):
            c2 = time.perf_counter()
            O.shlr_pi(Y, mask.astype(bool), prm1, g=g)
            c3 = time.perf_counter()
        result["cpu_baseline"]["single_thread"] = {
            "value": 1.0 / (c3 - c2), "unit": "iterations/s", "cores": 1,
            "sample": "the first iteration of the same workload, BLAS limited to one thread"}
        result["nmse_vs_oracle"] = O.nmse(k_check, k_ref)
        result["nmse_iters"] = args.check_iters
        if not args.no_forms:
            # the other precision forms on the same workload, same step counts: throughput and error
            forms = {}
            for name, pv in precs.items():
                if pv == prec:
                    continue
                p2, *_ = build_workload(args.workload, pv, args.n_cg, tune=not args.no_autotune)
                r2 = timed_run(p2, args.steps, args.warmup, args.check_iters)
                p2.close()
                forms[name] = {"value": args.steps / r2["elapsed"], "ms_per_step": 1e3 * r2["elapsed"] / args.steps,
                               "nmse_vs_oracle": O.nmse(r2["k_check"], k_ref),
                               "tridiag_ms_per_step": r2["warm"]["tridiag"][0] / r2["n_warm"],
                               "eig_ms_per_step": r2["warm"]["eig"][0] / r2["n_warm"]}
            result["other_forms"] = forms
    plan.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
