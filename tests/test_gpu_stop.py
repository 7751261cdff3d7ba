"""GPU parity of the relative-change stop (Algorithms S1 / S2) against the FP64 oracle.

The stop test runs on the device, per unit: every slice of a parallel-imaging batch and every
frequency-encode position of the parameter model stops on its own change.  Each case picks the
tolerance from the oracle's own change history so that no iterate lies within 5% of it; the
GPU must then stop every unit at the oracle's iteration and return the oracle's K to the usual
bar (NMSE 1e-18 in FP64, 1e-12 mixed).
"""

import numpy as np
import pytest

from oracle import shlr_oracle as O
from paper_2107_11650_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_2107_11650_amd import shlr
    return shlr


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def first_below(hist, tol):
    """1-based iteration at which the change first falls below tol (the printed rule), else None."""
    for k, r in enumerate(hist):
        if r < tol:
            return k + 1
    return None


def pick_tol(histories, margin=1.05, want_distinct=True, t_max=1e-3):
    """A tolerance below t_max between two consecutive values of the first history such that no
    value of any history up to its stop lies within a factor `margin` of it; with want_distinct,
    the units stop at different iterations where possible."""
    cands = []
    h0 = histories[0]
    for k in range(1, len(h0)):
        a, b = h0[k - 1], h0[k]
        if b < a and np.sqrt(a * b) < t_max:
            cands.append(np.sqrt(a * b))
    best = None
    for t in sorted(cands, reverse=True):
        stops = [first_below(h, t) for h in histories]
        if any(s is None for s in stops):
            continue
        ok = all(abs(np.log(h[j] / t)) > np.log(margin) for h, s in zip(histories, stops) for j in range(s))
        if not ok:
            continue
        if best is None:
            best = (t, stops)
        if not want_distinct or len(set(stops)) > 1:
            return t, stops
    assert best is not None, "no tolerance with the required margin"
    return best


def pi_problem(J, M, N, seed):
    k = inputs.phantom_kspace(J, M, N, seed=1000 + seed)
    mask = inputs.mask_cartesian_vd(M, N, R=3.0, n_center=6, seed=2000 + seed)
    return inputs.undersample(k, mask), mask


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-18), ("mixed", 1e-12)])
def test_pi_slices_stop_on_their_own_change(prec, bar):
    shlr = _lib()
    probs = [pi_problem(2, 32, 40, seed=21), pi_problem(2, 40, 32, seed=22), pi_problem(2, 36, 36, seed=23)]
    prm = O.PIParams(k_row=5, k_col=5, lam=1e3, beta=6.0, iters=40)
    hist = []
    for Y, m in probs:
        _, st = O.shlr_pi(Y, m, prm, return_state=True)
        hist.append(np.array(st.rel_change))
    tol, stops = pick_tol(hist)
    print(f"tol={tol:.4e} oracle stops={stops}", flush=True)
    prm_t = O.PIParams(k_row=5, k_col=5, lam=1e3, beta=6.0, iters=40, tol=tol)
    refs, its = [], []
    for Y, m in probs:
        r, st = O.shlr_pi(Y, m, prm_t, return_state=True)
        refs.append(r)
        its.append(st.it)
    assert its == stops
    p = shlr.Params(M=tuple(Y.shape[1] for Y, _ in probs), N=tuple(Y.shape[2] for Y, _ in probs), J=2, k_row=5,
                    k_col=5, lam=1e3, beta=6.0, tau=6.0, tol=tol, max_iter=40,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.init(torch.cat([dev(Y, plan.cdtype).reshape(-1) for Y, _ in probs]),
              torch.cat([dev(m.astype(np.uint8), torch.uint8).reshape(-1) for _, m in probs]))
    info = plan.iterate(40)
    it, rel, act = plan.unit_status()
    out = host(plan.kspace())
    plan.close()
    print(f"gpu iters={it.tolist()} info.iters_done={info.iters_done} converged={info.converged}", flush=True)
    assert it.tolist() == stops
    assert not act.any() and info.converged == 1 and info.iters_done == max(stops)
    o = 0
    for (Y, _), ref in zip(probs, refs):
        e = O.nmse(out[o:o + Y.size].reshape(Y.shape), ref)
        o += Y.size
        print(f"  slice nmse={e:.3e}", flush=True)
        assert e < bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-18), ("mixed", 1e-12)])
def test_pi_stop_through_the_graph(prec, bar):
    """The stop test inside the captured graph: replays past a unit's stop leave its K alone."""
    shlr = _lib()
    probs = [pi_problem(2, 32, 40, seed=21), pi_problem(2, 40, 32, seed=22)]
    prm = O.PIParams(k_row=5, k_col=5, lam=1e3, beta=6.0, iters=30)
    hist = [np.array(O.shlr_pi(Y, m, prm, return_state=True)[1].rel_change) for Y, m in probs]
    tol, stops = pick_tol(hist)
    prm_t = O.PIParams(k_row=5, k_col=5, lam=1e3, beta=6.0, iters=30, tol=tol)
    refs = [O.shlr_pi(Y, m, prm_t) for Y, m in probs]
    p = shlr.Params(M=(32, 40), N=(40, 32), J=2, k_row=5, k_col=5, lam=1e3, beta=6.0, tau=6.0, tol=tol, max_iter=30,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.init(torch.cat([dev(Y, plan.cdtype).reshape(-1) for Y, _ in probs]),
              torch.cat([dev(m.astype(np.uint8), torch.uint8).reshape(-1) for _, m in probs]))
    plan.iterate(max(stops) + 3, graph=True)
    it, _, act = plan.unit_status()
    out = host(plan.kspace())
    plan.close()
    assert it.tolist() == stops and not act.any()
    o = 0
    for (Y, _), ref in zip(probs, refs):
        e = O.nmse(out[o:o + Y.size].reshape(Y.shape), ref)
        o += Y.size
        assert e < bar, e


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-18), ("mixed", 1e-12)])
def test_spirit_stop(prec, bar):
    """SHLR-S: the PCG X-update feeds the same change test."""
    shlr = _lib()
    J, M, N = 4, 48, 40
    k = inputs.phantom_kspace(J, M, N, seed=1007)
    mask = inputs.mask_poisson_disc(M, N, R=3.0, acs=16, seed=2007)
    Y = inputs.undersample(k, mask)
    g = O.spirit_calibrate(Y / np.abs(Y).max(), acs=16, ks=5)
    prm = O.PIParams(k_row=6, k_col=6, lam=1e4, lam1=10.0, beta=10.0, n_cg=6, iters=30)
    _, st = O.shlr_pi(Y, mask, prm, g=g, return_state=True)
    tol, stops = pick_tol([np.array(st.rel_change)], want_distinct=False)
    prm.tol = tol
    ref, st = O.shlr_pi(Y, mask, prm, g=g, return_state=True)
    assert st.it == stops[0]
    p = shlr.Params(M=(M,), N=(N,), J=J, k_row=6, k_col=6, lam=1e4, lambda1=10.0, beta=10.0, tau=10.0, n_cg=6,
                    spirit_ksize=5, tol=tol, max_iter=30,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.init(dev(Y, plan.cdtype), dev(mask.astype(np.uint8), torch.uint8))
    plan.set_spirit_kernel(g)
    info = plan.iterate(30)
    it, rel, act = plan.unit_status()
    out = host(plan.kspace())
    plan.close()
    e = O.nmse(out, ref)
    print(f"SPIRiT stop: oracle {stops[0]}, gpu {it.tolist()} rel={rel.tolist()} nmse={e:.3e}", flush=True)
    assert np.isfinite(info.rel_change) and info.rel_change < tol
    assert it.tolist() == stops and info.converged == 1
    assert e < bar


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-18), ("mixed", 1e-12)])
def test_param_fe_positions_stop_on_their_own_change(prec, bar):
    shlr = _lib()
    L, J, M, N = 6, 3, 5, 48
    k = inputs.t2_kspace(J, M, N, L=L, seed=1011)
    # seeded noise, so that every FE position (the border rows of the phantom too) carries signal
    k = k + 0.02 * np.abs(k).max() * inputs.random_complex(k.shape, seed=1012)
    mask = inputs.mask_t2_cartesian(L, N, R=3, n_center=8)
    Y = inputs.undersample(k, mask[:, None, None, :])
    prm = O.ParamParams(k_pe=6, k_l=3, lam=1e3, lam2=2.0, beta=8.0, iters=40)
    _, st = O.shlr_param(Y, mask, prm, return_state=True)
    hist = np.array(st.rel_change)                     # (iters, M)
    tol, stops = pick_tol([hist[:, m] for m in range(M)])
    prm.tol = tol
    ref, st = O.shlr_param(Y, mask, prm, return_state=True)
    print(f"tol={tol:.4e} oracle stops={st.it_fe.tolist()}", flush=True)
    assert st.it_fe.tolist() == stops
    p = shlr.Params(model=shlr.MODEL_PARAM, M=(M,), N=(N,), J=J, L=L, k_row=6, k_col=3, lam=1e3, lambda2=2.0,
                    beta=8.0, tau=8.0, tol=tol, max_iter=40,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.init(dev(Y, plan.cdtype), dev(mask.astype(np.uint8), torch.uint8))
    info = plan.iterate(40)
    it, rel, act = plan.unit_status()
    out = host(plan.kspace())
    plan.close()
    e = O.nmse(out, ref)
    print(f"PARAM stop: gpu {it.tolist()} nmse={e:.3e}", flush=True)
    assert it.tolist() == stops and not act.any() and info.converged == 1
    assert e < bar


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_eigenpair_check_reports_through_status_and_flags(prec):
    """The residual check of every eigenpair (shlr_set_eig_check): passes at the default bound with
    no flag; forced to fail from the host with a zero bound, the call returns SHLR_E_EIG_NOCONV and
    bit 1 of the device flags while the iterate itself is unchanged."""
    import ctypes
    shlr = _lib()
    Y, m = pi_problem(2, 32, 40, seed=21)
    p = shlr.Params(M=(32,), N=(40,), J=2, k_row=5, k_col=5, lam=1e3, beta=6.0, tau=6.0,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    outs = []
    for lim in (None, 0.0):
        plan = shlr.Plan(p)
        plan.init(dev(Y, plan.cdtype), dev(m.astype(np.uint8), torch.uint8))
        if lim is not None:
            plan.set_eig_check(lim)
        info = shlr.CInfo()
        st = shlr.library().shlr_iterate(plan._h, 4, ctypes.byref(info))
        if lim is None:
            assert st == 0 and info.device_flags == 0
        else:
            assert st == 8, shlr.library().shlr_last_error()
            assert info.device_flags & 2 and not info.device_flags & 1
        outs.append(host(plan.kspace()))
        plan.close()
    assert np.array_equal(outs[0], outs[1])
