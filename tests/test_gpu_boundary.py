"""GPU checks of boundary calls beyond the iteration itself: caller weights W (shlr_set_weights)."""

import numpy as np
import pytest

from oracle import shlr_oracle as O
from paper_2107_11650_amd import inputs
from parity_util import check

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


BARS = {"fp64": (1e-18, 1e-11), "mixed": (1e-12, 2e-4)}


def _slices():
    out = []
    for seed, (M, N) in ((31, (32, 40)), (32, (40, 36))):
        k = inputs.phantom_kspace(2, M, N, seed=1000 + seed)
        m = inputs.mask_cartesian_vd(M, N, R=2.5, n_center=6, seed=2000 + seed)
        out.append((inputs.undersample(k, m), m))
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_caller_weights_pi_two_slices(prec):
    shlr = _lib()
    probs = _slices()
    ws = [(inputs.random_complex(Y.shape[2], seed=70 + i) + 1.0, inputs.random_complex(Y.shape[1], seed=80 + i) + 1.0)
          for i, (Y, _) in enumerate(probs)]
    p = shlr.Params(M=tuple(Y.shape[1] for Y, _ in probs), N=tuple(Y.shape[2] for Y, _ in probs), J=2, k_row=5,
                    k_col=5, use_vc=True, lam=1e3, beta=6.0, tau=6.0, max_iter=5,
                    precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.set_weights(np.concatenate([w[0] for w in ws]), np.concatenate([w[1] for w in ws]))
    plan.init(torch.cat([dev(Y, plan.cdtype).reshape(-1) for Y, _ in probs]),
              torch.cat([dev(m.astype(np.uint8), torch.uint8).reshape(-1) for _, m in probs]))
    plan.iterate(5)
    out = host(plan.kspace())
    plan.close()
    o = 0
    for (Y, m), (wr, wc) in zip(probs, ws):
        prm = O.PIParams(k_row=5, k_col=5, lam=1e3, beta=6.0, vc=True, iters=5, w_row=wr, w_col=wc)
        check(out[o:o + Y.size].reshape(Y.shape), O.shlr_pi(Y, m, prm), *BARS[prec], label=f"weights {Y.shape} {prec}")
        o += Y.size


def test_default_weights_given_explicitly_change_nothing():
    shlr = _lib()
    (Y, m), = _slices()[:1]
    p = shlr.Params(M=(Y.shape[1],), N=(Y.shape[2],), J=2, k_row=5, k_col=5, lam=1e3, beta=6.0, tau=6.0)
    outs = []
    for explicit in (False, True):
        plan = shlr.Plan(p)
        if explicit:
            plan.set_weights(O.weights(Y.shape[2]), O.weights(Y.shape[1]))
        plan.init(dev(Y, plan.cdtype), dev(m.astype(np.uint8), torch.uint8))
        plan.iterate(4)
        outs.append(host(plan.kspace()))
        plan.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_caller_weights_param(prec):
    shlr = _lib()
    L, J, M, N = 6, 3, 4, 48
    k = inputs.t2_kspace(J, M, N, L=L, seed=1021)
    mask = inputs.mask_t2_cartesian(L, N, R=3, n_center=8)
    Y = inputs.undersample(k, mask[:, None, None, :])
    w = inputs.random_complex(N, seed=90) + 1.0
    prm = O.ParamParams(k_pe=6, k_l=3, lam=1e3, lam2=2.0, beta=8.0, vc=True, iters=5, w_pe=w)
    ref = O.shlr_param(Y, mask, prm)
    p = shlr.Params(model=shlr.MODEL_PARAM, M=(M,), N=(N,), J=J, L=L, k_row=6, k_col=3, use_vc=True, lam=1e3,
                    lambda2=2.0, beta=8.0, tau=8.0, precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    plan = shlr.Plan(p)
    plan.set_weights(w)
    plan.init(dev(Y, plan.cdtype), dev(mask.astype(np.uint8), torch.uint8))
    plan.iterate(5)
    out = host(plan.kspace())
    plan.close()
    check(out, ref, *BARS[prec], label=f"PARAM weights {prec}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_with_spirit_match_eager(prec):
    """The captured iteration with the SPIRiT PCG X-update: each replay, with eager work and a
    synchronisation between replays (reading K back), equals the eager iteration bit for bit."""
    shlr = _lib()
    J, M, N = 4, 48, 40
    k = inputs.phantom_kspace(J, M, N, seed=1008)
    mask = inputs.mask_poisson_disc(M, N, R=3.0, acs=16, seed=2008)
    Y = inputs.undersample(k, mask)
    p = shlr.Params(M=(M,), N=(N,), J=J, k_row=6, k_col=6, use_vc=True, lam=1e4, lambda1=10.0, beta=10.0, tau=10.0,
                    n_cg=6, spirit_ksize=5, precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
    runs = []
    for graph in (False, True):
        plan = shlr.Plan(p)
        plan.init(dev(Y, plan.cdtype), dev(mask.astype(np.uint8), torch.uint8))
        plan.calibrate_spirit(acs=16, reg=1e-3)
        ks = []
        for _ in range(4):
            plan.iterate(1, graph=graph)
            ks.append(host(plan.kspace()))
        plan.close()
        runs.append(ks)
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    g = O.spirit_calibrate(Y / np.abs(Y).max(), acs=16, ks=5)
    ref = O.shlr_pi(Y, mask, O.PIParams(k_row=6, k_col=6, lam=1e4, lam1=10.0, beta=10.0, vc=True, n_cg=6, iters=4), g=g)
    check(runs[1][-1], ref, *BARS[prec], label=f"graph SHLR-SV {prec}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chunked_runs_match_one_chunk(prec):
    """A slot budget under one run's size splits each run into chunks with launches of their own
    (the per-matrix work is the same): three iterations of a ragged three-slice batch give K
    bitwise equal to the default budget's single chunk per run."""
    shlr = _lib()
    probs = _slices() + [(lambda k, m: (inputs.undersample(k, m), m))(
        inputs.phantom_kspace(2, 48, 44, seed=1033), inputs.mask_cartesian_vd(48, 44, R=2.5, n_center=6, seed=2033))]
    outs = []
    for budget in (0, 1 << 20):
        p = shlr.Params(M=tuple(Y.shape[1] for Y, _ in probs), N=tuple(Y.shape[2] for Y, _ in probs), J=2, k_row=5,
                        k_col=5, lam=1e3, beta=6.0, tau=6.0, max_iter=3, slot_budget=budget,
                        precision=shlr.PREC_FP64 if prec == "fp64" else shlr.PREC_MIXED)
        print(f"slot budget {budget}: workspace {shlr.plan_check(p)} bytes", flush=True)
        plan = shlr.Plan(p)
        plan.init(torch.cat([dev(Y, plan.cdtype).reshape(-1) for Y, _ in probs]),
                  torch.cat([dev(m.astype(np.uint8), torch.uint8).reshape(-1) for _, m in probs]))
        plan.iterate(3)
        outs.append(host(plan.kspace()))
        plan.close()
    assert np.array_equal(outs[0], outs[1])

