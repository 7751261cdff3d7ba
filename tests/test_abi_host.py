"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and validates plans without touching a GPU."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shlr.h")
LIB = os.path.join(ROOT, "paper_2107_11650_amd", "libshlr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libshlr.so not built (run __graft_entry__.build())")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(shlr_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    from paper_2107_11650_amd import shlr
    assert sorted(shlr.EXPORTED) == declared_functions()


def test_version_string():
    from paper_2107_11650_amd import shlr
    assert "gfx950" in shlr.version()


def _p(**kw):
    from paper_2107_11650_amd import shlr
    return shlr.Params(**kw)


def test_valid_plans_report_workspace():
    from paper_2107_11650_amd import shlr
    b1 = shlr.plan_check(_p(M=(64,), N=(64,), J=4, k_row=8, k_col=8))
    b2 = shlr.plan_check(_p(M=(256,), N=(256,), J=8, k_row=25, k_col=25))
    assert 0 < b1 < b2
    # FP64 form needs more memory than the mixed form
    assert shlr.plan_check(_p(precision=shlr.PREC_FP64)) > b1
    # ragged slices and the parameter model
    assert shlr.plan_check(_p(M=(40, 64), N=(48, 32), J=2, k_row=5, k_col=5)) > 0
    assert shlr.plan_check(_p(model=shlr.MODEL_PARAM, M=(8,), N=(64,), L=8, J=4, k_row=8, k_col=4, use_vc=True)) > 0


@pytest.mark.parametrize("kw,code", [
    (dict(beta=0.0), 1),
    (dict(beta=float("nan")), 1),
    (dict(tau=-1.0), 1),
    (dict(lam=0.0), 1),
    (dict(k_row=65), 1),
    (dict(k_col=0), 1),
    (dict(J=0), 1),
    (dict(M=(0,), N=(64,)), 1),
    (dict(model=7), 1),
    (dict(precision=3), 1),
    (dict(spirit_ksize=4), 1),
    (dict(spirit_ksize=5, hard_dc=True), 6),
    (dict(M=(1024,), N=(1024,), J=16, k_row=25, k_col=25), 6),   # min(p, q) > 320
    # FP64 virtual-coil lifts of 12-coil 256-point lines: line table beyond the LDS staging
    (dict(M=(256,), N=(256,), J=12, k_row=25, k_col=25, use_vc=True, precision=1), 6),
    (dict(slot_budget=-1), 1),
])
def test_invalid_plans_are_rejected(kw, code):
    from paper_2107_11650_amd import shlr
    with pytest.raises(shlr.ShlrError) as ei:
        shlr.plan_check(_p(**kw))
    assert ei.value.code == code
    assert str(ei.value)


def test_slot_budget_bounds_the_workspace():
    # a run's eigen-solver slots follow the budget: a small one gives a smaller workspace (more
    # chunks of launches), the default 0 is the 16 GiB budget, and a budget under one slot still
    # leaves one slot per run
    from paper_2107_11650_amd import shlr
    kw = dict(M=(40, 64), N=(48, 32), J=2, k_row=5, k_col=5)
    full = shlr.plan_check(_p(**kw))
    assert shlr.plan_check(_p(slot_budget=16 << 30, **kw)) == full
    small = shlr.plan_check(_p(slot_budget=1 << 20, **kw))
    one = shlr.plan_check(_p(slot_budget=1, **kw))
    assert 0 < one < small < full


def test_param_model_validation():
    from paper_2107_11650_amd import shlr
    with pytest.raises(shlr.ShlrError):
        shlr.plan_check(_p(model=shlr.MODEL_PARAM, M=(8, 8), N=(64, 64), L=8))   # one series only
    with pytest.raises(shlr.ShlrError):
        shlr.plan_check(_p(model=shlr.MODEL_PARAM, M=(8,), N=(64,), L=8, lambda2=0.0))
    with pytest.raises(shlr.ShlrError):
        shlr.plan_check(_p(model=shlr.MODEL_PARAM, M=(8,), N=(64,), L=8, k_col=9))


def test_lowrank_workspace_size_and_errors():
    from paper_2107_11650_amd import shlr
    assert shlr.lowrank_workspace_size(shlr.PREC_MIXED, 16, 4, 64, 8, False) > 0
    with pytest.raises(shlr.ShlrError):
        shlr.lowrank_workspace_size(shlr.PREC_MIXED, 16, 4, 64, 65, False)
    with pytest.raises(shlr.ShlrError):
        shlr.lowrank_workspace_size(5, 16, 4, 64, 8, False)
    # the same 12-coil virtual-coil shape is fine in mixed precision, unsupported in FP64
    assert shlr.lowrank_workspace_size(shlr.PREC_MIXED, 3, 12, 256, 25, True) > 0
    with pytest.raises(shlr.ShlrError) as ei:
        shlr.lowrank_workspace_size(shlr.PREC_FP64, 3, 12, 256, 25, True)
    assert ei.value.code == 6


def _raw_plan(shlr, **kw):
    import ctypes
    c, keep = _p(**kw).to_c()
    h = ctypes.c_void_p()
    shlr._check(shlr.library().shlr_plan_create(ctypes.byref(c), ctypes.byref(h)))
    return h, keep


@pytest.mark.parametrize("kw,ok", [
    (dict(normalize=False), True),
    (dict(normalize=False, use_vc=True, M=(40, 64), N=(48, 32), J=2, k_row=5, k_col=5), True),
    (dict(normalize=True), False),                         # the caller scales Y
    (dict(normalize=False, hard_dc=True), False),          # lambda = inf has no lambda derivative
    (dict(normalize=False, spirit_ksize=5, lambda1=1.0), False),
    (dict(normalize=False, model=1, M=(8,), N=(64,), L=8, k_col=4), False),
    (dict(normalize=False, precision=2), False),           # the opt-in FP32 reduction: not differentiated
])
def test_unrolled_scope_and_sizes(kw, ok):
    import ctypes
    from paper_2107_11650_amd import shlr
    h, keep = _raw_plan(shlr, **kw)
    try:
        ck, wk = ctypes.c_size_t(), ctypes.c_size_t()
        st = shlr.library().shlr_unrolled_sizes(h, 4, ctypes.byref(ck), ctypes.byref(wk))
        if ok:
            assert st == 0 and ck.value > 0 and wk.value > 0
            # checkpoints: K after each of 4 X-updates + D before each of 3 low-rank steps
            st1 = shlr.library().shlr_unrolled_sizes(h, 1, ctypes.byref(ck), ctypes.byref(wk))
            assert st1 == 0
        else:
            assert st == 6, shlr.library().shlr_last_error()
        assert shlr.library().shlr_unrolled_sizes(h, 0, ctypes.byref(ck), ctypes.byref(wk)) != 0
    finally:
        shlr.library().shlr_plan_destroy(h)


def test_library_defaults_are_the_papers():
    # shlr_params_default against the values Algorithms S1 / S2 print (tests/golden/paper_constants.json)
    import json
    from paper_2107_11650_amd import shlr
    with open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")) as f:
        c = json.load(f)
    pi = shlr.Params.paper_defaults(shlr.MODEL_PI)
    pa = shlr.Params.paper_defaults(shlr.MODEL_PARAM)
    assert pi.max_iter == c["alg_s1_caps"]["max_iter"] and pi.tol == c["alg_s1_caps"]["tol"]
    assert pa.max_iter == c["alg_s2_caps"]["max_iter"] and pa.tol == c["alg_s2_caps"]["tol"]
    assert pi.d0 == pa.d0 == c["alg_init"]["d0"]
    assert pi.precision == shlr.PREC_MIXED and pi.use_w and pi.normalize and not pi.use_vc
    with pytest.raises(shlr.ShlrError):
        shlr.Params.paper_defaults(7)


def test_unit_status_needs_an_initialised_plan():
    import ctypes
    from paper_2107_11650_amd import shlr
    h, keep = _raw_plan(shlr, M=(40, 64), N=(48, 32), J=2, k_row=5, k_col=5)
    try:
        it = (ctypes.c_int32 * 2)()
        st = shlr.library().shlr_unit_status(h, 2, it, None, None)
        assert st == 7, shlr.library().shlr_last_error()      # SHLR_E_STATE: no shlr_init yet
    finally:
        shlr.library().shlr_plan_destroy(h)


def test_eig_check_limit_is_validated():
    import ctypes
    from paper_2107_11650_amd import shlr
    h, keep = _raw_plan(shlr, M=(32,), N=(32,), J=2, k_row=4, k_col=4)
    try:
        lib = shlr.library()
        assert lib.shlr_set_eig_check(h, ctypes.c_double(-1.0)) == 1
        assert lib.shlr_set_eig_check(h, ctypes.c_double(float("nan"))) == 1
        assert lib.shlr_set_eig_check(h, ctypes.c_double(float("inf"))) == 1
        assert lib.shlr_set_eig_check(h, ctypes.c_double(0.0)) == 0
        assert lib.shlr_set_eig_check(h, ctypes.c_double(1e-6)) == 0
        assert lib.shlr_set_eig_check(None, ctypes.c_double(1e-6)) == 1
    finally:
        shlr.library().shlr_plan_destroy(h)


def test_set_weights_argument_checks():
    import ctypes
    from paper_2107_11650_amd import shlr
    lib = shlr.library()
    # no workspace bound yet: refused before any device access
    h, keep = _raw_plan(shlr, M=(32,), N=(32,), J=2, k_row=4, k_col=4)
    try:
        assert lib.shlr_set_weights(h, ctypes.c_void_p(16), ctypes.c_void_p(16)) == 4
        assert lib.shlr_set_weights(None, None, None) == 1
    finally:
        lib.shlr_plan_destroy(h)


def test_noalloc_rejects_batches_beyond_its_fixed_scratch():
    # a million 320-point lines need 72 MB of descriptors alone: refused before any device access
    from paper_2107_11650_amd import shlr
    lib = shlr.library()
    st = lib.shlr_lowrank_lines_noalloc(0, 1000000, 12, 320, 25, 0, 1, 3.0, 2.0, 1.0, None, None, None, None, None)
    assert st == 4 and b"fixed scratch" in lib.shlr_last_error()
    assert lib.shlr_lowrank_lines_noalloc(0, -1, 4, 64, 8, 0, 1, 3.0, 2.0, 1.0, None, None, None, None, None) == 1
