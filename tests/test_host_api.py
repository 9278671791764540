"""Host logic of the C ABI that runs without a GPU: workspace sizes of the
schedules and the argument checks that return IPR_EARG before any device
call (the pointers passed are never dereferenced on these paths)."""
import ctypes as ct

import pytest

import paper_1703_02283_amd as ipr
from paper_1703_02283_amd import binding

FAKE_A = ct.c_void_p(4096)      # never dereferenced: every call below fails its checks first
FAKE_C = ct.c_void_p(8192)
FAKE_W = ct.c_void_p(16384)


@pytest.fixture(scope="module", autouse=True)
def lib():
    ipr.load()


def solve_rc(n=64, p=2, tol=1e-10, **kw):
    s = ipr.ipr_schedule_default(**kw)
    res = ipr.IprResult()
    return binding._fn("ipr_solve")(FAKE_A, FAKE_C, n, p, tol, ct.byref(s), ct.byref(res),
                                    FAKE_W, 1 << 40, None)


def test_workspace_grows_with_each_option():
    n = 4096
    base = ipr.ipr_workspace_size(n, 2, 1, ipr.ipr_schedule_default())
    emul10 = ipr.ipr_workspace_size(n, 2, 1, ipr.ipr_schedule_default(
        bulk_dtype=ipr.IPR_FP64_INT8_EMUL))
    emul12 = ipr.ipr_workspace_size(n, 2, 1, ipr.ipr_schedule_default(
        bulk_dtype=ipr.IPR_FP64_INT8_EMUL, emul_slices=12))
    store = ipr.ipr_workspace_size(n, 2, 1, ipr.ipr_schedule_default(
        store_format=ipr.IPR_STORE_FLOAT, store_bits=10))
    nn8 = n * n * 8
    # (the size is the larger of the single solve's and one batched item's)
    assert base >= 6 * nn8                      # p = 2: six float64 work matrices
    # int8 slices: two operands of s digit matrices, two float64 scratch matrices
    assert emul10 >= 6 * nn8 + 2 * 10 * n * n + 2 * nn8
    assert emul12 - emul10 >= 2 * 2 * n * n
    assert store >= 7 * nn8                     # and A as stored
    assert ipr.ipr_workspace_size(n, 3, 1, ipr.ipr_schedule_default()) >= 7 * nn8   # p = 3


def test_product_workspaces():
    assert ipr.ipr_gemm_emul_workspace(1000, 10) >= 2 * 10 * 1024 * 1024 + 2 * 1000 * 1000 * 8
    assert ipr.ipr_gemm_emul_workspace(1000, 0) == 0
    assert ipr.ipr_gemm_emul_workspace(1000, 13) == 0
    assert ipr.ipr_gemm_emul_workspace(0, 10) == 0
    lw = binding._fn("ipr_lowdin_workspace")
    assert lw(3000, None) >= 3000 * 3000 * 8
    assert lw(3000, None) >= ipr.ipr_workspace_size(3000, 2, 1, None)
    assert lw(0, None) == 0


@pytest.mark.parametrize("kw", [
    {"bulk_dtype": 5},
    {"bulk_dtype": ipr.IPR_FP64_INT8_EMUL, "emul_slices": 13},
    {"bulk_dtype": ipr.IPR_FP64_INT8_EMUL, "emul_slices": -2},
    {"bulk_dtype": ipr.IPR_FP64_INT8_EMUL, "evaluation": ipr.IPR_EVAL_LITERAL},
    {"store_format": 3, "store_bits": 8},
    {"store_format": ipr.IPR_STORE_FLOAT, "store_bits": 0},
    {"store_format": ipr.IPR_STORE_FLOAT, "store_bits": 53},
    {"store_format": ipr.IPR_STORE_FIXED, "store_bits": 65},
    {"store_format": ipr.IPR_STORE_FLOAT, "store_bits": 10, "dynamic_scaling": 1},
    {"store_format": ipr.IPR_STORE_FLOAT, "store_bits": 10, "scale_squarings": 3},
    {"store_format": ipr.IPR_STORE_FLOAT, "store_bits": 10, "init": ipr.IPR_INIT_PAPER_EQ3},
    {"store_format": ipr.IPR_STORE_FIXED, "store_bits": 10, "bulk_dtype": ipr.IPR_BF16},
    {"evaluation": ipr.IPR_EVAL_NEWTON_SCHULZ},      # p = 2
    {"init": 9},
])
def test_solve_rejects_bad_schedules_before_any_device_call(kw):
    assert solve_rc(**kw) == ipr.IPR_EARG
    assert ipr.ipr_last_error()


def test_solve_rejects_bad_sizes_and_aliasing():
    assert solve_rc(n=0) == ipr.IPR_EARG
    assert solve_rc(p=0) == ipr.IPR_EARG
    assert solve_rc(tol=0.0) == ipr.IPR_EARG
    s = ipr.ipr_schedule_default()
    res = ipr.IprResult()
    rc = binding._fn("ipr_solve")(FAKE_A, FAKE_A, 64, 2, 1e-10, ct.byref(s), ct.byref(res),
                                  FAKE_W, 1 << 40, None)
    assert rc == ipr.IPR_EARG and "alias" in ipr.ipr_last_error()


def test_int8_slice_product_rejects_bad_arguments_before_any_device_call():
    f = binding._fn("ipr_gemm_emul")
    D = ct.c_void_p(1 << 20)
    for tri in (0, 1):
        for slices in (0, 13):
            assert f(FAKE_A, FAKE_C, D, 64, slices, tri, FAKE_W, 1 << 40, None) == ipr.IPR_EARG
        assert f(FAKE_A, FAKE_C, FAKE_A, 64, 10, tri, FAKE_W, 1 << 40, None) == ipr.IPR_EARG
        assert f(FAKE_A, FAKE_C, D, 200000, 10, tri, FAKE_W, 1 << 40, None) == ipr.IPR_EARG
        assert f(FAKE_A, FAKE_C, D, 64, 10, tri, FAKE_W, 16, None) == ipr.IPR_EARG


def test_low_precision_product_rejects_bad_arguments_before_any_device_call():
    f = binding._fn("ipr_gemm_lowp")
    D = ct.c_void_p(1 << 20)
    for tri in (0, 1):
        for dtype in (0, 4, 7):                     # FP64, INT8 emulation, unknown
            assert f(FAKE_A, FAKE_C, D, 64, dtype, tri, FAKE_W, 1 << 40, None) == ipr.IPR_EARG
        assert f(FAKE_A, FAKE_C, FAKE_A, 64, 1, tri, FAKE_W, 1 << 40, None) == ipr.IPR_EARG
        assert f(FAKE_A, FAKE_C, D, 64, 1, tri, FAKE_W, 16, None) == ipr.IPR_EARG


def test_lowdin_rejects_aliasing_and_short_workspace():
    f = binding._fn("ipr_lowdin")
    H = ct.c_void_p(1 << 21)
    X = ct.c_void_p(1 << 22)
    Ht = ct.c_void_p(1 << 23)
    s = ipr.ipr_schedule_default()
    res = ipr.IprResult()
    assert f(FAKE_A, H, X, H, 64, 1e-10, ct.byref(s), ct.byref(res), FAKE_W, 1 << 40,
             None) == ipr.IPR_EARG
    assert f(FAKE_A, H, H, Ht, 64, 1e-10, ct.byref(s), ct.byref(res), FAKE_W, 1 << 40,
             None) == ipr.IPR_EARG
    assert f(FAKE_A, H, X, Ht, 64, 1e-10, ct.byref(s), ct.byref(res), FAKE_W, 64,
             None) == ipr.IPR_EARG


def test_eigvalsh_checks_arguments_and_workspace_before_any_device_call():
    f = binding._fn("ipr_eigvalsh")
    ws = binding._fn("ipr_eigvalsh_workspace")
    assert ws(0) == 0 and ws(-3) == 0
    # the working copy of A dominates: at least n^2 doubles, growing with n
    assert ws(100) >= 100 * 100 * 8 and ws(1000) >= 1000 * 1000 * 8 and ws(1000) > ws(100)
    W = ct.c_void_p(32768)
    assert f(None, 64, W, FAKE_W, 1 << 30, None) == ipr.IPR_EARG
    assert f(FAKE_A, 64, None, FAKE_W, 1 << 30, None) == ipr.IPR_EARG
    assert f(FAKE_A, 64, W, None, 1 << 30, None) == ipr.IPR_EARG
    assert f(FAKE_A, 0, W, FAKE_W, 1 << 30, None) == ipr.IPR_EARG
    assert f(FAKE_A, 64, W, FAKE_W, ws(64) - 512, None) == ipr.IPR_EARG
    assert "workspace too small" in ipr.ipr_last_error()


def test_noalloc_rejects_what_it_cannot_hold_before_any_device_call():
    f = binding._fn("ipr_solve_noalloc")
    res = ipr.IprResult()

    def rc(n, p=2, **kw):
        s = ipr.ipr_schedule_default(**kw)
        return f(FAKE_A, FAKE_C, n, p, 1e-10, ct.byref(s), ct.byref(res), None)

    assert rc(0) == ipr.IPR_EARG
    assert rc(64, p=0) == ipr.IPR_EARG and rc(64, p=65) == ipr.IPR_EARG
    assert rc(64, timing=1) == ipr.IPR_EARG
    assert rc(4096) == ipr.IPR_EARG
    assert "fixed scratch" in ipr.ipr_last_error()


def test_batched_rejects_bad_arguments_before_any_device_call():
    f = binding._fn("ipr_solve_batched")
    offs = (ct.c_int64 * 2)(0, 64 * 64)
    ns = (ct.c_int * 2)(64, 64)
    ps = (ct.c_int * 2)(2, 2)

    def rc(batch=2, tol=1e-10, n=None, p=None, o=None, **kw):
        s = ipr.ipr_schedule_default(**kw)
        return f(FAKE_A, FAKE_C, o or offs, n or ns, p or ps, batch, tol, ct.byref(s), None,
                 FAKE_W, 1 << 40, None)

    assert rc(batch=0) == ipr.IPR_EARG
    assert rc(tol=0.0) == ipr.IPR_EARG and rc(tol=float("nan")) == ipr.IPR_EARG
    assert rc(init=ipr.IPR_INIT_PAPER_EQ3) == ipr.IPR_EARG
    assert rc(bulk_dtype=ipr.IPR_FP16) == ipr.IPR_EARG
    assert rc(tile=48) == ipr.IPR_EARG
    assert rc(max_iter=-1) == ipr.IPR_EARG
    assert rc(scale_lanczos=1, scale_squarings=6) == ipr.IPR_EARG
    assert rc(n=(ct.c_int * 2)(64, 1025)) == ipr.IPR_EARG
    assert rc(p=(ct.c_int * 2)(0, 2)) == ipr.IPR_EARG and rc(p=(ct.c_int * 2)(2, 9)) == ipr.IPR_EARG
    assert rc(o=(ct.c_int64 * 2)(0, -1)) == ipr.IPR_EARG
    assert "item 1" in ipr.ipr_last_error()


def test_one_scale_rule_at_a_time():
    assert solve_rc(scale_squarings=6, scale_lanczos=1) == ipr.IPR_EARG
    assert "choose one" in ipr.ipr_last_error()
    assert solve_rc(store_format=ipr.IPR_STORE_FLOAT, store_bits=10,
                    scale_lanczos=1) == ipr.IPR_EARG
