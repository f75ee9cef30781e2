"""CPU-only checks of the C ABI: the library loads, exports every declared
entry point, and validates descriptors on the host (before any GPU call),
returning the documented status and writing nothing.  Shape bookkeeping of
the queries is compared with the oracle's constructions."""
import ctypes
import os
import re
from ctypes import byref, c_int32, c_int64, c_size_t, c_void_p

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttc.h")
LIB = os.path.join(ROOT, "paper_2109_00626_amd", "libttc.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2109_00626_amd import build
        build.build(verbose=False)
    from paper_2109_00626_amd import _abi
    return _abi.load(LIB)


@pytest.fixture(scope="module")
def abi():
    from paper_2109_00626_amd import _abi
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^(?:ttc_status|const char\*|int32_t|void)\s+(\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol(lib, abi):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.EXPORTED)
    assert lib.ttc_abi_version() == 2
    assert b"gfx950" in lib.ttc_version()


FAKE = 0x7F0000001000  # never dereferenced: validation fails or only queries run


class Desc:
    def __init__(self, abi, modes, ranks, dtype=1):
        self.m = (c_int32 * len(modes))(*modes)
        self.r = (c_int32 * len(ranks))(*ranks)
        self.c = (c_void_p * len(modes))(*[FAKE + 4096 * k for k in range(len(modes))])
        self.s = abi.TT(len(modes), self.m, self.r, dtype, self.c)


def status_name(abi, s):
    return abi.STATUS_NAMES[s]


def test_inner_validation(lib, abi):
    need = c_size_t(0)
    x = Desc(abi, [3, 4], [1, 2, 1])
    y = Desc(abi, [3, 4], [1, 5, 1])
    assert lib.tt_contract_inner_query(byref(x.s), byref(y.s), 0, byref(need)) == 0
    assert need.value == 0  # FP32, ranks <= 128, order < 4: one LDS-resident sweep, no workspace
    x4 = Desc(abi, [3, 4, 5, 6], [1, 2, 7, 3, 1])
    y4 = Desc(abi, [3, 4, 5, 6], [1, 5, 9, 2, 1])
    assert lib.tt_contract_inner_query(byref(x4.s), byref(y4.s), 0, byref(need)) == 0
    # order 4: two LDS sweeps meeting at bond 2; W_2 and V_2 (7 x 9 FP32 each)
    # plus the reversed prefix cores (3*2 + 2*4*7 and 3*5 + 5*4*9 FP32)
    assert need.value >= 4 * (2 * 7 * 9 + 6 + 56 + 15 + 180)
    x64 = Desc(abi, [3, 4], [1, 2, 1], dtype=0)
    y64 = Desc(abi, [3, 4], [1, 5, 1], dtype=0)
    assert lib.tt_contract_inner_query(byref(x64.s), byref(y64.s), 0, byref(need)) == 0
    assert need.value > 0   # FP64: the two-half sweep with its interface buffers
    xb = Desc(abi, [3, 4], [1, 200, 1])
    yb = Desc(abi, [3, 4], [1, 150, 1])
    assert lib.tt_contract_inner_query(byref(xb.s), byref(yb.s), 0, byref(need)) == 0
    assert need.value > 0   # ranks above 128 take the same path
    bad = Desc(abi, [3, 4], [2, 2, 1])
    assert status_name(abi, lib.tt_contract_inner_query(byref(bad.s), byref(y.s), 0, byref(need))) == "TTC_ERR_RANK"
    assert b"boundary" in lib.ttc_last_error()
    other = Desc(abi, [3, 5], [1, 2, 1])
    assert status_name(abi, lib.tt_contract_inner_query(byref(x.s), byref(other.s), 0, byref(need))) == "TTC_ERR_SHAPE"
    d64 = Desc(abi, [3, 4], [1, 2, 1], dtype=0)
    assert status_name(abi, lib.tt_contract_inner_query(byref(x.s), byref(d64.s), 0, byref(need))) == "TTC_ERR_DTYPE"
    assert status_name(abi, lib.tt_contract_inner_query(None, byref(y.s), 0, byref(need))) == "TTC_ERR_NULL"
    assert status_name(abi, lib.tt_contract_inner_query(byref(x.s), byref(y.s), 1, byref(need))) == "TTC_ERR_UNSUPPORTED"
    # BF16 precision: BF16 cores with every rank <= 128 only
    assert status_name(abi, lib.tt_contract_inner_query(byref(x.s), byref(y.s), 3, byref(need))) == "TTC_ERR_UNSUPPORTED"
    xh, yh = Desc(abi, [3, 4], [1, 2, 1], dtype=2), Desc(abi, [3, 4], [1, 5, 1], dtype=2)
    assert lib.tt_contract_inner_query(byref(xh.s), byref(yh.s), 3, byref(need)) == abi.TTC_OK
    xhb, yhb = Desc(abi, [3, 4], [1, 200, 1], dtype=2), Desc(abi, [3, 4], [1, 5, 1], dtype=2)
    assert status_name(abi, lib.tt_contract_inner_query(byref(xhb.s), byref(yhb.s), 3, byref(need))) == \
        "TTC_ERR_UNSUPPORTED"
    # workspace too small and NULL output: rejected before any launch
    out = c_void_p(FAKE)
    assert status_name(abi, lib.tt_contract_inner(byref(x64.s), byref(y64.s), 0, out, c_void_p(FAKE), 1, None)) == \
        "TTC_ERR_WORKSPACE"
    assert status_name(abi, lib.tt_contract_inner(byref(x.s), byref(y.s), 0, None, c_void_p(FAKE), 1 << 30, None)) == \
        "TTC_ERR_NULL"
    zero = Desc(abi, [3, 0], [1, 2, 1])
    assert status_name(abi, lib.tt_contract_inner_query(byref(zero.s), byref(y.s), 0, byref(need))) == "TTC_ERR_SHAPE"


def _modes_query(lib, abi, x, y, modes, form, prec=0):
    m = (c_int32 * len(modes))(*modes)
    order = c_int32(0)
    om = (c_int32 * 64)()
    orr = (c_int32 * 65)()
    el = c_int64(0)
    ws = c_size_t(0)
    st = lib.tt_contract_modes_query(byref(x.s), byref(y.s), m, len(modes), form, prec, byref(order), om, orr,
                                     byref(el), byref(ws))
    return st, order.value, list(om[:order.value]), list(orr[:order.value + 1]), el.value


@pytest.mark.parametrize("which", ["pair10", "inner4"])
def test_modes_query_matches_oracle_shapes(lib, abi, which):
    if which == "pair10":
        sx, sy = C.pair10_shapes()
        modes = [0, 1, 2, 3, 4]
    else:
        sx, sy = C.inner4_shapes()
        modes = [2, 3]
    x = Desc(abi, sx.modes, sx.ranks)
    y = Desc(abi, sy.modes, sy.ranks)
    st, order, om, orr, el = _modes_query(lib, abi, x, y, modes, abi.FORM["natural"])
    assert st == 0
    xs = [np.zeros(sx.core_shape(k)) for k in range(sx.order)]
    ys = [np.zeros(sy.core_shape(k)) for k in range(sy.order)]
    want = O.contract_natural(xs, ys, modes)
    assert om == O.tt_modes(want)
    assert orr == O.tt_ranks(want)
    assert el == sum(G.size for G in want)
    st, order, om, orr, el = _modes_query(lib, abi, x, y, modes, abi.FORM["dense"])
    assert st == 0 and el == int(np.prod(O.tt_modes(want)))


def test_modes_query_errors(lib, abi):
    x = Desc(abi, [3, 4, 5], [1, 2, 2, 1])
    y = Desc(abi, [3, 4, 5], [1, 3, 3, 1])
    assert status_name(abi, _modes_query(lib, abi, x, y, [1], 0)[0]) == "TTC_ERR_UNSUPPORTED"
    assert status_name(abi, _modes_query(lib, abi, x, y, [0, 0], 0)[0]) == "TTC_ERR_MODE"
    assert status_name(abi, _modes_query(lib, abi, x, y, [3], 0)[0]) == "TTC_ERR_MODE"
    st, order, _, orr, el = _modes_query(lib, abi, x, y, [2, 1], 0)
    assert st == 0 and order == 2 and orr[:2] == [2, 3] and el == 6   # suffix K = V_1 (R_1 x P_1)
    st, order, _, _, el = _modes_query(lib, abi, x, y, [0, 1, 2], 1)
    assert st == 0 and order == 0 and el == 1


def test_mpo_query(lib, abi):
    sw, sv = C.mpo8_shapes()
    rows = (c_int32 * 8)(*sw.modes)
    cols = (c_int32 * 8)(*sw.cols)
    rk = (c_int32 * 9)(*sw.ranks)
    cores = (c_void_p * 8)(*[FAKE] * 8)
    m = abi.TTM(8, rows, cols, rk, 2, cores)
    v = Desc(abi, sv.modes, sv.ranks, dtype=2)
    orr = (c_int32 * 9)()
    el = c_int64(0)
    assert lib.ttm_apply_query(byref(m), byref(v.s), orr, byref(el)) == 0
    assert list(orr) == [1] + [1024] * 7 + [1]
    assert el.value == 2 * 32 * 1024 + 6 * 1024 * 32 * 1024
    v2 = Desc(abi, [32] * 7 + [16], sv.ranks, dtype=2)
    assert status_name(abi, lib.ttm_apply_query(byref(m), byref(v2.s), orr, byref(el))) == "TTC_ERR_SHAPE"


def test_mode_n_validation(lib, abi):
    x = Desc(abi, [3, 4], [1, 2, 1])
    y = Desc(abi, [3, 6], [1, 2, 1])
    A = (c_void_p * 1)(FAKE)
    J = (c_int32 * 1)(5)
    m = (c_int32 * 1)(1)
    assert status_name(abi, lib.tt_mode_n_product(byref(x.s), 1, m, A, J, byref(y.s), None)) == "TTC_ERR_SHAPE"
    m2 = (c_int32 * 1)(2)
    assert status_name(abi, lib.tt_mode_n_product(byref(x.s), 1, m2, A, J, byref(y.s), None)) == "TTC_ERR_MODE"


def test_grad_query(lib, abi):
    sx, sy = C.pair10_shapes()
    x = Desc(abi, sx.modes, sx.ranks)
    y = Desc(abi, sy.modes, sy.ranks)
    a, b = c_size_t(0), c_size_t(0)
    assert lib.tt_contract_inner_bwd_query(byref(x.s), byref(y.s), 1, byref(a)) == 0
    assert lib.tt_contract_inner_bwd_query(byref(x.s), byref(y.s), 4, byref(b)) == 0
    assert a.value > 0 and b.value > 0


def test_layer_schedule_queries(lib, abi):
    """Every layer schedule is accepted; AUTO takes the one with fewer FLOPs
    (the dense one for the 4096 x 4096 order-4 layer); the core-by-core
    backward keeps its three 8192 * 512 * 256 intermediates and two gradient
    buffers; the saving schedule's forward asks for the backward's
    workspace; an unknown schedule is refused."""
    s = C.layer4_shape()
    rows = (c_int32 * 4)(*s.modes)
    cols = (c_int32 * 4)(*s.cols)
    rk = (c_int32 * 5)(*s.ranks)
    cores = (c_void_p * 4)(*[FAKE] * 4)
    m = abi.TTM(4, rows, cols, rk, 1, cores)
    ws = {}
    for name in ("auto", "dense", "cores", "cores_saved"):
        for bwd in (0, 1):
            b = c_size_t(0)
            assert lib.ttm_apply_dense_query(byref(m), 8192, abi.PREC["f32"], abi.SCHED[name], bwd, byref(b)) == 0
            ws[name, bwd] = b.value
    assert ws["auto", 0] == ws["dense", 0] and ws["auto", 1] == ws["dense", 1]
    inter = 8192 * 512 * 8 * 32 * 4   # bytes of one intermediate
    assert ws["cores", 1] >= 3 * inter + 2 * inter
    assert 2 * inter <= ws["cores", 0] < 3 * inter
    assert ws["cores_saved", 0] == ws["cores_saved", 1] == ws["cores", 1]
    b = c_size_t(0)
    assert status_name(abi, lib.ttm_apply_dense_query(byref(m), 8192, abi.PREC["f32"], 4, 0, byref(b))) == \
        "TTC_ERR_UNSUPPORTED"


def test_svd_query_caps_and_errors(lib, abi):
    dims = (c_int32 * 5)(20, 20, 20, 5, 4)
    cap = (c_int32 * 6)()
    need = c_size_t(0)
    assert lib.tt_svd_query(5, dims, 0, 0, cap, byref(need)) == abi.TTC_OK
    # bond k can hold at most min(prod of modes left of it, prod right of it)
    assert list(cap) == [1, 20, 400, 20, 4, 1]
    assert need.value >= 3 * 160000 * 8 + 400 * 400 * 8
    assert lib.tt_svd_query(5, dims, 0, 7, cap, byref(need)) == abi.TTC_OK
    assert list(cap) == [1, 7, 7, 7, 4, 1]
    assert status_name(abi, lib.tt_svd_query(5, dims, 2, 0, cap, byref(need))) == "TTC_ERR_DTYPE"
    big = (c_int32 * 2)(5000, 5000)
    assert status_name(abi, lib.tt_svd_query(2, big, 0, 0, cap, byref(need))) == "TTC_ERR_UNSUPPORTED"
    zero = (c_int32 * 2)(3, 0)
    assert status_name(abi, lib.tt_svd_query(2, zero, 0, 0, cap, byref(need))) == "TTC_ERR_SHAPE"
    ranks = (c_int32 * 6)()
    cores = (c_void_p * 5)(*[FAKE] * 5)
    # validation happens before anything touches a pointer
    assert status_name(abi, lib.tt_svd(None, 5, dims, 0, 0.0, 0, ranks, cores, c_void_p(FAKE), 1 << 40,
                                       None)) == "TTC_ERR_NULL"
    assert status_name(abi, lib.tt_svd(c_void_p(FAKE), 5, dims, 0, -1.0, 0, ranks, cores, c_void_p(FAKE), 1 << 40,
                                       None)) == "TTC_ERR_SHAPE"
    assert status_name(abi, lib.tt_svd(c_void_p(FAKE), 5, dims, 0, 0.0, 0, ranks, cores, c_void_p(FAKE), 16,
                                       None)) == "TTC_ERR_WORKSPACE"


def test_pairs_query_matches_oracle_shapes(lib, abi):
    """The natural-form shapes the library reports for every block layout
    equal those of the oracle's construction; the junction is
    (R_a P_g) x (R_b P_d)."""
    from test_gpu_pairs import CASES
    for mx, rx, my, ry, xm, ym in CASES:
        dx, dy = Desc(abi, mx, rx, 0), Desc(abi, my, ry, 0)
        n = len(mx) + len(my)
        order, om, orr = c_int32(0), (c_int32 * n)(), (c_int32 * (n + 1))()
        elems, need = c_int64(0), c_size_t(0)
        xa, ya = (c_int32 * len(xm))(*xm), (c_int32 * len(ym))(*ym)
        assert lib.tt_contract_pairs_query(byref(dx.s), byref(dy.s), xa, ya, len(xm), 1, byref(order), om, orr,
                                           byref(elems), byref(need)) == abi.TTC_OK
        x = C.gen_tt_np(1, 1, C.TTShape(mx, rx))
        y = C.gen_tt_np(1, 2, C.TTShape(my, ry))
        want = O.contract_pairs_natural(x, y, xm, ym)
        k = order.value
        assert k == len(want)
        assert list(om[:k]) == [w.shape[1] for w in want]
        assert list(orr[:k + 1]) == [w.shape[0] for w in want] + [1]
        assert elems.value == sum(w.size for w in want)
        assert lib.tt_contract_pairs_query(byref(dx.s), byref(dy.s), xa, ya, len(xm), 0, byref(order), om, orr,
                                           byref(elems), byref(need)) == abi.TTC_OK
        T = O.transfer_junction(x, y, xm, ym)
        assert (order.value, orr[0], orr[1]) == (2, T.shape[0], T.shape[1])


def _pairs_array(abi, shapes, dtype=1):
    descs = [(Desc(abi, sx.modes, sx.ranks, dtype), Desc(abi, sy.modes, sy.ranks, dtype)) for sx, sy in shapes]
    arr = (abi.Pair * len(shapes))(*[abi.Pair(dx.s, dy.s) for dx, dy in descs])
    return arr, descs


def test_batch_plan_query_against_rederivation(lib, abi):
    """The batch planner's host bookkeeping on 300 pairs of the uneven
    workload's distribution, re-derived here: junction offsets, algorithmic
    FLOPs (the cheaper order of each right-to-left step) and bytes, and the
    claim order (decreasing modelled cost, ties by index)."""
    shapes = C.batch_pair_shapes(C.SEED_BATCH, 300)
    arr, keep = _pairs_array(abi, shapes)
    n = len(shapes)
    joff, cost, order = (c_int64 * (n + 1))(), (ctypes.c_double * n)(), (c_int32 * n)()
    fl, by = ctypes.c_double(0), ctypes.c_double(0)
    assert lib.tt_batch_plan_query(arr, n, 3, joff, byref(fl), byref(by), cost, order) == abi.TTC_OK
    want_off, want_fl, want_by = [0], 0.0, 0.0
    for sx, sy in shapes:
        N, I, R, P = sx.order, sx.modes, sx.ranks, sy.ranks
        want_off.append(want_off[-1] + R[N - 2] * P[N - 2])
        for k in range(1, N):
            a = 2 * I[k] * R[k] * P[k + 1] * (R[k + 1] + P[k])
            b = 2 * I[k] * R[k + 1] * P[k] * (P[k + 1] + R[k])
            want_fl += min(a, b)
        want_fl += 2 * I[0] * R[1] * P[1] + 2 * R[1] * P[1]
        want_by += 4 * sum(R[k] * I[k] * R[k + 1] + P[k] * I[k] * P[k + 1] for k in range(N)) + 8
        want_by += 4 * R[N - 2] * P[N - 2]
    assert list(joff) == want_off
    assert fl.value == pytest.approx(want_fl, rel=1e-12)
    assert by.value == pytest.approx(want_by, rel=1e-12)
    c = np.array(list(cost))
    assert np.all(c > 0)
    assert list(order) == list(np.argsort(-c, kind="stable"))
    # a pair's modelled cost grows with its ranks and its order
    sx, sy = C.TTShape([16] * 6, [1] + [32] * 5 + [1]), C.TTShape([16] * 6, [1] + [32] * 5 + [1])
    sx2, sy2 = C.TTShape([16] * 6, [1] + [64] * 5 + [1]), C.TTShape([16] * 6, [1] + [64] * 5 + [1])
    sx3, sy3 = C.TTShape([16] * 9, [1] + [32] * 8 + [1]), C.TTShape([16] * 9, [1] + [32] * 8 + [1])
    arr, keep = _pairs_array(abi, [(sx, sy), (sx2, sy2), (sx3, sy3)])
    cost3 = (ctypes.c_double * 3)()
    assert lib.tt_batch_plan_query(arr, 3, 3, None, None, None, cost3, None) == abi.TTC_OK
    assert cost3[1] > cost3[0] and cost3[2] > cost3[0]


def test_batch_plan_query_errors(lib, abi):
    ok = (C.TTShape([4, 5, 6], [1, 3, 2, 1]), C.TTShape([4, 5, 6], [1, 2, 2, 1]))
    cases = [
        ([ok], 0, "TTC_ERR_UNSUPPORTED"),                                                  # no ops
        ([(C.TTShape([4, 5, 6], [1, 200, 2, 1]), ok[1])], 3, "TTC_ERR_UNSUPPORTED"),       # rank > 128
        ([(ok[0], C.TTShape([4, 5, 7], [1, 2, 2, 1]))], 3, "TTC_ERR_SHAPE"),               # modes differ
        ([(C.TTShape([4, 5], [1, 3, 1]), C.TTShape([4, 5], [1, 2, 1]))], 3, "TTC_ERR_SHAPE"),  # SUFFIX2 at order 2
        ([(ok[0], C.TTShape([4, 5, 6], [1, 2, 2, 2]))], 3, "TTC_ERR_RANK"),                # boundary rank
    ]
    for shapes, ops, want in cases:
        arr, keep = _pairs_array(abi, shapes)
        assert status_name(abi, lib.tt_batch_plan_query(arr, len(shapes), ops, None, None, None, None, None)) == want
    # order 2 is fine for the inner product alone
    arr, keep = _pairs_array(abi, [(C.TTShape([4, 5], [1, 3, 1]), C.TTShape([4, 5], [1, 2, 1]))])
    assert lib.tt_batch_plan_query(arr, 1, 1, None, None, None, None, None) == abi.TTC_OK
    # one dtype per batch
    dx, dy = Desc(abi, [4, 5, 6], [1, 3, 2, 1], 1), Desc(abi, [4, 5, 6], [1, 2, 2, 1], 1)
    ex, ey = Desc(abi, [4, 5, 6], [1, 3, 2, 1], 2), Desc(abi, [4, 5, 6], [1, 2, 2, 1], 2)
    arr = (abi.Pair * 2)(abi.Pair(dx.s, dy.s), abi.Pair(ex.s, ey.s))
    assert status_name(abi, lib.tt_batch_plan_query(arr, 2, 3, None, None, None, None, None)) == "TTC_ERR_DTYPE"
    # plan precision: BF16 needs BF16 cores, FP64 is not a batched precision
    # (both refused before any device call)
    arr = (abi.Pair * 1)(abi.Pair(dx.s, dy.s))
    h = c_void_p(0)
    assert status_name(abi, lib.tt_batch_plan_create(arr, 1, 3, abi.PREC["bf16"], byref(h))) == "TTC_ERR_UNSUPPORTED"
    assert status_name(abi, lib.tt_batch_plan_create(arr, 1, 3, abi.PREC["f64"], byref(h))) == "TTC_ERR_UNSUPPORTED"
    assert not h.value
