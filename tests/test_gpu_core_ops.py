"""GPU parity of the single-pair operations against the FP64 oracle, called
through the C ABI: inner products, shared-block contractions (junction,
natural and dense forms), mode-n products, MPO x TT, and the inner-product
gradient.  Tolerances: FP64 1e-12, FP32 1e-5, BF16 inputs 2e-2 (relative,
measured as documented in helpers)."""
import math

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

from helpers import TOL, max_core_rel, random_pair, rel_err, scalar_err, to_gpu, to_np, tt_norm

pytestmark = pytest.mark.gpu


def _inner_case(ttc, x, y, dtype):
    xg, xs = to_gpu(x, dtype)
    yg, ys = to_gpu(y, dtype)
    z = float(ttc.tt_contract_inner(xg, yg).item())
    # arithmetic error: oracle on the values the GPU holds
    zr = O.inner_lr(xs, ys)
    e = scalar_err(z, zr, tt_norm(xs), tt_norm(ys))
    # total error: oracle on the unrounded FP64 inputs
    et = scalar_err(z, O.inner_lr(x, y), tt_norm(x), tt_norm(y))
    return e, et


# ------------------------------------------------------------------ inner
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_inner_inner4(ttc, dtype):
    sx, sy = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    y = C.gen_tt_np(C.SEED_INNER4, 2, sy)
    e, et = _inner_case(ttc, x, y, dtype)
    print(f"inner4 {dtype}: arithmetic {e:.3e} total {et:.3e}")
    assert (et if dtype == "bf16" else e) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_inner_pair10(ttc, dtype):
    sx, sy = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    y = C.gen_tt_np(C.SEED_PAIR10, 2, sy)
    e, et = _inner_case(ttc, x, y, dtype)
    print(f"pair10 {dtype}: arithmetic {e:.3e} total {et:.3e}")
    assert (et if dtype == "bf16" else e) <= TOL[dtype]


@pytest.mark.parametrize("case", [
    ([3, 5, 2, 7, 4], [1, 3, 17, 5, 2, 1], [1, 9, 2, 33, 6, 1]),          # ragged ranks
    ([64, 4], [1, 70, 1], [1, 37, 1]),                                      # several tiles, ragged tail
    ([5], [1, 1], [1, 1]),                                                  # order 1
    ([6, 9], [1, 7, 1], [1, 12, 1]),                                        # order 2
    ([16, 32, 8], [1, 128, 100, 1], [1, 90, 128, 1]),                       # large ranks
    ([2, 3, 2, 3, 2, 3, 2], [1, 2, 3, 4, 5, 4, 3, 1], [1, 1, 2, 1, 2, 1, 2, 1]),
    ([8, 4, 16, 4, 8, 4], [1, 64, 128, 96, 128, 50, 1], [1, 100, 128, 77, 128, 33, 1]),  # two halves, wide middle bond
])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_inner_ragged(ttc, case, dtype):
    modes, rx, ry = case
    x, y = random_pair(77, modes, rx, ry)
    e, et = _inner_case(ttc, x, y, dtype)
    # BF16 cores: the single-pair sweeps compute in FP32, so the error on
    # the rounded values meets the FP32 bound; the total error the BF16 one
    assert e <= (TOL["f32"] if dtype == "bf16" else TOL[dtype])
    assert et <= TOL[dtype]


# The BF16-MFMA steps carry the interface and each per-index product as a
# BF16 hi / lo pair (about 16 significant bits), so each step adds about
# 2^-17 relative to the arithmetic error; 1e-4 leaves a wide margin for the
# at most ten steps below.
ARITH_BF16_MFMA = 1e-4


@pytest.mark.parametrize("case", [
    ([3, 5, 2, 7, 4], [1, 3, 17, 5, 2, 1], [1, 9, 2, 33, 6, 1]),          # two halves, ragged ranks
    ([6, 9], [1, 7, 1], [1, 12, 1]),                                        # one sweep
    ([16, 32, 8], [1, 128, 100, 1], [1, 90, 128, 1]),                       # large ranks
    ([8, 4, 16, 4, 8, 4], [1, 64, 128, 96, 128, 50, 1], [1, 100, 128, 77, 128, 33, 1]),
])
def test_inner_bf16_mfma(ttc, case):
    """prec BF16 on BF16 cores: the steps on BF16 MFMA, against the oracle on
    the unrounded inputs (the BF16 bound) and on the values the GPU holds
    (the arithmetic bound above); also the order-10 rank-32 pair."""
    modes, rx, ry = case
    x, y = random_pair(78, modes, rx, ry)
    for xx, yy in ((x, y), (C.gen_tt_np(C.SEED_PAIR10, 1, C.pair10_shapes()[0]),
                            C.gen_tt_np(C.SEED_PAIR10, 2, C.pair10_shapes()[1]))):
        xg, xs = to_gpu(xx, "bf16")
        yg, ys = to_gpu(yy, "bf16")
        z = float(ttc.tt_contract_inner(xg, yg, prec="bf16").item())
        assert scalar_err(z, O.inner_lr(xs, ys), tt_norm(xs), tt_norm(ys)) <= ARITH_BF16_MFMA
        assert scalar_err(z, O.inner_lr(xx, yy), tt_norm(xx), tt_norm(yy)) <= TOL["bf16"]


def test_inner_bf16_prec_refusals(ttc):
    x, y = random_pair(79, [4, 5, 3], [1, 3, 4, 1], [1, 2, 5, 1])
    xf, _ = to_gpu(x, "f32")
    yf, _ = to_gpu(y, "f32")
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_inner(xf, yf, prec="bf16")
    assert ei.value.name == "TTC_ERR_UNSUPPORTED"
    xw, yw = random_pair(79, [4, 5], [1, 130, 1], [1, 3, 1])
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_inner(to_gpu(xw, "bf16")[0], to_gpu(yw, "bf16")[0], prec="bf16")
    assert ei.value.name == "TTC_ERR_UNSUPPORTED"


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_inner_integer_cores_bit_exact(ttc, dtype):
    s = C.TTShape([4, 8, 3, 5, 6], [1, 5, 7, 3, 4, 1])
    x = C.gen_int_tt_np(31, 1, s)
    y = C.gen_int_tt_np(31, 2, s)
    want = O.inner_lr(x, y)  # exact: integer partial sums well below 2^24
    xg, _ = to_gpu(x, dtype)
    yg, _ = to_gpu(y, dtype)
    z = float(ttc.tt_contract_inner(xg, yg).item())
    assert z == want


def test_inner_deterministic(ttc):
    sx, sy = C.pair10_shapes()
    xg, _ = to_gpu(C.gen_tt_np(C.SEED_PAIR10, 1, sx), "f32")
    yg, _ = to_gpu(C.gen_tt_np(C.SEED_PAIR10, 2, sy), "f32")
    a = ttc.tt_contract_inner(xg, yg).item()
    b = ttc.tt_contract_inner(xg, yg).item()
    assert a == b


def test_inner_from_host_threads(ttc):
    """Four host threads, each on its own stream with its own inputs and
    workspace, call the inner product at the same time (FP64 chained sweeps,
    FP32 and BF16 two-half LDS sweeps, an FP32 single sweep below order 4).
    Every result equals the same call made alone, bit for bit, and the FP64
    oracle within the dtype's tolerance."""
    import threading

    import torch

    cases = [("f64", [6, 4, 8, 5, 3], [1, 9, 17, 12, 4, 1], [1, 5, 33, 8, 6, 1]),
             ("f32", [8, 4, 16, 4, 8, 4], [1, 64, 128, 96, 128, 50, 1], [1, 100, 128, 77, 128, 33, 1]),
             ("bf16", [16, 8, 4, 8, 16], [1, 16, 70, 33, 16, 1], [1, 16, 40, 65, 12, 1]),
             ("f32", [32, 64, 16], [1, 32, 100, 1], [1, 20, 128, 1])]
    inputs, alone = [], []
    for n, (dtype, modes, rx, ry) in enumerate(cases):
        x, y = random_pair(500 + n, modes, rx, ry)
        xg, xs = to_gpu(x, dtype)
        yg, ys = to_gpu(y, dtype)
        z = float(ttc.tt_contract_inner(xg, yg).item())
        assert scalar_err(z, O.inner_lr(xs, ys), tt_norm(xs), tt_norm(ys)) <= (TOL["f32"] if dtype == "bf16" else TOL[dtype])
        inputs.append((xg, yg))
        alone.append(z)
    torch.cuda.synchronize()
    reps = 25
    got = [None] * len(cases)
    errors = []
    start = threading.Barrier(len(cases))

    def work(n):
        try:
            s = torch.cuda.Stream()
            xg, yg = inputs[n]
            start.wait()
            with torch.cuda.stream(s):
                outs = [ttc.tt_contract_inner(xg, yg) for _ in range(reps)]
            s.synchronize()
            got[n] = [float(o.item()) for o in outs]
        except Exception as exc:  # re-raised in the main thread
            errors.append(exc)

    threads = [threading.Thread(target=work, args=(n,)) for n in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    if errors:
        raise errors[0]
    for n in range(len(cases)):
        assert got[n] == [alone[n]] * reps, (cases[n][0], n)


# ------------------------------------------------------------------ modes
def test_modes_inner4_all_forms(ttc):
    sx, sy = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    y = C.gen_tt_np(C.SEED_INNER4, 2, sy)
    xg, _ = to_gpu(x, "f64")
    yg, _ = to_gpu(y, "f64")
    modes = [2, 3]  # the paper's modes 3-4
    K = to_np(ttc.tt_contract_modes(xg, yg, modes, "junction"))
    assert rel_err(K, O.contract_junction(x, y, modes)[2]) <= TOL["f64"]
    nat = [to_np(t) for t in ttc.tt_contract_modes(xg, yg, modes, "natural")]
    want = O.contract_natural(x, y, modes)
    assert [G.shape for G in nat] == [G.shape for G in want]
    assert max_core_rel(nat, want) <= TOL["f64"]
    Z = to_np(ttc.tt_contract_modes(xg, yg, modes, "dense"))
    assert Z.shape == (8, 8, 8, 8)
    assert rel_err(Z, O.contract_dense(x, y, modes)) <= TOL["f64"]
    z = ttc.tt_contract_modes(xg, yg, [3, 1, 0, 2], "natural").item()
    assert scalar_err(z, O.inner_lr(x, y), tt_norm(x), tt_norm(y)) <= TOL["f64"]


@pytest.mark.parametrize("modes", [[0], [0, 1], [0, 1, 2], [3], [1, 2, 3], [2, 3]])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_modes_ragged_prefix_suffix(ttc, modes, dtype):
    x, y = random_pair(91, [3, 5, 2, 4], [1, 3, 6, 2, 1], [1, 2, 5, 7, 1])
    xg, xs = to_gpu(x, dtype)
    yg, ys = to_gpu(y, dtype)
    ref = (x, y) if dtype == "bf16" else (xs, ys)
    tol = TOL[dtype]
    K = to_np(ttc.tt_contract_modes(xg, yg, modes, "junction"))
    assert rel_err(K, O.contract_junction(*ref, modes)[2]) <= tol
    nat = [to_np(t) for t in ttc.tt_contract_modes(xg, yg, modes, "natural")]
    assert max_core_rel(nat, O.contract_natural(*ref, modes)) <= tol
    Z = to_np(ttc.tt_contract_modes(xg, yg, modes, "dense"))
    assert rel_err(Z, O.contract_dense(*ref, modes)) <= tol


@pytest.mark.parametrize("modes", [[0], [0, 1, 2], [3], [1, 2, 3], [0, 1, 2, 3]])
def test_modes_bf16_mfma(ttc, modes):
    """prec BF16 on BF16 cores: the junction sweep on BF16 MFMA, every form,
    against the oracle on the unrounded inputs (BF16 bound) and on the
    values the GPU holds (the BF16-MFMA arithmetic bound)."""
    x, y = random_pair(92, [3, 5, 2, 4], [1, 3, 6, 2, 1], [1, 2, 5, 7, 1])
    xg, xs = to_gpu(x, "bf16")
    yg, ys = to_gpu(y, "bf16")
    if len(modes) == 4:
        z = ttc.tt_contract_modes(xg, yg, modes, "junction", prec="bf16").item()
        assert scalar_err(z, O.inner_lr(xs, ys), tt_norm(xs), tt_norm(ys)) <= ARITH_BF16_MFMA
        return
    for ref, tol in (((x, y), TOL["bf16"]), ((xs, ys), ARITH_BF16_MFMA)):
        K = to_np(ttc.tt_contract_modes(xg, yg, modes, "junction", prec="bf16"))
        assert rel_err(K, O.contract_junction(*ref, modes)[2]) <= tol
        nat = [to_np(t) for t in ttc.tt_contract_modes(xg, yg, modes, "natural", prec="bf16")]
        assert max_core_rel(nat, O.contract_natural(*ref, modes)) <= tol
        Z = to_np(ttc.tt_contract_modes(xg, yg, modes, "dense", prec="bf16"))
        assert rel_err(Z, O.contract_dense(*ref, modes)) <= tol


@pytest.mark.parametrize("modes", [[0], [1], [0, 1]])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_modes_order2(ttc, modes, dtype):
    """Order-2 pairs: a one-core prefix, a one-core suffix and both modes, in
    the junction, natural and dense forms."""
    x, y = random_pair(93, [5, 7], [1, 4, 1], [1, 6, 1])
    xg, xs = to_gpu(x, dtype)
    yg, ys = to_gpu(y, dtype)
    tol = TOL[dtype]
    if modes != [0, 1]:
        K = to_np(ttc.tt_contract_modes(xg, yg, modes, "junction"))
        assert rel_err(K, O.contract_junction(xs, ys, modes)[2]) <= tol
    nat = ttc.tt_contract_modes(xg, yg, modes, "natural")
    if modes == [0, 1]:
        assert scalar_err(nat.item(), O.inner_lr(xs, ys), tt_norm(xs), tt_norm(ys)) <= tol
    else:
        assert max_core_rel([to_np(t) for t in nat], O.contract_natural(xs, ys, modes)) <= tol
        Z = to_np(ttc.tt_contract_modes(xg, yg, modes, "dense"))
        assert rel_err(Z, O.contract_dense(xs, ys, modes)) <= tol


def test_modes_pair10_prefix5(ttc):
    """Modes 1-5 of the order-10 pair: junction, then the natural TT with
    ranks 32*32 at full size, checked core by core."""
    sx, sy = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    y = C.gen_tt_np(C.SEED_PAIR10, 2, sy)
    xg, xs = to_gpu(x, "f32")
    yg, ys = to_gpu(y, "f32")
    modes = [0, 1, 2, 3, 4]
    K = to_np(ttc.tt_contract_modes(xg, yg, modes, "junction"))
    Kr = O.contract_junction(xs, ys, modes)[2]
    assert rel_err(K, Kr) <= TOL["f32"]
    nat = ttc.tt_contract_modes(xg, yg, modes, "natural")
    want = O.contract_natural(xs, ys, modes)
    assert [tuple(t.shape) for t in nat] == [G.shape for G in want]
    assert [int(t.shape[0]) for t in nat] + [1] == [1, 1024, 1024, 1024, 1024, 32, 32, 32, 32, 32, 1]
    for t, w in zip(nat, want):
        assert rel_err(to_np(t), w) <= TOL["f32"]


def test_modes_unsupported_and_errors(ttc):
    x, y = random_pair(5, [3, 4, 5], [1, 2, 2, 1], [1, 2, 2, 1])
    xg, _ = to_gpu(x, "f32")
    yg, _ = to_gpu(y, "f32")
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_modes(xg, yg, [1], "junction")  # middle position
    assert ei.value.name == "TTC_ERR_UNSUPPORTED"
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_modes(xg, yg, [0, 0], "junction")
    assert ei.value.name == "TTC_ERR_MODE"


# ------------------------------------------------------------------ mode-n
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_mode_n_inner4(ttc, dtype):
    sx, _ = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    A = C.gen_matrix_np(C.SEED_INNER4, 3, 8, 8)
    xg, xs = to_gpu(x, dtype)
    Ag, As = to_gpu([A], dtype)
    out = ttc.tt_mode_n_product(xg, [1], Ag)  # the paper's mode 2
    assert out[0] is xg[0] and out[2] is xg[2]
    want = O.mode_n_tt(xs, 1, As[0])
    got = to_np(out[1])
    if dtype == "bf16":
        # output rounded to BF16: compare with the FP64 product on the unrounded inputs
        assert rel_err(got, O.mode_n_tt(x, 1, A)[1]) <= TOL["bf16"]
    else:
        assert rel_err(got, want[1]) <= TOL[dtype]
    # dense check against Def. 5 on the reconstructed tensor
    if dtype == "f64":
        full = O.tt_full([to_np(t) for t in out])
        assert rel_err(full, O.mode_n_product(O.tt_full(x), A, 1)) <= 1e-12


def test_mode_n_pair10_every_mode(ttc):
    sx, _ = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    mats = [C.gen_matrix_np(C.SEED_PAIR10, 3 + n, 16, 16) for n in range(10)]
    xg, xs = to_gpu(x, "f32")
    Ag, As = to_gpu(mats, "f32")
    out = ttc.tt_mode_n_product(xg, list(range(10)), Ag)
    want = xs
    for n in range(10):
        want = O.mode_n_tt(want, n, As[n])
    assert max_core_rel([to_np(t) for t in out], want) <= TOL["f32"]


def test_mode_n_identity_and_rectangular(ttc):
    x, _ = random_pair(12, [5, 7, 3], [1, 4, 6, 1], [1, 1, 1, 1])
    xg, xs = to_gpu(x, "f32")
    import torch
    I7 = torch.eye(7, dtype=torch.float32, device="cuda")
    out = ttc.tt_mode_n_product(xg, [1], [I7])
    assert torch.equal(out[1], xg[1])
    A = C.gen_matrix_np(12, 9, 11, 5)  # J = 11 from I = 5
    Ag, As = to_gpu([A], "f32")
    out = ttc.tt_mode_n_product(xg, [0], Ag)
    assert tuple(out[0].shape) == (1, 11, 4)
    assert rel_err(to_np(out[0]), O.mode_n_tt(xs, 0, As[0])[0]) <= TOL["f32"]


# ------------------------------------------------------------------ MPO x TT
def test_mpo_small_dtypes(ttc):
    sw = C.TTShape([3, 5, 2], [1, 4, 3, 1], [4, 6, 3])
    sv = C.TTShape([4, 6, 3], [1, 5, 2, 1])
    w = C.gen_tt_np(41, 1, sw)
    v = C.gen_tt_np(41, 2, sv)
    for dtype in ("f64", "f32", "bf16"):
        wg, ws = to_gpu(w, dtype)
        vg, vs = to_gpu(v, dtype)
        out = [to_np(t) for t in ttc.ttm_apply(wg, vg)]
        want = O.mpo_tt(ws, vs) if dtype != "bf16" else O.mpo_tt(w, v)
        assert max_core_rel(out, want) <= TOL[dtype], dtype
    # identity MPO returns V exactly
    import torch
    ident = [torch.eye(d, dtype=torch.float32, device="cuda").reshape(1, d, d, 1).contiguous() for d in sv.modes]
    vg, _ = to_gpu(v, "f32")
    out = ttc.ttm_apply(ident, vg)
    assert all(torch.equal(a, b) for a, b in zip(out, vg))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_mpo_orders_1_2(ttc, dtype):
    for sw, sv in ((C.TTShape([6], [1, 1], [5]), C.TTShape([5], [1, 1])),
                   (C.TTShape([3, 4], [1, 7, 1], [5, 2]), C.TTShape([5, 2], [1, 3, 1]))):
        w = C.gen_tt_np(47, 1, sw)
        v = C.gen_tt_np(47, 2, sv)
        wg, ws = to_gpu(w, dtype)
        vg, vs = to_gpu(v, dtype)
        out = [to_np(t) for t in ttc.ttm_apply(wg, vg)]
        want = O.mpo_tt(ws, vs) if dtype != "bf16" else O.mpo_tt(w, v)
        assert max_core_rel(out, want) <= TOL[dtype], (sw.order, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_mpo_tiles_and_tails(ttc, dtype):
    """Several MFMA tiles along a' and r', K chunks with a ragged tail (J = 40,
    33), row lengths with and without vector stores (r' = 20, 8, 1), and a
    W slice larger than the per-lane prefetch (J * a' = 1200)."""
    sw = C.TTShape([3, 2, 4], [1, 30, 3, 1], [40, 5, 33])
    sv = C.TTShape([40, 5, 33], [1, 20, 8, 1])
    w = C.gen_tt_np(43, 1, sw)
    v = C.gen_tt_np(43, 2, sv)
    wg, ws = to_gpu(w, dtype)
    vg, vs = to_gpu(v, dtype)
    out = [to_np(t) for t in ttc.ttm_apply(wg, vg)]
    want = O.mpo_tt(ws, vs) if dtype == "f32" else O.mpo_tt(w, v)
    assert max_core_rel(out, want) <= TOL[dtype]


@pytest.mark.parametrize("case", [
    # r' tiles 7 (r1 = 100), J = 50 (two K steps), I = 13 (a ragged chunk of
    # mode indices), r0 = 100 (a ragged group of waves), r1 = 1 (scalar stores)
    (C.TTShape([13, 3], [1, 5, 1], [50, 7]), C.TTShape([50, 7], [1, 100, 1])),
    # a1 = 200: the staged W chunk shrinks to fit; a ragged a' tile
    (C.TTShape([5, 2], [1, 200, 1], [64, 3]), C.TTShape([64, 3], [1, 8, 1])),
    # r1 = 130 and J = 70: beyond the register fragments (the LDS kernel)
    (C.TTShape([3, 2], [1, 3, 1], [70, 4]), C.TTShape([70, 4], [1, 130, 1])),
])
def test_mpo_bf16_shapes(ttc, case):
    """BF16 MPO x TT across the limits of the register-fragment kernel and
    the fallback beyond them: every core against the oracle on the rounded
    inputs (FP32 bound) and on the unrounded ones (BF16 bound)."""
    sw, sv = case
    w = C.gen_tt_np(44, 1, sw)
    v = C.gen_tt_np(44, 2, sv)
    wg, ws = to_gpu(w, "bf16")
    vg, vs = to_gpu(v, "bf16")
    out = [to_np(t) for t in ttc.ttm_apply(wg, vg)]
    assert max_core_rel(out, O.mpo_tt(ws, vs)) <= TOL["f32"]
    assert max_core_rel(out, O.mpo_tt(w, v)) <= TOL["bf16"]


def test_mpo8_bf16_full(ttc):
    """Order-8 MPO (I = J = 32, rank 16) on an order-8 TT (mode 32, rank 64),
    BF16 inputs, FP32 output with ranks 1024.  Every core in full: the total
    error against the FP64 oracle on the unrounded inputs at the BF16 bound,
    and the arithmetic error against the oracle on the rounded inputs at
    the FP32 bound (products of BF16 values are exact in FP32, so only the
    FP32 accumulation of 32 terms remains)."""
    sw, sv = C.mpo8_shapes()
    w = C.gen_tt_np(C.SEED_MPO8, 1, sw)
    v = C.gen_tt_np(C.SEED_MPO8, 2, sv)
    wg, ws = to_gpu(w, "bf16")
    vg, vs = to_gpu(v, "bf16")
    out = ttc.ttm_apply(wg, vg)
    assert [int(t.shape[0]) for t in out] + [1] == [1] + [1024] * 7 + [1]
    for k in range(8):
        got = to_np(out[k])
        et = rel_err(got, O.mpo_tt([w[k]], [v[k]])[0])
        ea = rel_err(got, O.mpo_tt([ws[k]], [vs[k]])[0])
        print(f"mpo8 core {k}: total {et:.3e} arithmetic {ea:.3e}")
        assert et <= TOL["bf16"]
        assert ea <= TOL["f32"]


# ------------------------------------------------------------------ gradient
def _grad_case(ttc, x, y, dtype, gz, stride=0):
    """Gradients of <X, Y> from the GPU against the oracle: FP64 and FP32
    on the values the GPU holds; BF16 cores (FP32 sweeps) on the rounded
    values at the FP32 bound, and the total error against the unrounded
    FP64 cores at the BF16 bound."""
    xg, xs = to_gpu(x, dtype)
    yg, ys = to_gpu(y, dtype)
    gx, gy = ttc.tt_contract_inner_bwd(xg, yg, gz, ckpt_stride=stride)
    got = [to_np(t) for t in gx + gy]
    wx, wy = O.inner_grad(xs, ys, gz)
    e = max_core_rel(got, wx + wy)
    assert e <= (TOL["f32"] if dtype == "bf16" else TOL[dtype])
    if dtype == "bf16":
        ux, uy = O.inner_grad(x, y, gz)
        assert max_core_rel(got, ux + uy) <= TOL["bf16"]
    return e


@pytest.mark.parametrize("stride", [1, 2, 3, 0])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_inner_grad(ttc, dtype, stride):
    """Stride 0 lets the library choose (FP32 and BF16 pairs with ranks <=
    128 store every interface from the LDS-resident sweeps); a positive
    stride keeps every stride-th interface and recomputes the rest."""
    x, y = random_pair(55, [3, 4, 2, 5, 3, 2, 4], [1, 3, 5, 2, 4, 3, 2, 1], [1, 2, 3, 4, 2, 5, 3, 1])
    _grad_case(ttc, x, y, dtype, 0.75, stride)


@pytest.mark.parametrize("stride", [0, 3, 4])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_inner_grad_pair10(ttc, dtype, stride):
    """The order-10 rank-32 pair: every interface stored (stride 0) or
    checkpoints every 3 / 4 cores with the segments recomputed."""
    sx, sy = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    y = C.gen_tt_np(C.SEED_PAIR10, 2, sy)
    _grad_case(ttc, x, y, dtype, 1.25, stride)


@pytest.mark.parametrize("case", [
    ([5], [1, 1], [1, 1]),                                  # order 1
    ([4, 6], [1, 3, 1], [1, 5, 1]),                         # order 2
    ([2, 3, 2], [1, 160, 150, 1], [1, 150, 160, 1]),       # slices too large for LDS (FP64)
    ([2, 2, 2], [1, 210, 200, 1], [1, 200, 210, 1]),       # and for FP32
])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_inner_grad_shapes(ttc, case, dtype):
    modes, rx, ry = case
    x, y = random_pair(57, modes, rx, ry)
    _grad_case(ttc, x, y, dtype, -1.5)


def test_inner_grad_pair10_autograd(ttc):
    import torch
    sx, sy = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    y = C.gen_tt_np(C.SEED_PAIR10, 2, sy)
    xg, xs = to_gpu(x, "f32")
    yg, ys = to_gpu(y, "f32")
    xv = [t.clone().requires_grad_(True) for t in xg]
    z = ttc.tt_inner(xv, yg, ckpt_stride=3)
    z.backward(torch.tensor(2.0, dtype=torch.float64, device="cuda"))
    wx, _ = O.inner_grad(xs, ys, 2.0)
    assert max_core_rel([to_np(t.grad) for t in xv], wx) <= TOL["f32"]
