"""GPU parity of the TT layer (TT-matrix x dense batch, MSE loss, backward)
against the FP64 oracle's dense route, through the C ABI."""
import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

from helpers import TOL, max_core_rel, rel_err, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _batch(seed, obj, rows, cols):
    return C.gen_matrix_np(seed, obj, rows, cols)


def _upload(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.float32).cuda()


def _ws(ttc, wg, batch, prec, sched):
    """The workspace kept from the forward to the backward for the schedule
    that saves its intermediates (None for the others: the call allocates)."""
    if sched != "cores_saved":
        return None
    import torch
    need = ttc.ttm_apply_dense_query(wg, batch, prec, sched, backward=True)
    return torch.empty(need, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("sched", ["dense", "cores", "cores_saved"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_layer_fd_instance(ttc, prec, sched):
    """Order 3, I = J = 4, ranks (1,4,4,1), batch 8: forward, loss and every
    gradient against the oracle's FP64 dense route (which itself is pinned by
    finite differences)."""
    s = C.layer_fd_shape()
    w = C.gen_tt_np(C.SEED_LAYER, 11, s)
    X = _batch(C.SEED_LAYER, 12, 8, 64)
    T = _batch(C.SEED_LAYER, 13, 8, 64)
    wg, ws = to_gpu(w, "f32")
    Xg, Tg = _upload(X), _upload(T)
    Xs, Ts = to_np(Xg), to_np(Tg)
    ref = O.layer_forward_backward(ws, Xs, Ts) if prec == "f32" else O.layer_forward_backward(w, X, T)
    tol = TOL[prec]
    wsp = _ws(ttc, wg, 8, prec, sched)
    Y = ttc.ttm_apply_dense(wg, Xg, prec=prec, sched=sched, ws=wsp)
    assert rel_err(to_np(Y), ref["Y"]) <= tol
    L, dY = ttc.ttc_mse_loss(Y, Tg)
    assert abs(L.item() - ref["L"]) <= tol * ref["L"]
    assert rel_err(to_np(dY), ref["dY"]) <= tol
    dX, dG = ttc.ttm_apply_dense_bwd(wg, Xg, dY, prec=prec, sched=sched, ws=wsp)
    assert rel_err(to_np(dX), ref["dX"]) <= tol
    assert max_core_rel([to_np(g) for g in dG], ref["dG"]) <= tol


@pytest.mark.parametrize("sched", ["auto", "cores_saved"])
def test_layer_autograd_matches_oracle(ttc, sched):
    import torch
    s = C.TTShape([4, 2, 3], [1, 3, 5, 1], [3, 4, 2])   # rectangular: 24 x 24
    w = C.gen_tt_np(C.SEED_LAYER, 21, s)
    X = _batch(C.SEED_LAYER, 22, 37, 24)                   # ragged batch
    T = _batch(C.SEED_LAYER, 23, 37, 24)
    wg, ws = to_gpu(w, "f32")
    Xg, Tg = _upload(X), _upload(T)
    ref = O.layer_forward_backward(ws, to_np(Xg), to_np(Tg))
    cores = [c.clone().requires_grad_(True) for c in wg]
    xv = Xg.clone().requires_grad_(True)
    Y = ttc.tt_linear(xv, cores, sched=sched)
    L, dY = ttc.ttc_mse_loss(Y.detach(), Tg)
    Y.backward(dY)
    assert rel_err(to_np(xv.grad), ref["dX"]) <= TOL["f32"]
    assert max_core_rel([to_np(c.grad) for c in cores], ref["dG"]) <= TOL["f32"]


_L4 = {}


def _layer4(ttc):
    """Full-size layer inputs (order-4 TT-matrix 4096 -> 4096, modes 8, ranks
    32; X and T 8192 x 4096) and the oracle's FP64 dense route on them,
    cached: "f32" on the FP32 values the GPU holds, "bf16" on the unrounded
    FP64 cores (the BF16 option's total error)."""
    if _L4:
        return _L4
    import torch
    s = C.layer4_shape()
    w = C.gen_tt_np(C.SEED_LAYER, 1, s)
    wg, ws = to_gpu(w, "f32")
    Xg = C.gen_matrix_torch(C.SEED_LAYER, 2, 8192, 4096, "cuda", torch.float32)
    Tg = C.gen_matrix_torch(C.SEED_LAYER, 3, 8192, 4096, "cuda", torch.float32)
    Xn, Tn = to_np(Xg), to_np(Tg)
    _L4.update(w=w, ws=ws, wg=wg, Xg=Xg, Tg=Tg,
               f32=O.layer_forward_backward(ws, Xn, Tn),
               bf16=O.layer_forward_backward(w, Xn, Tn))
    return _L4


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("sched", ["dense", "cores", "cores_saved"])
def test_layer4_full_size(ttc, sched, prec):
    """The full 8192 x 4096 batch through both schedules, FP32 and the BF16
    MFMA option: Y, the loss, dY, dX and every core gradient against the
    oracle's dense route, whole arrays (rel_err: relative Frobenius and per
    row); and the Euler identity <dL/dG_k, G_k> = <dL/dY, Y> for every core
    (Y is linear in each core)."""
    d = _layer4(ttc)
    ref, tol = d[prec], TOL[prec]
    wsp = _ws(ttc, d["wg"], 8192, prec, sched)
    Y = ttc.ttm_apply_dense(d["wg"], d["Xg"], prec=prec, sched=sched, ws=wsp)
    Yn = to_np(Y)
    assert rel_err(Yn, ref["Y"]) <= tol
    L, dY = ttc.ttc_mse_loss(Y, d["Tg"])
    assert abs(L.item() - ref["L"]) <= tol * ref["L"]
    dYn = to_np(dY)
    assert rel_err(dYn, ref["dY"]) <= tol
    dX, dG = ttc.ttm_apply_dense_bwd(d["wg"], d["Xg"], dY, prec=prec, sched=sched, ws=wsp)
    del wsp
    assert rel_err(to_np(dX), ref["dX"]) <= tol
    dGn = [to_np(g) for g in dG]
    errs = [rel_err(g, r) for g, r in zip(dGn, ref["dG"])]
    print(f"layer4 {sched} {prec}: dG errors {errs}")
    assert max(errs) <= tol
    euler = float(np.sum(dYn * Yn))
    for k in range(4):
        got = float(np.sum(dGn[k] * d["ws"][k]))
        assert abs(got - euler) <= (1e-4 if prec == "f32" else 2e-2) * abs(euler)


@pytest.mark.parametrize("sched", ["cores", "dense", "cores_saved"])
@pytest.mark.parametrize("dims", [
    ([4, 2, 3], [1, 3, 5, 1], [3, 4, 2], 37),       # rectangular, ragged batch
    ([5], [1, 1], [7], 3),                          # order 1
    ([3, 2, 2, 3], [1, 2, 6, 3, 1], [2, 3, 3, 2], 130),
    ([16, 3], [1, 5, 1], [40, 9], 21),              # wide last pair block, long leading column mode
])
def test_layer_cores_schedule(ttc, dims, sched):
    """Both schedules against the oracle: forward, dX and every core
    gradient, on shapes with uneven modes, ranks and a ragged batch."""
    rows, ranks, cols, B = dims
    s = C.TTShape(rows, ranks, cols)
    w = C.gen_tt_np(C.SEED_LAYER, 31, s)
    ncol = int(np.prod(cols))
    X = _batch(C.SEED_LAYER, 32, B, ncol)
    T = _batch(C.SEED_LAYER, 33, B, int(np.prod(rows)))
    wg, ws = to_gpu(w, "f32")
    Xg, Tg = _upload(X), _upload(T)
    ref = O.layer_forward_backward(ws, to_np(Xg), to_np(Tg))
    wsp = _ws(ttc, wg, B, "auto", sched)
    Y = ttc.ttm_apply_dense(wg, Xg, sched=sched, ws=wsp)
    assert rel_err(to_np(Y), ref["Y"]) <= TOL["f32"]
    _, dY = ttc.ttc_mse_loss(Y, Tg)
    dX, dG = ttc.ttm_apply_dense_bwd(wg, Xg, dY, sched=sched, ws=wsp)
    assert rel_err(to_np(dX), ref["dX"]) <= TOL["f32"]
    assert max_core_rel([to_np(g) for g in dG], ref["dG"]) <= TOL["f32"]


def test_mse_loss_odd_size(ttc):
    import torch
    y = torch.randn(1001, device="cuda")
    t = torch.randn(1001, device="cuda")
    L, dy = ttc.ttc_mse_loss(y, t)
    yn, tn = to_np(y), to_np(t)
    assert abs(L.item() - np.mean((yn - tn) ** 2)) <= 1e-12 * np.mean((yn - tn) ** 2)
    assert rel_err(to_np(dy), 2 * (yn - tn) / 1001) <= 1e-6


@pytest.mark.parametrize("sched", ["dense"])
def test_layer_bf16_tile_kernel_ragged(ttc, sched):
    """The BF16 dense schedule on a shape whose products take the 256 x 256
    BF16 tile kernel with ragged edges (4000 x 1080 output, 960-long
    reduction; 4000 x 960 output, 1080-long reduction): forward, dX and
    every core gradient against the oracle's dense route on the unrounded
    cores (total error, BF16 bound)."""
    s = C.TTShape([10, 12, 9], [1, 6, 5, 1], [8, 12, 10])
    w = C.gen_tt_np(C.SEED_LAYER, 41, s)
    X = _batch(C.SEED_LAYER, 42, 4000, 960)
    T = _batch(C.SEED_LAYER, 43, 4000, 1080)
    wg, _ = to_gpu(w, "f32")
    Xg, Tg = _upload(X), _upload(T)
    ref = O.layer_forward_backward(w, to_np(Xg), to_np(Tg))
    Y = ttc.ttm_apply_dense(wg, Xg, prec="bf16", sched=sched)
    assert rel_err(to_np(Y), ref["Y"]) <= TOL["bf16"]
    _, dY = ttc.ttc_mse_loss(Y, Tg)
    dX, dG = ttc.ttm_apply_dense_bwd(wg, Xg, dY, prec="bf16", sched=sched)
    assert rel_err(to_np(dX), ref["dX"]) <= TOL["bf16"]
    assert max_core_rel([to_np(g) for g in dG], ref["dG"]) <= TOL["bf16"]
