"""GPU parity of contractions at any positions (X's modes a1..a2 with Y's
b1..b2; eq. (8) once per pair; Example 1's x_n^m) against the FP64 oracle,
through the C ABI: the junction T, the natural-order TT and the dense
result on every block layout (middle blocks, prefix/suffix on one side,
either tensor fully contracted), in FP64 (per-entry sums), FP32 and BF16
(MFMA products batched over the transfer's rows); a middle block of the
order-10 rank-32 pair; transfers with more rows than one batch takes; and
Algorithm 2 from dense inputs with TT-SVD on the GPU (Example 1)."""
import json
import os

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

from helpers import TOL, max_core_rel, rel_err, scalar_err, to_gpu, to_np, tt_norm

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")

CASES = [
    # (X modes, X ranks, Y modes, Y ranks, xmodes, ymodes)
    ([3, 4, 5, 2], [1, 2, 3, 2, 1], [3, 5, 4], [1, 2, 3, 1], [2], [1]),
    ([3, 4, 5, 2], [1, 2, 3, 2, 1], [2, 4, 5, 3], [1, 3, 2, 2, 1], [1, 2], [1, 2]),
    ([4, 3, 2], [1, 2, 3, 1], [2, 4, 3], [1, 3, 2, 1], [0], [1]),
    ([3, 2, 4], [1, 2, 2, 1], [4, 3, 2], [1, 2, 3, 1], [2], [0]),
    ([3, 4, 2], [1, 3, 2, 1], [2, 3, 4], [1, 2, 2, 1], [1], [2]),
    ([3, 4], [1, 2, 1], [2, 3, 4, 2], [1, 2, 3, 2, 1], [0, 1], [1, 2]),
    ([3, 4], [1, 2, 1], [3, 4, 2], [1, 2, 3, 1], [0, 1], [0, 1]),
    ([3, 4], [1, 2, 1], [2, 3, 4], [1, 2, 3, 1], [0, 1], [1, 2]),
    ([2, 3, 4, 2], [1, 2, 3, 2, 1], [3, 4], [1, 2, 1], [1, 2], [0, 1]),
    ([2, 3, 4], [1, 2, 3, 1], [3, 4], [1, 2, 1], [1, 2], [0, 1]),
    # larger ranks, several MFMA-sized tiles in T, a long block
    ([5, 6, 4, 7, 3, 2], [1, 5, 9, 7, 6, 4, 1], [2, 4, 7, 3, 5], [1, 2, 8, 5, 3, 1], [2, 3, 4], [1, 2, 3]),
]


def _tt(obj, modes, ranks):
    return C.gen_tt_np(C.SEED_INNER4 + 40, obj, C.TTShape(list(modes), list(ranks)))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_pairs_every_layout(ttc, case, dtype):
    mx, rx, my, ry, xm, ym = case
    x, y = _tt(1, mx, rx), _tt(2, my, ry)
    xg, xs = to_gpu(x, dtype)
    yg, ys = to_gpu(y, dtype)
    ref = (x, y) if dtype == "bf16" else (xs, ys)
    tol = TOL[dtype]
    T = to_np(ttc.tt_contract_pairs(xg, yg, xm, ym, "junction"))
    assert rel_err(T, O.transfer_junction(*ref, xm, ym)) <= tol
    nat = [to_np(t) for t in ttc.tt_contract_pairs(xg, yg, xm, ym, "natural")]
    want = O.contract_pairs_natural(*ref, xm, ym)
    assert [g.shape for g in nat] == [w.shape for w in want]
    assert max_core_rel(nat, want) <= tol
    Z = to_np(ttc.tt_contract_pairs(xg, yg, xm, ym, "dense"))
    assert rel_err(Z, O.contract_pairs_dense(O.tt_full(ref[0]), O.tt_full(ref[1]), xm, ym)) <= tol
    if dtype == "bf16":
        # arithmetic only (FP32 sums of the rounded values)
        assert rel_err(T, O.transfer_junction(xs, ys, xm, ym)) <= TOL["f32"]


@pytest.mark.parametrize("r", [255, 256])
def test_pairs_transfer_many_rows(ttc, r):
    """A two-pair middle block whose transfer has r^2 rows (a, g): 65025 run
    as one batch of MFMA products per step, 65536 beyond the batch limit on
    the per-entry path; both against the oracle's junction."""
    sx = C.TTShape([2, 3, 3], [1, r, 4, 1])
    sy = C.TTShape([2, 3, 3], [1, r, 3, 1])
    x, y = _tt(5, sx.modes, sx.ranks), _tt(6, sy.modes, sy.ranks)
    xg, xs = to_gpu(x, "f32")
    yg, ys = to_gpu(y, "f32")
    T = to_np(ttc.tt_contract_pairs(xg, yg, [1, 2], [1, 2], "junction"))
    assert T.shape == (r * r, 1)
    assert rel_err(T, O.transfer_junction(xs, ys, [1, 2], [1, 2])) <= TOL["f32"]


def test_pairs_integer_cores_bit_exact(ttc):
    mx, rx, my, ry, xm, ym = CASES[-1]
    x = C.gen_int_tt_np(61, 1, C.TTShape(mx, rx))
    y = C.gen_int_tt_np(61, 2, C.TTShape(my, ry))
    want = O.transfer_junction(x, y, xm, ym)
    assert np.max(np.abs(want)) < 2 ** 20
    for dtype in ("f64", "f32", "bf16"):
        T = to_np(ttc.tt_contract_pairs(to_gpu(x, dtype)[0], to_gpu(y, dtype)[0], xm, ym, "junction"))
        assert np.array_equal(T, want), dtype


def test_pairs_middle_block_pair10(ttc):
    """Modes 4-7 of the order-10 rank-32 FP32 pair against each other: the
    1024 x 1024 junction against the oracle's, whole."""
    sx, sy = C.pair10_shapes()
    x = C.gen_tt_np(C.SEED_PAIR10, 1, sx)
    y = C.gen_tt_np(C.SEED_PAIR10, 2, sy)
    xg, xs = to_gpu(x, "f32")
    yg, ys = to_gpu(y, "f32")
    m = [3, 4, 5, 6]
    T = to_np(ttc.tt_contract_pairs(xg, yg, m, m, "junction"))
    assert T.shape == (1024, 1024)
    assert rel_err(T, O.transfer_junction(xs, ys, m, m)) <= TOL["f32"]


def test_pairs_all_modes_and_errors(ttc):
    x, y = _tt(3, [3, 4, 2], [1, 2, 3, 1]), _tt(4, [3, 4, 2], [1, 3, 2, 1])
    xg, _ = to_gpu(x, "f64")
    yg, _ = to_gpu(y, "f64")
    z = ttc.tt_contract_pairs(xg, yg, [0, 1, 2], [0, 1, 2]).item()
    assert scalar_err(z, O.inner_lr(x, y), tt_norm(x), tt_norm(y)) <= TOL["f64"]
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_pairs(xg, yg, [0, 2], [0, 2])
    assert ei.value.name == "TTC_ERR_UNSUPPORTED"
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_pairs(xg, yg, [0], [1])
    assert ei.value.name == "TTC_ERR_SHAPE"
    with pytest.raises(ttc.TTCError) as ei:
        ttc.tt_contract_pairs(xg, yg, [3], [0])
    assert ei.value.name == "TTC_ERR_MODE"


def _example1():
    with open(os.path.join(GOLD, "example1_shapes.json")) as f:
        g = json.load(f)
    sz = g["sizes"]
    X = C.gen_matrix_np(C.SEED_INNER4 + 41, 1, 1, int(np.prod([sz[m] for m in g["X_modes"]])))
    Y = C.gen_matrix_np(C.SEED_INNER4 + 41, 2, 1, int(np.prod([sz[m] for m in g["Y_modes"]])))
    X = X.reshape([sz[m] for m in g["X_modes"]])
    Y = Y.reshape([sz[m] for m in g["Y_modes"]])
    return X, Y, g["contract"]["n"] - 1, g["contract"]["m"] - 1


def test_example1_on_cores_end_to_end(ttc):
    """Example 1 (X of order 4, Y of order 3, X's third mode with Y's
    second) from dense inputs: TT-SVD of X and Y on the GPU, then the
    contraction directly on the cores at positions 3 and 2; the dense result
    against eq. (8) on the dense inputs."""
    import torch
    X, Y, n, m = _example1()
    gx = ttc.tt_svd(torch.from_numpy(X).cuda())
    gy = ttc.tt_svd(torch.from_numpy(Y).cuda())
    Z = to_np(ttc.tt_contract_pairs(gx, gy, [n], [m], "dense"))
    assert rel_err(Z, O.tcp(X, Y, n, m)) <= 1e-12
    nat = [to_np(t) for t in ttc.tt_contract_pairs(gx, gy, [n], [m], "natural")]
    assert rel_err(O.tt_full(nat), O.tcp(X, Y, n, m)) <= 1e-12


def test_example1_algorithm2_route(ttc):
    """Algorithm 2 as the paper states it: the contracted modes moved first
    (the permuted copies are the test's inputs), TT-SVD of both on the GPU,
    K = A_x^T A_y as the junction of the first positions, and Z^rho built
    from X's remaining cores reversed and transposed, K and Y's cores.  The
    singular vectors' signs are free, so K is compared entrywise in absolute
    value and Z^rho (sign free) in full."""
    import torch
    X, Y, n, m = _example1()
    Xp = np.ascontiguousarray(np.transpose(X, [n] + [k for k in range(X.ndim) if k != n]))
    Yp = np.ascontiguousarray(np.transpose(Y, [m] + [k for k in range(Y.ndim) if k != m]))
    gx = ttc.tt_svd(torch.from_numpy(Xp).cuda())
    gy = ttc.tt_svd(torch.from_numpy(Yp).cuda())
    K = to_np(ttc.tt_contract_pairs(gx, gy, [0], [0], "junction")).reshape(gx[0].shape[2], gy[0].shape[2])
    _, parts = O.ttcp(X, Y, n, m)
    assert K.shape == parts["K"].shape
    assert rel_err(np.abs(K), np.abs(parts["K"])) <= 1e-12
    xs = [np.transpose(to_np(G), (2, 1, 0)) for G in gx[1:][::-1]]
    ys = [to_np(G) for G in gy[1:]]
    Zr = xs[0]
    for G in xs[1:] + [K] + ys:
        Zr = np.tensordot(Zr, G, axes=([Zr.ndim - 1], [0]))
    Zr = Zr.reshape(Zr.shape[1:-1])
    assert rel_err(Zr, parts["Zrho"]) <= 1e-12
