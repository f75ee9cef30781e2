"""GPU parity of TT-SVD (Algorithm 1) against the FP64 oracle, through the C
ABI: the kept ranks, the cores (a singular vector is fixed only up to its
sign, so each bond's columns are aligned to the oracle's before the
comparison, the next core's rows flipped with them), the reconstruction and
Algorithm 1's error bound, on the paper's Example 2 shapes, truncated
low-rank tensors, wide and tall unfoldings, and degenerate cases."""
import math

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

from helpers import TOL, rel_err, to_gpu, to_np

pytestmark = pytest.mark.gpu

SEED_SVD = C.BASE_SEED + 6


def _dense(obj, dims):
    n = int(np.prod(dims))
    return C.gen_matrix_np(SEED_SVD, obj, 1, n).reshape(dims)


def _upload(X, dtype):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(X)).to(torch.float64 if dtype == "f64" else torch.float32)
    return t.cuda(), t.to(torch.float64).numpy()


def _align(got, want):
    """Flip each bond's singular-vector signs in `got` to match `want`
    (column c of core k and row c of core k + 1 together); shapes must
    match."""
    got = [g.copy() for g in got]
    for k in range(len(got) - 1):
        r = got[k].shape[2]
        U, Ur = got[k].reshape(-1, r), want[k].reshape(-1, r)
        sgn = np.sign(np.sum(U * Ur, axis=0))
        sgn[sgn == 0] = 1.0
        got[k] = got[k] * sgn[None, None, :]
        got[k + 1] = got[k + 1] * sgn[:, None, None]
    return got


def _check(ttc, X, dtype, eps, core_tol, max_rank=0):
    xg, Xs = _upload(X, dtype)
    cores = [to_np(c) for c in ttc.tt_svd(xg, eps=eps, max_rank=max_rank)]
    ref = O.tt_svd(Xs, eps)
    assert [c.shape for c in cores] == [c.shape for c in ref]
    Xh = O.tt_full(cores)
    nx = np.linalg.norm(Xs)
    # Algorithm 1's bound, plus the arithmetic's rounding
    err = np.linalg.norm(Xh - Xs)
    assert err <= eps * nx + TOL[dtype] * nx, (err, eps * nx)
    e = max(rel_err(g, w) for g, w in zip(_align(cores, ref), ref))
    assert e <= core_tol, e
    return cores, ref


@pytest.mark.parametrize("dims", [(20, 20, 20), (20, 20, 20, 5), (20, 20, 20, 5, 4)])
def test_svd_example2_shapes_exact(ttc, dims):
    """The shapes of the paper's Example 2 (Gaussian N(0, 1) entries), eps = 0:
    full ranks, cores equal to the oracle's up to the sign of each singular
    vector, reconstruction to FP64 rounding."""
    X = _dense(1, dims)
    cores, _ = _check(ttc, X, "f64", 0.0, 1e-9)
    assert rel_err(O.tt_full(cores), X) <= 1e-12


@pytest.mark.parametrize("eps", [1e-4, 3e-2])
def test_svd_truncates_low_rank_plus_noise(ttc, eps):
    """A TT of ranks (1, 3, 5, 2, 1) plus noise 1e-7: at eps = 1e-4 both keep
    exactly those ranks; at eps = 3e-2 the truncation also cuts signal, and
    the GPU and the oracle still pick the same ranks and cores."""
    s = C.TTShape([6, 7, 5, 4], [1, 3, 5, 2, 1])
    X = O.tt_full(C.gen_tt_np(SEED_SVD, 2, s)) + 1e-7 * _dense(3, (6, 7, 5, 4))
    cores, _ = _check(ttc, X, "f64", eps, 1e-8)
    if eps == 1e-4:
        assert [c.shape[0] for c in cores] + [1] == [1, 3, 5, 2, 1]


@pytest.mark.parametrize("dims", [(50, 7), (7, 50), (3, 40, 2), (64, 2, 2, 2), (5,)])
def test_svd_wide_tall_and_small(ttc, dims):
    """Orders 1-4 with wide (rows <= columns) and tall first unfoldings."""
    X = _dense(4, dims)
    _check(ttc, X, "f64", 0.0, 1e-9)


def test_svd_rank_one_and_zero(ttc):
    import torch
    vs = [C.gen_matrix_np(SEED_SVD, 10 + k, 1, d)[0] for k, d in enumerate((4, 6, 5))]
    X = np.einsum("a,b,c->abc", *vs)
    cores, _ = _check(ttc, X, "f64", 1e-10, 1e-9)
    assert [c.shape[0] for c in cores] == [1, 1, 1]
    z = torch.zeros(3, 4, 5, dtype=torch.float64, device="cuda")
    zc = ttc.tt_svd(z)
    assert [tuple(c.shape) for c in zc] == [(1, 3, 1), (1, 4, 1), (1, 5, 1)]
    assert all(bool(torch.all(torch.isfinite(c))) for c in zc)
    assert np.all(O.tt_full([to_np(c) for c in zc]) == 0.0)


def test_svd_fp32(ttc):
    """FP32 tensor, FP32 storage with FP64 dot products: ranks equal the
    oracle's (on the FP32 values), reconstruction within the FP32 bound,
    left cores orthonormal to the Jacobi threshold (pairs stop rotating at
    |a_i . a_j| <= 32 u sqrt(L) ||a_i|| ||a_j||, about 4e-5 for L = 480 in
    FP32)."""
    X = _dense(5, (12, 10, 8, 6))
    xg, Xs = _upload(X, "f32")
    cores = [to_np(c) for c in ttc.tt_svd(xg)]
    ref = O.tt_svd(Xs, 0.0)
    assert [c.shape for c in cores] == [c.shape for c in ref]
    assert rel_err(O.tt_full(cores), Xs) <= TOL["f32"]
    for G in cores[:-1]:
        U = G.reshape(-1, G.shape[2])
        assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) <= 1e-4


def test_svd_max_rank_caps(ttc):
    X = _dense(6, (8, 9, 10))
    xg, _ = _upload(X, "f64")
    cores = ttc.tt_svd(xg, max_rank=3)
    assert [int(c.shape[0]) for c in cores] + [1] == [1, 3, 3, 1]
    # the first core is the oracle's first three singular vectors
    ref = O.tt_svd(X, 0.0)
    got = to_np(cores[0]).reshape(8, 3)
    want = ref[0].reshape(8, 8)[:, :3]
    assert np.max(np.abs(np.abs(np.sum(got * want, axis=0)) - 1.0)) <= 1e-12


# ------------------------------------------------------------ TT-rounding
def _tt_sum(x, y):
    """Cores of X + Y (block-diagonal middle cores, concatenated ends): a
    valid TT with the ranks added, used as redundant input to rounding."""
    N = len(x)
    out = []
    for k in range(N):
        a, b = x[k], y[k]
        if k == 0:
            out.append(np.concatenate([a, b], axis=2))
        elif k == N - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            G = np.zeros((a.shape[0] + b.shape[0], a.shape[1], a.shape[2] + b.shape[2]))
            G[:a.shape[0], :, :a.shape[2]] = a
            G[a.shape[0]:, :, a.shape[2]:] = b
            out.append(G)
    return out


def _round_check(ttc, x, eps, dtype="f64", core_tol=1e-9, max_rank=0):
    from helpers import to_gpu
    xg, xs = to_gpu(x, dtype)
    cores = [to_np(c) for c in ttc.tt_round(xg, eps=eps, max_rank=max_rank)]
    Xs = O.tt_full(xs)
    ref = O.tt_svd(Xs, eps)
    assert [c.shape for c in cores] == [c.shape for c in ref]
    nx = np.linalg.norm(Xs)
    assert np.linalg.norm(O.tt_full(cores) - Xs) <= eps * nx + TOL[dtype] * nx
    if core_tol is not None:
        assert max(rel_err(g, w) for g, w in zip(_align(cores, ref), ref)) <= core_tol
    return cores


def test_round_recovers_ranks_of_a_redundant_sum(ttc):
    """X + X held with doubled ranks: rounding at eps = 1e-10 returns the
    ranks of X and the cores of TT-SVD of the dense 2X."""
    s = C.TTShape([5, 6, 4, 3], [1, 3, 4, 2, 1])
    x = C.gen_tt_np(SEED_SVD, 20, s)
    cores = _round_check(ttc, _tt_sum(x, x), 1e-10)
    assert [c.shape[0] for c in cores] + [1] == [1, 3, 4, 2, 1]


@pytest.mark.parametrize("eps", [1e-12, 0.05, 0.3])
def test_round_truncates_like_tt_svd(ttc, eps):
    """eps 1e-12: the exact ranks (the dense tensor's rounding-level
    singular values, about 1e-16, fall below delta); larger eps truncate
    signal, and the ranks and cores follow TT-SVD of the dense tensor."""
    s = C.TTShape([4, 5, 6, 3], [1, 4, 8, 3, 1])
    x = C.gen_tt_np(SEED_SVD, 21, s)
    _round_check(ttc, x, eps)


def test_round_mpo_product(ttc):
    """The MPO x TT output (ranks multiplied, 3 x 4 = 12) rounded back."""
    from helpers import to_gpu
    sw = C.TTShape([4, 3, 4, 2], [1, 3, 3, 3, 1], [3, 4, 2, 3])
    sv = C.TTShape([3, 4, 2, 3], [1, 4, 4, 4, 1])
    wg, _ = to_gpu(C.gen_tt_np(SEED_SVD, 22, sw), "f64")
    vg, _ = to_gpu(C.gen_tt_np(SEED_SVD, 23, sv), "f64")
    out = [to_np(t) for t in ttc.ttm_apply(wg, vg)]
    assert [c.shape[0] for c in out][1:] == [12, 12, 12]
    _round_check(ttc, out, 1e-8)


def test_round_fp32_and_cap(ttc):
    s = C.TTShape([4, 5, 6, 3], [1, 4, 8, 3, 1])
    x = C.gen_tt_np(SEED_SVD, 24, s)
    _round_check(ttc, x, 1e-6, dtype="f32", core_tol=None)
    from helpers import to_gpu
    xg, _ = to_gpu(x, "f64")
    cores = ttc.tt_round(xg, max_rank=2)
    assert [int(c.shape[0]) for c in cores] + [1] == [1, 2, 2, 2, 1]


def test_round_mpo8_rank1024(ttc):
    """The order-8 MPO x TT product (BF16 inputs, FP32 cores of ranks 1024)
    rounded at eps = 0.3 on the GPU: every core unfolding is 1024 x 32768,
    so each Jacobi SVD rotates 1024 vectors.  Checked at full size through
    properties (no dense tensor exists: 32^8 entries): ranks below 1024;
    cores 0..6 left-orthonormal to the FP32 Jacobi threshold (32 u sqrt(L),
    about 3.5e-4 at L = 32768); and Algorithm 1's bound through the
    inner products of the library, ||X - X'||^2 = <X, X> - 2 <X, X'> +
    <X', X'> <= eps^2 ||X||^2."""
    import torch
    sw, sv = C.mpo8_shapes()
    wg, _ = to_gpu(C.gen_tt_np(C.SEED_MPO8, 1, sw), "bf16")
    vg, _ = to_gpu(C.gen_tt_np(C.SEED_MPO8, 2, sv), "bf16")
    x = ttc.ttm_apply(wg, vg)
    eps = 0.3
    r = ttc.tt_round(x, eps=eps)
    ranks = [int(c.shape[0]) for c in r] + [1]
    print("rounded ranks", ranks)
    assert all(1 <= a <= 1024 for a in ranks) and ranks[1] < 1024
    for G in r[:-1]:
        U = G.reshape(-1, G.shape[2]).to(torch.float64)
        I = torch.eye(U.shape[1], dtype=torch.float64, device=U.device)
        assert float(torch.max(torch.abs(U.T @ U - I))) <= 1e-3
    xx = ttc.tt_contract_inner(x, x).item()
    xr = ttc.tt_contract_inner(x, r).item()
    rr = ttc.tt_contract_inner(r, r).item()
    err2 = xx - 2 * xr + rr
    print("relative error", math.sqrt(max(err2, 0.0) / xx))
    assert err2 <= (eps ** 2 + 1e-3) * xx
