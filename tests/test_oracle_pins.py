"""Pins of the FP64 oracle against things other than itself: brute force on
tiny inputs, closed forms, invariants, exact integer arithmetic, the paper's
printed operation counts and the index wiring of its worked example.
CPU only."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C
from ttgen import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_pair(seed, modes, rx, ry):
    x = C.gen_tt_np(seed, 1, C.TTShape(list(modes), list(rx)))
    y = C.gen_tt_np(seed, 2, C.TTShape(list(modes), list(ry)))
    return x, y


# ----------------------------------------------------------------- index maps
def test_lin_index_little_endian():
    dims = [3, 4, 2]
    X = np.arange(24).reshape(dims, order="F")
    for idx in itertools.product(range(3), range(4), range(2)):
        # Def. 2: first index fastest
        assert O.lin_index(idx, dims) == idx[0] + 3 * idx[1] + 12 * idx[2]
        assert O.vec(X)[O.lin_index(idx, dims)] == X[idx]
    assert np.array_equal(O.fold(O.vec(X), dims), X)


def test_unfold_fold_roundtrip_and_columns():
    X = np.random.RandomState(1).randn(2, 3, 4)
    for n in range(3):
        M = O.unfold(X, n)
        assert M.shape == (X.shape[n], X.size // X.shape[n])
        assert np.array_equal(O.refold(M, n, X.shape), X)
    M1 = O.unfold(X, 1)
    # column index = little-endian over (i_0, i_2)
    for i0, i1, i2 in itertools.product(range(2), range(3), range(4)):
        assert M1[i1, i0 + 2 * i2] == X[i0, i1, i2]


def test_stacking_mode():
    s = [np.random.RandomState(k).randn(2, 3) for k in range(4)]
    Y = O.stack(s)
    U = O.unfold(Y, 2)  # mode-(N+1) unfolding: rows are the samples' vec
    for k in range(4):
        assert np.array_equal(U[k], O.vec(s[k]))


# ------------------------------------------------------------- eq. (8), Def. 5
def test_tcp_matches_elementwise_definition():
    rs = np.random.RandomState(2)
    X = rs.randn(2, 3, 4)
    Y = rs.randn(4, 2, 3)
    assert rel(O.tcp(X, Y, 2, 0), O.tcp_loops(X, Y, 2, 0)) < 1e-14
    assert rel(O.tcp(X, Y, 1, 2), O.tcp_loops(X, Y, 1, 2)) < 1e-14


def test_mode_n_matches_elementwise_definition():
    rs = np.random.RandomState(3)
    X = rs.randn(3, 4, 2)
    A = rs.randn(5, 4)
    assert rel(O.mode_n_product(X, A, 1), O.mode_n_loops(X, A, 1)) < 1e-14


# ------------------------------------------------------------ TT reconstruction
def test_tt_full_matches_entrywise_products():
    x, _ = small_pair(5, [2, 3, 2, 3], [1, 2, 3, 2, 1], [1, 1, 1, 1, 1])
    X = O.tt_full(x)
    for idx in itertools.product(*[range(d) for d in X.shape]):
        assert abs(X[idx] - O.tt_entry(x, idx)) < 1e-14


# ------------------------------------------------------------ inner products
def test_inner_all_routes_agree_and_match_brute_force_inner4():
    sx, sy = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    y = C.gen_tt_np(C.SEED_INNER4, 2, sy)
    z = O.inner_lr(x, y)
    bf = O.inner_bruteforce(x, y)   # 8^4 entries, every one a product of slices
    scale = math.sqrt(O.tt_norm2_dense(x) * O.tt_norm2_dense(y))
    assert abs(z - bf) / scale < 1e-14
    assert abs(O.inner_rl(x, y) - z) / scale < 1e-14
    for c in range(1, 4):
        assert abs(O.inner_meet(x, y, c) - z) / scale < 1e-14


def test_inner_rank1_closed_form_pair10_size():
    # <x1 o ... o xN, y1 o ... o yN> = prod_n <x_n, y_n>
    rs = np.random.RandomState(4)
    xs = [rs.randn(16) for _ in range(10)]
    ys = [rs.randn(16) for _ in range(10)]
    x = [v.reshape(1, 16, 1) for v in xs]
    y = [v.reshape(1, 16, 1) for v in ys]
    want = math.prod(float(a @ b) for a, b in zip(xs, ys))
    assert abs(O.inner_lr(x, y) - want) <= 1e-13 * abs(want)
    assert abs(O.inner_rl(x, y) - want) <= 1e-13 * abs(want)


def test_inner_integer_cores_exact():
    s = C.TTShape([3, 4, 2, 3], [1, 3, 2, 4, 1])
    x = C.gen_int_tt_np(9, 1, s)
    y = C.gen_int_tt_np(9, 2, s)
    # exact integer dense reconstruction with Python ints
    xi = [G.astype(np.int64) for G in x]
    yi = [G.astype(np.int64) for G in y]
    want = 0
    for idx in itertools.product(*[range(d) for d in s.modes]):
        a = np.ones((1,), dtype=np.int64)
        b = np.ones((1,), dtype=np.int64)
        for k, i in enumerate(idx):
            a = a @ xi[k][:, i, :]
            b = b @ yi[k][:, i, :]
        want += int(a[0]) * int(b[0])
    assert O.inner_lr(x, y) == float(want)
    assert O.inner_rl(x, y) == float(want)


def test_inner_norm_symmetry_cauchy_schwarz():
    x, y = small_pair(11, [3, 2, 4, 3], [1, 2, 4, 3, 1], [1, 3, 2, 2, 1])
    xx = O.inner_lr(x, x)
    assert xx >= 0
    assert abs(xx - O.tt_norm2_dense(x)) <= 1e-13 * xx
    assert abs(O.inner_lr(x, y) - O.inner_lr(y, x)) <= 1e-13 * math.sqrt(xx * O.inner_lr(y, y))
    assert abs(O.inner_lr(x, y)) <= math.sqrt(xx * O.inner_lr(y, y)) * (1 + 1e-14)


def test_inner_scaling_exact_and_linearity():
    x, y = small_pair(12, [3, 2, 4], [1, 2, 3, 1], [1, 3, 2, 1])
    z = O.inner_lr(x, y)
    x2 = [G.copy() for G in x]
    x2[1] = x2[1] * 8.0
    assert O.inner_lr(x2, y) == 8.0 * z  # power-of-two scaling is exact
    # linearity in core 2 of X
    xa = [G.copy() for G in x]
    xb = [G.copy() for G in x]
    xb[2] = np.random.RandomState(5).randn(*x[2].shape)
    xs = [G.copy() for G in x]
    xs[2] = 0.3 * xa[2] - 1.7 * xb[2]
    lhs = O.inner_lr(xs, y)
    rhs = 0.3 * O.inner_lr(xa, y) - 1.7 * O.inner_lr(xb, y)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs) + 1)


def test_inner_gauge_invariance():
    x, y = small_pair(13, [3, 4, 2, 3], [1, 3, 4, 2, 1], [1, 2, 2, 3, 1])
    z = O.inner_lr(x, y)
    Q = np.random.RandomState(6).randn(4, 4) + 4 * np.eye(4)
    xg = [G.copy() for G in x]
    xg[1] = np.einsum("ais,st->ait", x[1], Q)
    xg[2] = np.einsum("st,tib->sib", np.linalg.inv(Q), x[2])
    assert abs(O.inner_lr(xg, y) - z) <= 1e-12 * max(1.0, abs(z))


# ------------------------------------------------------- partial contractions
@pytest.mark.parametrize("modes", [[2, 3], [0, 1], [0], [3], [0, 1, 2], [1, 2, 3]])
def test_natural_form_matches_eq8_on_dense(modes):
    sx, sy = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    y = C.gen_tt_np(C.SEED_INNER4, 2, sy)
    Zn = O.tt_full(O.contract_natural(x, y, modes))
    Zd = O.contract_dense(x, y, modes)
    assert Zn.shape == Zd.shape
    assert rel(Zn, Zd) < 1e-13


def test_dense_contraction_is_iterated_eq8():
    x, y = small_pair(14, [2, 3, 2], [1, 2, 2, 1], [1, 2, 3, 1])
    X, Y = O.tt_full(x), O.tt_full(y)
    # contract position 2 then position 1 one pair at a time with eq. (8)
    Z1 = O.tcp_loops(X, Y, 2, 2)            # (i0, i1, j0, j1)
    Z2 = np.einsum("abcb->ac", Z1)          # pair the remaining shared position
    assert rel(O.contract_dense(x, y, [1, 2]), Z2) < 1e-14


def test_all_modes_is_inner_and_one_block_is_K():
    sx, sy = C.inner4_shapes()
    x = C.gen_tt_np(C.SEED_INNER4, 1, sx)
    y = C.gen_tt_np(C.SEED_INNER4, 2, sy)
    kind, _, K = O.contract_junction(x, y, [0, 1, 2, 3])
    assert kind == "all" and abs(K[0, 0] - O.inner_bruteforce(x, y)) < 1e-12
    # first-core block: K = A_x^T A_y (Example 1)
    kind, k, K1 = O.contract_junction(x, y, [0])
    Ax, Ay = x[0][0], y[0][0]
    assert kind == "prefix" and k == 1
    assert rel(K1, Ax.T @ Ay) < 1e-15 * 8  # same products, summed in another order


def test_natural_ranks_pair10_and_inner4():
    sx, sy = C.pair10_shapes()
    x = [np.zeros(sx.core_shape(k)) for k in range(10)]
    y = [np.zeros(sy.core_shape(k)) for k in range(10)]
    Zn = O.contract_natural(x, y, [0, 1, 2, 3, 4])
    ranks = O.tt_ranks(Zn)
    assert ranks == [1, 1024, 1024, 1024, 1024, 32, 32, 32, 32, 32, 1]
    # 1x16x1024 + 3 x 1024x16x1024 + 1024x16x32 + 4 x 32x16x32 + 32x16x1
    assert sum(G.size for G in Zn) == 16384 + 3 * 16777216 + 524288 + 4 * 16384 + 512
    sx, sy = C.inner4_shapes()
    Zn = O.contract_natural([np.zeros(sx.core_shape(k)) for k in range(4)],
                            [np.zeros(sy.core_shape(k)) for k in range(4)], [2, 3])
    assert O.tt_ranks(Zn) == [1, 4, 4, 16, 1]


# --------------------------------------------------------------- Algorithms 1, 2
def test_tt_svd_exact_and_error_bound():
    rs = np.random.RandomState(7)
    X = rs.randn(4, 5, 3, 4)
    assert rel(O.tt_full(O.tt_svd(X, 0.0)), X) < 1e-13
    # low-rank tensor is recovered at its rank
    x, _ = small_pair(15, [4, 5, 3, 4], [1, 2, 3, 2, 1], [1, 1, 1, 1, 1])
    Xl = O.tt_full(x)
    g = O.tt_svd(Xl, 1e-10)
    assert O.tt_ranks(g) == [1, 2, 3, 2, 1]
    eps = 0.3
    g = O.tt_svd(X, eps)
    assert np.linalg.norm(O.tt_full(g) - X) <= eps * np.linalg.norm(X) * (1 + 1e-12)


def test_ttcp_example1_wiring_and_values():
    with open(os.path.join(GOLD, "example1_shapes.json")) as f:
        g = json.load(f)
    sz = g["sizes"]
    rs = np.random.RandomState(8)
    X = rs.randn(*[sz[m] for m in g["X_modes"]])
    Y = rs.randn(*[sz[m] for m in g["Y_modes"]])
    n, m = g["contract"]["n"] - 1, g["contract"]["m"] - 1
    Z, parts = O.ttcp(X, Y, n, m)
    assert list(Z.shape) == [sz[k] for k in g["Z_modes"]]
    assert list(parts["Zrho"].shape) == [sz[k] for k in g["Zrho_modes"]]
    assert parts["K"].shape == (parts["x_rev"][-1].shape[2], parts["y"][0].shape[0])
    assert rel(Z, O.tcp_loops(X, Y, n, m)) < 1e-12


@pytest.mark.parametrize("dims", [(20, 20, 20), (20, 20, 20, 5)])
def test_ttcp_example2_shapes(dims):
    rs = np.random.RandomState(9)
    X = rs.randn(*dims)
    Y = rs.randn(*dims)
    Z, _ = O.ttcp(X, Y, 0, 0)
    assert rel(Z, O.tcp(X, Y, 0, 0)) < 1e-11


# ------------------------------------------------------------ mode-n products
def test_mode_n_tt_matches_def5_and_identities():
    x, y = small_pair(16, [3, 4, 2], [1, 2, 3, 1], [1, 3, 2, 1])
    X, Y = O.tt_full(x), O.tt_full(y)
    rs = np.random.RandomState(10)
    A = rs.randn(5, 4)
    B = rs.randn(2, 5)
    assert rel(O.tt_full(O.mode_n_tt(x, 1, A)), O.mode_n_loops(X, A, 1)) < 1e-14
    # identity and permutation are exact
    assert all(np.array_equal(a, b) for a, b in zip(O.mode_n_tt(x, 1, np.eye(4)), x))
    P = np.eye(4)[[2, 0, 3, 1]]
    xp = O.mode_n_tt(x, 1, P)
    assert np.array_equal(xp[1], x[1][:, [2, 0, 3, 1], :])
    # composition (X x_n A) x_n B = X x_n (B A)
    lhs = O.tt_full(O.mode_n_tt(O.mode_n_tt(x, 1, A), 1, B))
    assert rel(lhs, O.tt_full(O.mode_n_tt(x, 1, B @ A))) < 1e-13
    # products on different modes commute
    C0 = rs.randn(3, 3)
    a = O.tt_full(O.mode_n_tt(O.mode_n_tt(x, 0, C0), 1, A))
    b = O.tt_full(O.mode_n_tt(O.mode_n_tt(x, 1, A), 0, C0))
    assert rel(a, b) < 1e-13
    # adjoint: <X x_n A, Z> = <X, Z x_n A^T>
    Zt = rs.randn(3, 5, 2)
    lhs = np.sum(O.mode_n_product(X, A, 1) * Zt)
    rhs = np.sum(X * O.mode_n_product(Zt, A.T, 1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ TT-matrix
def test_mpo_full_entrywise():
    sw = C.TTShape([3, 2, 3], [1, 2, 3, 1], [4, 3, 2])
    w = C.gen_tt_np(17, 1, sw)
    Wd = O.mpo_full(w)
    for i in itertools.product(range(3), range(2), range(3)):
        for j in itertools.product(range(4), range(3), range(2)):
            M = np.ones((1, 1))
            for k in range(3):
                M = M @ w[k][:, i[k], j[k], :]
            assert abs(M[0, 0] - Wd[O.lin_index(i, [3, 2, 3]), O.lin_index(j, [4, 3, 2])]) < 1e-14


def test_mpo_tt_identity_kronecker_and_matvec():
    sv = C.TTShape([4, 3, 2], [1, 2, 3, 1])
    v = C.gen_tt_np(18, 2, sv)
    # identity MPO returns V exactly
    ident = [np.eye(d).reshape(1, d, d, 1) for d in sv.modes]
    out = O.mpo_tt(ident, v)
    assert all(np.array_equal(a, b) for a, b in zip(out, v))
    # rank-1 MPO of two factors: (A (x) B) with little-endian vec:
    # W[i0 + I0 i1, j0 + J0 j1] = A0[i0, j0] A1[i1, j1]  => W = kron(A1, A0)
    rs = np.random.RandomState(11)
    A0, A1 = rs.randn(3, 4), rs.randn(2, 3)
    w = [A0.reshape(1, 3, 4, 1), A1.reshape(1, 2, 3, 1)]
    assert np.abs(O.mpo_full(w) - np.kron(A1, A0)).max() == 0.0
    # textbook: kron(A1, A0) vec(X) = vec(A0 X A1^T) (column-major vec)
    Xm = rs.randn(4, 3)
    assert rel(np.kron(A1, A0) @ Xm.reshape(-1, order="F"), (A0 @ Xm @ A1.T).reshape(-1, order="F")) < 1e-14
    # MPO x TT against the dense matvec
    sw = C.TTShape([3, 2, 2], [1, 2, 2, 1], [4, 3, 2])
    w = C.gen_tt_np(18, 1, sw)
    y = O.mpo_tt(w, v)
    assert rel(O.vec(O.tt_full(y)), O.mpo_full(w) @ O.vec(O.tt_full(v))) < 1e-13
    # adjoint: <M v, u> = <v, M^T u>
    u = rs.randn(12)
    Md = O.mpo_full(w)
    vv = O.vec(O.tt_full(v))
    assert abs((Md @ vv) @ u - vv @ (Md.T @ u)) < 1e-12


# --------------------------------------------------------------------- layer
def test_layer_finite_differences_and_euler():
    s = C.layer_fd_shape()
    w = C.gen_tt_np(19, 1, s)
    rs = np.random.RandomState(12)
    X = rs.randn(8, 64)
    T = rs.randn(8, 64)
    r = O.layer_forward_backward(w, X, T)
    h = 1e-3
    worst = 0.0
    for k in range(3):
        g = r["dG"][k]
        for flat in range(0, g.size, 7):
            idx = np.unravel_index(flat, g.shape)
            wp = [G.copy() for G in w]
            wm = [G.copy() for G in w]
            wp[k][idx] += h
            wm[k][idx] -= h
            fd = (O.layer_loss(wp, X, T) - O.layer_loss(wm, X, T)) / (2 * h)
            worst = max(worst, abs(fd - g[idx]) / np.abs(g).max())
    assert worst < 1e-8  # L is quadratic along one parameter: FD exact up to rounding
    for flat in range(0, X.size, 37):
        idx = np.unravel_index(flat, X.shape)
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        fd = (O.layer_loss(w, Xp, T) - O.layer_loss(w, Xm, T)) / (2 * h)
        assert abs(fd - r["dX"][idx]) <= 1e-8 * np.abs(r["dX"]).max()
    # Euler: Y is linear in each core and in X
    e = float(np.sum(r["dX"] * X))
    want = 2.0 / X.size * float(np.sum((r["Y"] - T) * r["Y"]))
    assert abs(e - want) <= 1e-12 * abs(want)
    for k in range(3):
        assert abs(float(np.sum(r["dG"][k] * w[k])) - want) <= 1e-12 * abs(want)


def test_inner_grad_fd_and_euler():
    x, y = small_pair(20, [3, 2, 4, 2], [1, 2, 3, 2, 1], [1, 3, 2, 2, 1])
    dx, dy = O.inner_grad(x, y, gz=1.5)
    z = O.inner_lr(x, y)
    for k in range(4):
        # z is linear in each core: <dz/dG, G> = z
        assert abs(float(np.sum(dx[k] * x[k])) - 1.5 * z) <= 1e-12 * max(1, abs(z))
        assert abs(float(np.sum(dy[k] * y[k])) - 1.5 * z) <= 1e-12 * max(1, abs(z))
    h = 1e-3
    for k in range(4):
        for flat in range(0, x[k].size, 3):
            idx = np.unravel_index(flat, x[k].shape)
            xp = [G.copy() for G in x]
            xm = [G.copy() for G in x]
            xp[k][idx] += h
            xm[k][idx] -= h
            fd = 1.5 * (O.inner_lr(xp, y) - O.inner_lr(xm, y)) / (2 * h)
            assert abs(fd - dx[k][idx]) < 1e-10


# --------------------------------------------------------------- op counts
def test_paper_operation_counts():
    with open(os.path.join(GOLD, "op_counts.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        if "N" in c:
            assert O.tcp_op_count(c["I"], c["N"]) == c["value"]
        else:
            assert O.ttcp_op_count(c["I"], c["R"]) == c["value"]


# --------------------------------------------------------------- generator
def test_generator_reproducible_and_independent():
    a = rng.normal_np(rng.derive_key(1, 2, 3), 1000)
    b = rng.normal_np(rng.derive_key(1, 2, 3), 1000)
    c = rng.normal_np(rng.derive_key(1, 2, 4), 1000)
    assert np.array_equal(a, b)
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.15
    assert abs(a.mean()) < 0.15 and abs(a.std() - 1) < 0.1
    # SplitMix64 reference value: first output of a generator seeded with 0
    # (state += GAMMA, then the finaliser) is 0xE220A8397B1DCDAF
    assert rng.mix64_int(rng.GAMMA) == 0xE220A8397B1DCDAF


def test_generator_numpy_torch_same_integer_stream():
    torch = pytest.importorskip("torch")
    key = rng.derive_key(210900626, 7, 1)
    zn = rng.raw_np(key, 5, 100).view(np.int64)
    zt = rng.raw_t(key, 5, 100, "cpu").numpy()
    assert np.array_equal(zn, zt)


def test_bf16_rne_against_integer_reference():
    rs = np.random.RandomState(13)
    x = np.concatenate([rs.randn(2000).astype(np.float32),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0], dtype=np.float32)])
    got = rng.f32_to_bf16_bits(x)
    for v, g in zip(x, got):
        bits = int(np.float32(v).view(np.uint32))
        hi, lo = bits >> 16, bits & 0xFFFF
        if lo > 0x8000 or (lo == 0x8000 and (hi & 1)):
            hi += 1
        assert g == (hi & 0xFFFF)
    torch = pytest.importorskip("torch")
    t = rng.f32_to_bf16_t(torch.from_numpy(x)).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(t, got)


# ----------------------------------------- contractions at any positions
# (eq. (8) once per pair; Example 1's x_3^2 on cores)
def _tt(seed, obj, modes, ranks):
    return C.gen_tt_np(seed, obj, C.TTShape(list(modes), list(ranks)))


PAIR_CASES = [
    # (X modes, X ranks, Y modes, Y ranks, xmodes, ymodes)
    ([3, 4, 5, 2], [1, 2, 3, 2, 1], [3, 5, 4], [1, 2, 3, 1], [2], [1]),          # Example 1: middle / middle
    ([3, 4, 5, 2], [1, 2, 3, 2, 1], [2, 4, 5, 3], [1, 3, 2, 2, 1], [1, 2], [1, 2]),  # middle blocks of two
    ([4, 3, 2], [1, 2, 3, 1], [2, 4, 3], [1, 3, 2, 1], [0], [1]),                # X prefix, Y middle
    ([3, 2, 4], [1, 2, 2, 1], [4, 3, 2], [1, 2, 3, 1], [2], [0]),                # X suffix, Y prefix
    ([3, 4, 2], [1, 3, 2, 1], [2, 3, 4], [1, 2, 2, 1], [1], [2]),                # X middle, Y suffix
    ([3, 4], [1, 2, 1], [2, 3, 4, 2], [1, 2, 3, 2, 1], [0, 1], [1, 2]),          # X fully, Y middle
    ([3, 4], [1, 2, 1], [3, 4, 2], [1, 2, 3, 1], [0, 1], [0, 1]),                # X fully, Y prefix
    ([3, 4], [1, 2, 1], [2, 3, 4], [1, 2, 3, 1], [0, 1], [1, 2]),                # X fully, Y suffix
    ([2, 3, 4, 2], [1, 2, 3, 2, 1], [3, 4], [1, 2, 1], [1, 2], [0, 1]),          # Y fully, X middle
    ([2, 3, 4], [1, 2, 3, 1], [3, 4], [1, 2, 1], [1, 2], [0, 1]),                # Y fully, X suffix
]


def test_contract_pairs_dense_single_pair_is_literal_eq8():
    rs = np.random.RandomState(31)
    X = rs.randn(3, 4, 5)
    Y = rs.randn(5, 2, 4)
    for n, m in ((2, 0), (1, 2)):
        assert rel(O.contract_pairs_dense(X, Y, [n], [m]), O.tcp_loops(X, Y, n, m)) < 1e-13


def test_contract_pairs_dense_two_pairs_is_eq8_twice():
    rs = np.random.RandomState(32)
    X = rs.randn(3, 4, 5, 2)
    Y = rs.randn(2, 4, 5, 3)
    Z = O.contract_pairs_dense(X, Y, [1, 2], [1, 2])
    # eq. (8) on the pair (2, 2), then on the pair that X's mode 1 and Y's mode 1 became
    Z1 = O.tcp_loops(X, Y, 2, 2)          # modes: X 0,1,3 then Y 0,1,3
    Z2 = np.trace(Z1, axis1=1, axis2=4)  # X's mode 1 against Y's mode 1
    assert rel(Z, Z2) < 1e-13


@pytest.mark.parametrize("case", PAIR_CASES)
def test_contract_pairs_natural_reconstructs_eq8(case):
    mx, rx, my, ry, xm, ym = case
    x, y = _tt(33, 1, mx, rx), _tt(33, 2, my, ry)
    nat = O.contract_pairs_natural(x, y, xm, ym)
    for a, b in zip(nat[:-1], nat[1:]):
        assert a.shape[2] == b.shape[0]
    assert nat[0].shape[0] == 1 and nat[-1].shape[2] == 1
    want = O.contract_pairs_dense(O.tt_full(x), O.tt_full(y), xm, ym)
    assert rel(O.tt_full(nat), want) < 1e-12


def test_transfer_junction_ends_are_the_sweep_interfaces():
    x, y = small_pair(34, [3, 4, 2, 5], [1, 2, 3, 4, 1], [1, 3, 2, 2, 1])
    for k in (1, 2, 3):
        W = O.sweep_lr(x, y, upto=k)[-1]
        # a prefix block's T is 1 x (R_k P_k): W_k's entries, row-major
        T = O.transfer_junction(x, y, list(range(k)), list(range(k)))
        assert T.shape == (1, W.size) and rel(T.reshape(W.shape), W) < 1e-13
        V = O.sweep_rl(x, y, downto=k)[k]
        T = O.transfer_junction(x, y, list(range(k, 4)), list(range(k, 4)))
        assert T.shape == (V.size, 1) and rel(T.reshape(V.shape), V) < 1e-13
    # the general construction at equal prefix / suffix blocks is the pinned one
    for modes in ([0, 1], [0], [2, 3], [3]):
        got = O.contract_pairs_natural(x, y, modes, modes)
        want = O.contract_natural(x, y, modes)
        assert len(got) == len(want)
        assert all(g.shape == w.shape and rel(g, w) < 1e-13 for g, w in zip(got, want))


def test_contract_pairs_example1_on_cores_matches_ttcp():
    with open(os.path.join(GOLD, "example1_shapes.json")) as f:
        g = json.load(f)
    sz = g["sizes"]
    rs = np.random.RandomState(35)
    X = rs.randn(*[sz[m] for m in g["X_modes"]])
    Y = rs.randn(*[sz[m] for m in g["Y_modes"]])
    n, m = g["contract"]["n"] - 1, g["contract"]["m"] - 1
    Z, _ = O.ttcp(X, Y, n, m)
    x, y = O.tt_svd(X), O.tt_svd(Y)
    assert rel(O.tt_full(O.contract_pairs_natural(x, y, [n], [m])), Z) < 1e-12
