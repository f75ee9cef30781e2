"""FP64 CPU oracle for tensor contraction products on Tensor-Train cores.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may import, call or
link this module: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the GPU path.

Everything here is plain float64 NumPy written from the paper's definitions
(Kisil, Calvi, Konstantinidis, Xu, Mandic, "Reducing Computational Complexity
of Tensor Contractions via Tensor-Train Networks", arXiv 2109.00626).  A
library matmul / tensordot / SVD serves as a step where the definition calls
for that operation; there is no blocking or fusion beyond the definitions.

Index conventions (shared with the library, fixed by the paper):
  * flat (vectorised) indices are little-endian: first index fastest
    (Def. 2, eq. (2) first line, and Def. 3), 0-based here;
  * a TT is a list of cores, core k a (R_k, I_k, R_{k+1}) array with
    R_0 = R_N = 1 (Def. 7, eq. (9); Example 1);
  * a TT-matrix (MPO) core k is (R_k, I_k, J_k, R_{k+1}); its dense matrix has
    rows i = little-endian(i_1..i_N) and columns j = little-endian(j_1..j_N).

Readings of passages the paper leaves open are listed where they are used.
Every function here is pinned by a test against something other than itself
(brute force, closed forms, invariants, the paper's printed counts).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# =========================================================================
# Section II-A: basic tensor definitions
# =========================================================================
def lin_index(idx, dims) -> int:
    """Little-endian linear index, 0-based (Def. 2, eq. (2), first line):
    i = sum_n i_n * prod_{k<n} I_k.  The second line of eq. (2) is garbled
    (an extra '1 +' and i_n where i_N is meant); the first line and Def. 3
    agree, so they are taken."""
    out, stride = 0, 1
    for i, d in zip(idx, dims):
        out += int(i) * stride
        stride *= int(d)
    return out


def vec(X: np.ndarray) -> np.ndarray:
    """Vectorisation with the little-endian index of Def. 3 (first index fastest)."""
    return np.asarray(X).reshape(-1, order="F")


def fold(x: np.ndarray, dims) -> np.ndarray:
    """Folding of a vector into a tensor (Def. 3, eq. (3))."""
    return np.asarray(x).reshape(tuple(dims), order="F")


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding (Def. 2): row index i_n, column index the
    little-endian linear index of the remaining modes in increasing order."""
    Xn = np.moveaxis(X, n, 0)
    return Xn.reshape(X.shape[n], -1, order="F")


def refold(M: np.ndarray, n: int, dims) -> np.ndarray:
    """Inverse of unfold for a tensor of shape dims."""
    dims = list(dims)
    rest = [dims[n]] + dims[:n] + dims[n + 1:]
    return np.moveaxis(M.reshape(rest, order="F"), 0, n)


def stack(samples) -> np.ndarray:
    """Stacking of J order-N samples along a new last mode (Def. 4)."""
    return np.stack(samples, axis=-1)


def mode_n_product(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """Mode-n product Y = X x_n A (Def. 5): unfold, multiply by A, fold."""
    dims = list(X.shape)
    Yn = A @ unfold(X, n)
    dims[n] = A.shape[0]
    return refold(Yn, n, dims)


def tcp(X: np.ndarray, Y: np.ndarray, n: int, m: int) -> np.ndarray:
    """(n, m)-contraction of Def. 6, eq. (8), 0-based modes: the sum over the
    common index; output modes are X's free modes then Y's free modes.  The
    subscript brace of eq. (8) is misplaced in the paper; the standard
    sum_i x[..i..] y[..i..] is meant."""
    return np.tensordot(X, Y, axes=([n], [m]))


def tcp_loops(X: np.ndarray, Y: np.ndarray, n: int, m: int) -> np.ndarray:
    """eq. (8) written out element by element (pure Python; tiny inputs only)."""
    fx = [d for k, d in enumerate(X.shape) if k != n]
    fy = [d for k, d in enumerate(Y.shape) if k != m]
    Z = np.zeros(fx + fy)
    for ix in itertools.product(*[range(d) for d in fx]):
        for iy in itertools.product(*[range(d) for d in fy]):
            s = 0.0
            for c in range(X.shape[n]):
                xi = ix[:n] + (c,) + ix[n:]
                yi = iy[:m] + (c,) + iy[m:]
                s += X[xi] * Y[yi]
            Z[ix + iy] = s
    return Z


def contract_positions(X: np.ndarray, Y: np.ndarray, positions) -> np.ndarray:
    """Contraction of X and Y over a set of shared positions: eq. (8) applied
    once per pair of equal positions (the order of the pairs does not
    matter).  The paper defines a single pair; a set of pairs is read as
    eq. (8) iterated.  Output: X's free modes, then Y's, each in order."""
    positions = list(positions)
    return np.tensordot(X, Y, axes=(positions, positions))


# =========================================================================
# Def. 7, eq. (9): the TT format
# =========================================================================
def tt_full(cores) -> np.ndarray:
    """Dense tensor of a TT: X = G1 x_2^1 G2 x_3^1 G3 ... (eq. (9)), each step
    a contraction (Def. 6) of the running tensor's last mode with the next
    core's first mode; the two boundary rank-1 modes are dropped at the end."""
    Z = cores[0]
    for G in cores[1:]:
        Z = tcp(Z, G, Z.ndim - 1, 0)
    return Z.reshape(Z.shape[1:-1])


def tt_entry(cores, idx) -> float:
    """One entry of a TT: product of the core slices G_k[:, i_k, :] (eq. (9)),
    written as explicit loops (tiny inputs only)."""
    v = [1.0]
    for G, i in zip(cores, idx):
        r0, _, r1 = G.shape
        nv = [0.0] * r1
        for b in range(r1):
            s = 0.0
            for a in range(r0):
                s += v[a] * G[a, i, b]
            nv[b] = s
        v = nv
    return v[0]


def tt_norm2_dense(cores) -> float:
    X = tt_full(cores)
    return float(np.sum(X * X))


def tt_ranks(cores):
    return [cores[0].shape[0]] + [G.shape[-1] for G in cores]


def tt_modes(cores):
    return [G.shape[1] for G in cores]


# =========================================================================
# Algorithm 1: TT-SVD
# =========================================================================
def tt_svd(X: np.ndarray, eps: float = 0.0):
    """TT-SVD (Algorithm 1): delta = eps / sqrt(N-1) * ||X||_F, then N-1
    delta-truncated SVDs of the running unfolding; the truncation keeps the
    smallest rank whose discarded singular values have norm <= delta.  The
    update uses S V^T (the paper's 'USV' misses the transpose)."""
    dims = X.shape
    N = len(dims)
    delta = eps / math.sqrt(max(N - 1, 1)) * np.linalg.norm(X)
    cores = []
    r_prev = 1
    # the running tensor keeps (R_{n-1}, I_n, rest) so that a row-major
    # reshape gives the unfolding whose rows are (r, i_n)
    Zt = X.reshape((1,) + dims)
    for n in range(N - 1):
        M = Zt.reshape(r_prev * dims[n], -1)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        tail2 = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])  # ||s[r:]||^2
        r = next(c for c in range(1, len(s) + 1) if math.sqrt(tail2[c]) <= delta)
        cores.append(U[:, :r].reshape(r_prev, dims[n], r))
        Zt = (s[:r, None] * Vt[:r]).reshape((r,) + dims[n + 1:])
        r_prev = r
    cores.append(Zt.reshape(r_prev, dims[-1], 1))
    return cores


# =========================================================================
# Section III, Algorithm 2: TTCP on dense inputs
# =========================================================================
def ttcp(X: np.ndarray, Y: np.ndarray, n: int, m: int, eps: float = 0.0):
    """Tensor-Train Contraction Product (Algorithm 2), 0-based n, m.

    1. permute X so that mode n comes first (X^rho), same for Y with mode m;
    2. TT-decompose both (Algorithm 1);
    3. K = A_x^T A_y with A_x = G_x^(1) as an I_n x R_1 matrix (Example 1;
       the paper labels A_x as I_1 x R_1, the contracted mode is meant);
    4. Z^rho: X's remaining cores in reverse order, each transposed by
       T_[1;3] (first and third modes exchanged), then K, then Y's cores;
    5. permute Z^rho into the order of eq. (8).
    Returns (Z, parts) where parts holds K and the cores of Z^rho."""
    N, M = X.ndim, Y.ndim
    px = [n] + [k for k in range(N) if k != n]
    py = [m] + [k for k in range(M) if k != m]
    Xr = np.transpose(X, px)
    Yr = np.transpose(Y, py)
    gx = tt_svd(Xr, eps)
    gy = tt_svd(Yr, eps)
    Ax = gx[0][0]            # I_n x R_1
    Ay = gy[0][0]            # J_m x P_1
    K = Ax.T @ Ay            # R_1 x P_1
    # X side reversed, cores transposed by T_[1;3]: (R_k, I, R_{k-1})
    xs = [np.transpose(G, (2, 1, 0)) for G in gx[1:][::-1]]
    ys = list(gy[1:])
    # Z^rho network: xs[0] ... xs[-1] -- K -- ys[0] ... ys[-1]
    Zr = xs[0]
    for G in xs[1:]:
        Zr = tcp(Zr, G, Zr.ndim - 1, 0)
    Zr = tcp(Zr, K, Zr.ndim - 1, 0)
    for G in ys:
        Zr = tcp(Zr, G, Zr.ndim - 1, 0)
    Zr = Zr.reshape(Zr.shape[1:-1])
    # Z^rho modes: X free modes in reverse order (of X^rho's), then Y's free modes
    xf = px[1:][::-1]
    nx = len(xf)
    # natural order: X free modes increasing, then Y's
    perm = [xf.index(k) for k in sorted(xf)] + [nx + j for j in range(M - 1)]
    Z = np.transpose(Zr, perm)
    return Z, {"K": K, "x_rev": xs, "y": ys, "Zrho": Zr}


# =========================================================================
# Interface sweeps on given cores (inner products, partial contractions)
# =========================================================================
def sweep_lr(x, y, upto=None):
    """Left-to-right interfaces W_0 .. W_upto with W_0 = [1] and
    W_k = sum_i G_x^(k)[:, i, :]^T W_{k-1} G_y^(k)[:, i, :]  (R_k x P_k).
    W_1 is the paper's K = A_x^T A_y (Example 1) for the first core pair."""
    N = len(x)
    upto = N if upto is None else upto
    Ws = [np.ones((1, 1))]
    for k in range(upto):
        Gx, Gy = x[k], y[k]
        W = np.zeros((Gx.shape[2], Gy.shape[2]))
        for i in range(Gx.shape[1]):
            W += Gx[:, i, :].T @ Ws[-1] @ Gy[:, i, :]
        Ws.append(W)
    return Ws


def sweep_rl(x, y, downto=0):
    """Right-to-left interfaces V_N .. V_downto with V_N = [1] and
    V_{k} = sum_i G_x^(k)[:, i, :] V_{k+1} G_y^(k)[:, i, :]^T  (R_k x P_k),
    returned as a dict {k: V_k}."""
    N = len(x)
    Vs = {N: np.ones((1, 1))}
    for k in range(N - 1, downto - 1, -1):
        Gx, Gy = x[k], y[k]
        V = np.zeros((Gx.shape[0], Gy.shape[0]))
        for i in range(Gx.shape[1]):
            V += Gx[:, i, :] @ Vs[k + 1] @ Gy[:, i, :].T
        Vs[k] = V
    return Vs


def inner_lr(x, y) -> float:
    """<X, Y> by the left-to-right sweep: the all-mode contraction of Fig. 1(b)."""
    return float(sweep_lr(x, y)[-1][0, 0])


def inner_rl(x, y) -> float:
    return float(sweep_rl(x, y)[0][0, 0])


def inner_meet(x, y, c: int) -> float:
    """<X, Y> = sum_{r,p} W_c[r,p] V_c[r,p] for a meeting bond c (0 < c < N)."""
    W = sweep_lr(x, y, upto=c)[-1]
    V = sweep_rl(x, y, downto=c)[c]
    return float(np.sum(W * V))


def inner_dense(x, y) -> float:
    """<X, Y> from the dense tensors (eq. (9) reconstruction, then the sum)."""
    return float(np.sum(tt_full(x) * tt_full(y)))


def inner_bruteforce(x, y) -> float:
    """Literal sum over every multi-index of X[i] * Y[i] (tiny inputs)."""
    modes = tt_modes(x)
    s = 0.0
    for idx in itertools.product(*[range(d) for d in modes]):
        s += tt_entry(x, idx) * tt_entry(y, idx)
    return s


def block_kind(N: int, modes) -> tuple:
    """Classify a set of shared 0-based positions as ('prefix', k) for
    {0..k-1}, ('suffix', k) for {k..N-1}, ('all', N), or ('other', None)."""
    s = sorted(set(int(m) for m in modes))
    if len(s) == N and s == list(range(N)):
        return ("all", N)
    if s and s == list(range(len(s))):
        return ("prefix", len(s))
    if s and s == list(range(N - len(s), N)):
        return ("suffix", N - len(s))
    return ("other", None)


def contract_junction(x, y, modes):
    """Junction form of a shared-block contraction: the matrix K that joins
    X's free cores to Y's free cores (the 'K' node of Fig. 3).  Prefix
    {0..k-1}: K = W_k.  Suffix {k..N-1}: K = V_k.  All modes: the scalar."""
    kind, k = block_kind(len(x), modes)
    if kind == "all":
        return kind, k, np.array([[inner_lr(x, y)]])
    if kind == "prefix":
        return kind, k, sweep_lr(x, y, upto=k)[-1]
    if kind == "suffix":
        return kind, k, sweep_rl(x, y, downto=k)[k]
    raise ValueError("junction form needs a prefix, suffix or all modes")


def contract_natural(x, y, modes):
    """Natural-order TT of the contraction (eq. (8) mode order: X's free modes,
    then Y's).  Reading adopted for the construction, so that outputs compare
    core by core: merged bond index = (own bond) * Q + q, where q is the
    carried index of K (Q = its size).

    Prefix {0..k-1} (K = W_k, R_k x P_k):
      C_k[0, i, s*Q + q]   = sum_r K[r, q] G_x^(k)[r, i, s]
      C_m[(s,q), i, (s',q')] = G_x^(m)[s, i, s'] delta(q, q')   (k < m < N)
      the last X core ends with bond q (size Q = P_k), then Y's cores k..N-1.
    Suffix {k..N-1} (K = V_k):
      X's cores 0..k-2 unchanged; C_{k-1}[s, i, q] = sum_r G_x^(k-1)[s, i, r] K[r, q];
      Y's cores lifted: D_0[q, j, p*Q + q'] = G_y^(0)[0, j, p] delta(q, q'),
      D_m[(p,q), j, (p',q')] = G_y^(m)[p, j, p'] delta(q, q'),
      D_{k-1}[(p,q), j, 0] = G_y^(k-1)[p, j, q].
    """
    N = len(x)
    kind, k = block_kind(N, modes)
    _, _, K = contract_junction(x, y, modes)
    Q = K.shape[1]
    out = []
    if kind == "prefix":
        if k == N:
            raise ValueError("all modes give a scalar")
        for m in range(k, N):
            G = x[m]
            r0, I, r1 = G.shape
            if m == k:
                C = np.einsum("rq,ris->isq", K, G).reshape(1, I, r1 * Q)
            else:
                C = np.einsum("ais,qt->aqist", G, np.eye(Q)).reshape(r0 * Q, I, r1 * Q)
            out.append(C)
        out.extend(G.copy() for G in y[k:])
        return out
    if kind == "suffix":
        if k == 0:
            raise ValueError("all modes give a scalar")
        out.extend(G.copy() for G in x[: k - 1])
        out.append(np.einsum("sir,rq->siq", x[k - 1], K))
        for m in range(k):
            G = y[m]
            p0, J, p1 = G.shape
            if m == k - 1:
                # right bond of the last free Y core is the carried index q
                D = np.einsum("pjq->pqj", G).reshape(p0 * Q, J, 1)
            else:
                D = np.einsum("ajp,qt->aqjpt", G, np.eye(Q)).reshape(p0 * Q, J, p1 * Q)
            out.append(D)
        return out
    raise ValueError("natural form needs a prefix or suffix block")


def contract_dense(x, y, modes) -> np.ndarray:
    """Dense result of the shared-position contraction, from the definitions
    only: reconstruct both tensors (eq. (9)) and apply eq. (8) per pair."""
    return contract_positions(tt_full(x), tt_full(y), modes)


# =========================================================================
# Contractions of X's modes a1..a2 with Y's modes b1..b2 at any positions
# (eq. (8) once per pair; Example 1's X x_3^2 Y is a1 = a2 = 2, b1 = b2 = 1)
# =========================================================================
def contract_pairs_dense(X: np.ndarray, Y: np.ndarray, xmodes, ymodes) -> np.ndarray:
    """eq. (8) applied once per pair (X's mode xmodes[l] with Y's ymodes[l]),
    0-based; output modes: X's free modes, then Y's, each in order."""
    return np.tensordot(X, Y, axes=(list(xmodes), list(ymodes)))


def block_product(cores, lo: int, hi: int) -> np.ndarray:
    """Cores lo..hi multiplied along their shared bonds (eq. (9)'s product of
    slices, kept open at both ends): shape (R_lo, I_lo, ..., I_hi, R_{hi+1})."""
    B = cores[lo]
    for k in range(lo + 1, hi + 1):
        B = np.tensordot(B, cores[k], axes=([B.ndim - 1], [0]))
    return B


def transfer_junction(x, y, xmodes, ymodes) -> np.ndarray:
    """Junction of a contraction over consecutive blocks: with a, b X's bonds
    before and after its block and g, d Y's,
      T[(a, g), (b, d)] = sum over the block indices of Xblock[a, i.., b] Yblock[g, i.., d],
    rows a * |g| + g, columns b * |d| + d.  A prefix block gives W_k, a
    suffix block V_k (the matrix K of Example 1 / Fig. 3)."""
    a1, a2 = int(xmodes[0]), int(xmodes[-1])
    b1, b2 = int(ymodes[0]), int(ymodes[-1])
    L = a2 - a1 + 1
    Xb = block_product(x, a1, a2)
    Yb = block_product(y, b1, b2)
    T = np.tensordot(Xb, Yb, axes=(list(range(1, L + 1)), list(range(1, L + 1))))  # (a, b, g, d)
    ka, kb, kg, kd = T.shape
    return np.transpose(T, (0, 2, 1, 3)).reshape(ka * kg, kb * kd)


def contract_pairs_natural(x, y, xmodes, ymodes):
    """Natural-order TT (eq. (8) mode order) of the contraction over the
    blocks, with the junction's Y-side indices q = g * |d| + d carried as an
    extra bond factor (merged index (own bond) * Q + q, Q = |g| |d|):
      X's cores left of the block are copied (the last absorbs T when X has
      no cores right of the block: C[s, i, q] = sum_a G[s, i, a] T[(a, g), d]);
      the first X core right of the block absorbs T:
        C[a, i, s*Q + q] = sum_b T[(a, g), (b, d)] G[b, i, s];
      the other X cores right of it: C[(s,q), i, (s',q')] = G[s, i, s'] delta(q, q');
      Y's cores left of its block carry q; the last of them contracts g:
        D[(p,q), j, d'] = G[p, j, g] delta(d, d');
      Y's cores right of its block are copied.
    X fully contracted: T (|g| x |d|) is absorbed into the last Y core left
    of the block (D[p, j, d] = sum_g G[p, j, g] T[g, d]), or, with none, into
    the first core right of it (D[0, j, s] = sum_d T[0, d] G[d, j, s])."""
    N, M = len(x), len(y)
    a1, a2 = int(xmodes[0]), int(xmodes[-1])
    b1, b2 = int(ymodes[0]), int(ymodes[-1])
    ka, kb = x[a1].shape[0], x[a2].shape[2]
    kg, kd = y[b1].shape[0], y[b2].shape[2]
    T4 = transfer_junction(x, y, xmodes, ymodes).reshape(ka, kg, kb, kd)
    out = []
    xfree = a1 > 0 or a2 < N - 1
    if xfree:
        Q = kg * kd
        for m in range(a1):
            G = x[m]
            if a2 == N - 1 and m == a1 - 1:
                out.append(np.einsum("sia,agd->sigd", G, T4[:, :, 0, :]).reshape(G.shape[0], G.shape[1], Q))
            else:
                out.append(G.copy())
        for m in range(a2 + 1, N):
            G = x[m]
            r0, I, r1 = G.shape
            if m == a2 + 1:
                out.append(np.einsum("agbd,bis->aisgd", T4, G).reshape(ka, I, r1 * Q))
            else:
                out.append(np.einsum("sit,qu->sqitu", G, np.eye(Q)).reshape(r0 * Q, I, r1 * Q))
        for m in range(b1):
            G = y[m]
            p0, J, p1 = G.shape
            if m == b1 - 1:
                D = np.einsum("pjg,de->pgdje", G, np.eye(kd)).reshape(p0 * Q, J, kd)
            else:
                D = np.einsum("pjt,qu->pqjtu", G, np.eye(Q)).reshape(p0 * Q, J, p1 * Q)
            out.append(D)
        out.extend(G.copy() for G in y[b2 + 1:])
        return out
    if b1 == 0 and b2 == M - 1:
        raise ValueError("every mode of both contracted: the scalar <X, Y>")
    T = T4[0, :, 0, :]  # (g, d)
    for m in range(b1):
        G = y[m]
        out.append(np.einsum("pjg,gd->pjd", G, T) if m == b1 - 1 else G.copy())
    for m in range(b2 + 1, M):
        G = y[m]
        if b1 == 0 and m == b2 + 1:
            out.append(np.einsum("d,djs->js", T[0], G)[None])
        else:
            out.append(G.copy())
    return out


# =========================================================================
# Def. 5 on a TT: mode-n product rewrites one core
# =========================================================================
def mode_n_tt(x, n: int, A: np.ndarray):
    """TT of X x_n A: core n becomes G'[r, j, s] = sum_i A[j, i] G[r, i, s];
    every other core is unchanged (Def. 5 applied to eq. (9))."""
    out = [G.copy() for G in x]
    out[n] = np.einsum("ji,ris->rjs", A, x[n])
    return out


def mode_n_loops(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """Def. 5 written element by element (tiny inputs)."""
    dims = list(X.shape)
    dims[n] = A.shape[0]
    Y = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for i in range(X.shape[n]):
            src = idx[:n] + (i,) + idx[n + 1:]
            s += A[idx[n], i] * X[src]
        Y[idx] = s
    return Y


# =========================================================================
# TT-matrix (MPO) products
# =========================================================================
def mpo_full(w) -> np.ndarray:
    """Dense matrix of a TT-matrix: W[i, j] = prod_k W^(k)[:, i_k, j_k, :] with
    row i and column j little-endian over (i_1..i_N), (j_1..j_N) (Def. 3)."""
    N = len(w)
    T = w[0]
    for G in w[1:]:
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    T = T.reshape(T.shape[1:-1])  # (i1, j1, i2, j2, ..., iN, jN)
    rows = [w[k].shape[1] for k in range(N)]
    cols = [w[k].shape[2] for k in range(N)]
    # order axes as (iN .. i1, jN .. j1) so that a row-major reshape gives
    # little-endian flat indices
    perm = [2 * k for k in reversed(range(N))] + [2 * k + 1 for k in reversed(range(N))]
    return np.transpose(T, perm).reshape(int(np.prod(rows)), int(np.prod(cols)))


def mpo_tt(w, v):
    """TT-matrix x TT-vector on cores: C^(k)[(a,r), i, (a',r')] =
    sum_j W^(k)[a, i, j, a'] V^(k)[r, j, r'], merged bond a*R_v + r."""
    out = []
    for W, V in zip(w, v):
        a0, I, J, a1 = W.shape
        r0, J2, r1 = V.shape
        assert J == J2
        C = np.einsum("aijb,rjs->aribs", W, V).reshape(a0 * r0, I, a1 * r1)
        out.append(C)
    return out


def mpo_apply_dense_vector(w, xvec: np.ndarray) -> np.ndarray:
    return mpo_full(w) @ xvec


# =========================================================================
# TT layer: y = W x per row, MSE loss, gradients (dense route, FP64)
# =========================================================================
def layer_forward(w, X: np.ndarray):
    """Y = X W^T for a batch X (B x prod J), rows little-endian vectors."""
    return X @ mpo_full(w).T


def mse_loss(Y: np.ndarray, T: np.ndarray):
    """L = mean((Y - T)^2) over every entry; dL/dY = 2 (Y - T) / numel."""
    D = Y - T
    return float(np.mean(D * D)), 2.0 * D / D.size


def mpo_core_grads_from_dense(w, dW: np.ndarray):
    """Project a gradient with respect to the dense matrix W onto every core:
    dG^(k) = sum over all (i, j) of dW[i, j] * dW[i, j]/dG^(k), where W[i, j]
    is the product of core slices, so the derivative is the product of the
    slices left of k (row r) and right of k (column s)."""
    N = len(w)
    rows = [G.shape[1] for G in w]
    cols = [G.shape[2] for G in w]
    # dense gradient as a tensor over (i_1..i_N, j_1..j_N)
    D = dW.reshape(list(reversed(rows)) + list(reversed(cols)))
    D = np.transpose(D, list(reversed(range(N))) + [N + k for k in reversed(range(N))])
    grads = []
    for k in range(N):
        # left partial product: (i_<k, j_<k, r)
        L = np.ones((1,))
        lshape = []
        for m in range(k):
            L = np.tensordot(L, w[m], axes=([L.ndim - 1], [0]))
            lshape += [rows[m], cols[m]]
        L = L.reshape(lshape + [w[k].shape[0]]) if k > 0 else np.ones((1,))
        Rt = np.ones((1,))
        for m in range(N - 1, k, -1):
            Rt = np.tensordot(w[m], Rt, axes=([3], [0]))
        # Rt: (s, i_{k+1}, j_{k+1}, ..., i_N, j_N) or (1,) if k == N-1
        # move D axes to (i_1, j_1, ..., i_N, j_N)
        perm = []
        for m in range(N):
            perm += [m, N + m]
        Dp = np.transpose(D, perm)
        # contract left
        if k > 0:
            Dp = np.tensordot(L, Dp, axes=(list(range(2 * k)), list(range(2 * k))))
        else:
            Dp = Dp[None]
        # Dp: (r, i_k, j_k, i_{k+1}, j_{k+1}, ...)
        if k < N - 1:
            nrest = 2 * (N - 1 - k)
            Dp = np.tensordot(Dp, Rt, axes=(list(range(3, 3 + nrest)), list(range(1, 1 + nrest))))
        else:
            Dp = Dp[..., None]
        grads.append(Dp)
    return grads


def layer_forward_backward(w, X: np.ndarray, T: np.ndarray):
    """Dense route in FP64: Y, L, dY, dX = dY W, dW = dY^T X, dG^(k)."""
    Wd = mpo_full(w)
    Y = X @ Wd.T
    L, dY = mse_loss(Y, T)
    dX = dY @ Wd
    dW = dY.T @ X
    dG = mpo_core_grads_from_dense(w, dW)
    return {"Y": Y, "L": L, "dY": dY, "dX": dX, "dG": dG}


def layer_loss(w, X, T) -> float:
    return mse_loss(layer_forward(w, X), T)[0]


# =========================================================================
# Gradient of the inner product with respect to every core
# =========================================================================
def inner_grad(x, y, gz: float = 1.0):
    """d<X,Y>/dG_x^(k)[:, i, :] = W_{k-1} G_y^(k)[:, i, :] V_{k+1}^T and
    d<X,Y>/dG_y^(k)[:, i, :] = W_{k-1}^T G_x^(k)[:, i, :] V_{k+1}, scaled by
    the upstream gradient gz (W from the left sweep, V from the right)."""
    N = len(x)
    Ws = sweep_lr(x, y)
    Vs = sweep_rl(x, y)
    dx, dy = [], []
    for k in range(N):
        Wl, Vr = Ws[k], Vs[k + 1]
        gx = np.zeros_like(x[k])
        gy = np.zeros_like(y[k])
        for i in range(x[k].shape[1]):
            gx[:, i, :] = gz * (Wl @ y[k][:, i, :] @ Vr.T)
            gy[:, i, :] = gz * (Wl.T @ x[k][:, i, :] @ Vr)
        dx.append(gx)
        dy.append(gy)
    return dx, dy


# =========================================================================
# Operation-count model of Section IV
# =========================================================================
def tcp_op_count(I: int, N: int) -> int:
    """Dense contraction of two order-N tensors with all modes I: I^(2N-1)."""
    return I ** (2 * N - 1)


def ttcp_op_count(I: int, R: int) -> int:
    """TTCP's single K product: I * R^2 (R_1 = P_1 = R)."""
    return I * R * R
