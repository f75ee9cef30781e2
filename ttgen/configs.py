"""Seeded synthetic workloads: shapes and values of every TT, TT-matrix and
dense operand used by the tests and the benchmark.

Conventions (also those of the library):
  * a TT of order N has mode sizes I[0..N-1] and ranks R[0..N], R[0] = R[N] = 1;
    core k is a row-major (R[k], I[k], R[k+1]) array;
  * a TT-matrix (MPO) core k is a row-major (R[k], I[k], J[k], R[k+1]) array;
  * core entries are iid N(0, sigma2) with sigma2 = 1 / max(R[k], R[k+1]).

Workloads (sizes as named):
  inner4  : order-4 pair, modes 8, ranks 4, FP64, plus an 8x8 matrix
  pair10  : order-10 pair, modes 16, ranks 32, FP32, plus ten 16x16 matrices
  mpo8    : order-8 MPO (I = J = 32, rank 16) and order-8 TT-vector (mode 32, rank 64), BF16
  batch4096 : 4096 pairs of uneven order / modes / ranks, FP32 and BF16
  layer4  : order-4 TT-matrix 4096 -> 4096 (modes 8, ranks 32), batch 8192 x 4096
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import rng

BASE_SEED = 210900626
SEED_INNER4 = BASE_SEED + 1
SEED_PAIR10 = BASE_SEED + 2
SEED_MPO8 = BASE_SEED + 3
SEED_BATCH = BASE_SEED + 4
SEED_LAYER = BASE_SEED + 5

C4_MODE_CHOICES = (4, 8, 16, 32, 64)


@dataclass
class TTShape:
    modes: list
    ranks: list
    cols: list | None = None  # TT-matrix column modes (None for a TT-vector)

    @property
    def order(self) -> int:
        return len(self.modes)

    def core_shape(self, k: int) -> tuple:
        if self.cols is None:
            return (self.ranks[k], self.modes[k], self.ranks[k + 1])
        return (self.ranks[k], self.modes[k], self.cols[k], self.ranks[k + 1])

    def core_numel(self, k: int) -> int:
        return int(np.prod(self.core_shape(k)))

    def numel(self) -> int:
        return sum(self.core_numel(k) for k in range(self.order))


def sigma2_of(shape: TTShape, k: int) -> float:
    return 1.0 / max(shape.ranks[k], shape.ranks[k + 1])


def gen_tt_np(seed: int, obj: int, shape: TTShape, sigma2=None) -> list:
    """FP64 cores (list of numpy arrays) for object `obj` under `seed`."""
    cores = []
    for k in range(shape.order):
        s2 = sigma2_of(shape, k) if sigma2 is None else sigma2
        v = rng.normal_np(rng.derive_key(seed, obj, k), shape.core_numel(k))
        cores.append((v * math.sqrt(s2)).reshape(shape.core_shape(k)))
    return cores


def gen_matrix_np(seed: int, obj: int, rows: int, cols: int, scale: float = 1.0) -> np.ndarray:
    v = rng.normal_np(rng.derive_key(seed, obj, 0), rows * cols)
    return (v * scale).reshape(rows, cols)


def gen_int_tt_np(seed: int, obj: int, shape: TTShape) -> list:
    """Cores with entries in {-1, 0, 1} (exact in every precision)."""
    cores = []
    for k in range(shape.order):
        v = rng.uniform_int_np(rng.derive_key(seed, obj, k), shape.core_numel(k), -1, 1)
        cores.append(v.astype(np.float64).reshape(shape.core_shape(k)))
    return cores


def uniform_shape(order: int, mode: int, rank: int, cols: int | None = None) -> TTShape:
    ranks = [1] + [rank] * (order - 1) + [1]
    return TTShape([mode] * order, ranks, None if cols is None else [cols] * order)


# ------------------------------------------------------------- named workloads
def inner4_shapes():
    return uniform_shape(4, 8, 4), uniform_shape(4, 8, 4)


def pair10_shapes():
    return uniform_shape(10, 16, 32), uniform_shape(10, 16, 32)


def mpo8_shapes():
    return uniform_shape(8, 32, 16, cols=32), uniform_shape(8, 32, 64)


def layer4_shape():
    return uniform_shape(4, 8, 32, cols=8)


def layer_fd_shape():
    return uniform_shape(3, 4, 4, cols=4)


def batch_pair_shapes(seed: int, n_pairs: int):
    """Shapes of the uneven batch: order U{3..12}; modes uniform over
    {4,8,16,32,64} per position (shared by X and Y); ranks per bond
    round(exp(U[ln 8, ln 128])), drawn independently for X and Y."""
    out = []
    lo, hi = math.log(8.0), math.log(128.0)
    for p in range(n_pairs):
        u = rng.uniform_np(rng.derive_key(seed, 0, p), 40)
        order = 3 + int(math.floor(u[0] * 10))
        modes = [C4_MODE_CHOICES[int(math.floor(u[1 + k] * 5))] for k in range(order)]
        rx = [1] + [int(round(math.exp(lo + u[13 + k] * (hi - lo)))) for k in range(order - 1)] + [1]
        ry = [1] + [int(round(math.exp(lo + u[26 + k] * (hi - lo)))) for k in range(order - 1)] + [1]
        out.append((TTShape(modes, rx), TTShape(list(modes), ry)))
    return out


# ------------------------------------------------------------- torch fillers
def gen_tt_torch(seed: int, obj: int, shape: TTShape, device, dtype):
    """Same values as gen_tt_np (up to the last bit of Box-Muller), produced on
    `device`; FP64 -> dtype with RNE (BF16 through FP32)."""
    import torch
    cores = []
    for k in range(shape.order):
        v = rng.normal_t(rng.derive_key(seed, obj, k), shape.core_numel(k), device)
        v = v * math.sqrt(sigma2_of(shape, k))
        cores.append(cast_t(v, dtype).reshape(shape.core_shape(k)))
    return cores


def gen_matrix_torch(seed: int, obj: int, rows: int, cols: int, device, dtype, chunk=1 << 26):
    import torch
    key = rng.derive_key(seed, obj, 0)
    n = rows * cols
    out = torch.empty(n, dtype=dtype, device=device)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        u = rng.uniform_t(key, 2 * c, device, start=2 * s)
        v = torch.sqrt(-2.0 * torch.log(1.0 - u[0::2])) * torch.cos(2.0 * np.pi * u[1::2])
        out[s:s + c] = cast_t(v, dtype)
    return out.reshape(rows, cols)


def cast_t(v64, dtype):
    import torch
    if dtype == torch.float64:
        return v64
    v32 = v64.to(torch.float32)
    if dtype == torch.float32:
        return v32
    if dtype == torch.bfloat16:
        return rng.f32_to_bf16_t(v32)
    raise ValueError(dtype)


def cast_np(v64: np.ndarray, dtype: str) -> np.ndarray:
    """Value as seen after rounding to dtype ('f64', 'f32', 'bf16'), in float64."""
    if dtype == "f64":
        return np.asarray(v64, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(v64, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return rng.round_to_bf16(v64)
    raise ValueError(dtype)


def gen_many_torch(specs, device, dtype, chunk_elems=1 << 27):
    """Fill many cores in one flat device buffer.  specs: list of
    (seed, obj, core_id, shape, sigma2).  Element e of a core uses the same
    counters (2e, 2e + 1) under the same key as gen_tt_np / gen_tt_torch, so
    the values agree with theirs up to the last bit of Box-Muller.  Returns
    one tensor view per spec (contiguous, in spec order)."""
    import torch
    sizes = [int(np.prod(s[3])) for s in specs]
    total = int(sum(sizes))
    flat = torch.empty(max(total, 1), dtype=dtype, device=device)
    views = []
    off = 0
    i = 0
    while i < len(specs):
        j, acc = i, 0
        while j < len(specs) and (acc == 0 or acc + sizes[j] <= chunk_elems):
            acc += sizes[j]
            j += 1
        keys = torch.tensor([rng._s64(rng.derive_key(s[0], s[1], s[2])) for s in specs[i:j]],
                            dtype=torch.int64, device=device)
        scl = torch.tensor([math.sqrt(s[4]) for s in specs[i:j]], dtype=torch.float64, device=device)
        cnt = torch.tensor(sizes[i:j], dtype=torch.int64, device=device)
        starts = torch.cumsum(cnt, 0) - cnt
        kk = torch.repeat_interleave(keys, cnt)
        ss = torch.repeat_interleave(scl, cnt)
        e = torch.arange(acc, dtype=torch.int64, device=device) - torch.repeat_interleave(starts, cnt)
        z0 = rng._mix64_t((2 * e + 1) * rng._s64(rng.GAMMA) + kk)
        z1 = rng._mix64_t((2 * e + 2) * rng._s64(rng.GAMMA) + kk)
        del e
        u0 = rng._lsr(z0, 11).to(torch.float64) * (2.0 ** -53)
        u1 = rng._lsr(z1, 11).to(torch.float64) * (2.0 ** -53)
        del z0, z1
        v = torch.sqrt(-2.0 * torch.log(1.0 - u0)) * torch.cos(2.0 * np.pi * u1) * ss
        flat[off:off + acc] = cast_t(v, dtype)
        del u0, u1, v, kk, ss
        off += acc
        i = j
    off = 0
    for s, n in zip(specs, sizes):
        views.append(flat[off:off + n].view(*s[3]))
        off += n
    return views


def batch_specs(seed: int, shapes):
    """Generator specs of the uneven batch: X of pair p is object 1 + 2p,
    Y is object 2 + 2p; core k of each has sigma2 = 1 / max(R_k, R_{k+1})."""
    specs = []
    for p, (sx, sy) in enumerate(shapes):
        for obj, sh in ((1 + 2 * p, sx), (2 + 2 * p, sy)):
            for k in range(sh.order):
                specs.append((seed, obj, k, sh.core_shape(k), sigma2_of(sh, k)))
    return specs


def gen_batch_torch(seed: int, shapes, device, dtype):
    views = gen_many_torch(batch_specs(seed, shapes), device, dtype)
    pairs, i = [], 0
    for sx, sy in shapes:
        x = views[i:i + sx.order]
        i += sx.order
        y = views[i:i + sy.order]
        i += sy.order
        pairs.append((x, y))
    return pairs
