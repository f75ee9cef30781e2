"""Shared test utilities: moving seeded inputs to the GPU, error measures."""
from __future__ import annotations

import math

import numpy as np

from ttgen import configs as C

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def torch_dtype(name):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[name]


def to_gpu(cores64, dtype: str):
    """Upload FP64 numpy cores rounded (RNE) to dtype; returns (tensors,
    the exact float64 values the GPU holds)."""
    import torch
    td = torch_dtype(dtype)
    out, seen = [], []
    for G in cores64:
        t = torch.from_numpy(np.ascontiguousarray(G)).to(torch.float32 if dtype != "f64" else torch.float64)
        t = t.to(td).cuda().contiguous()
        out.append(t)
        seen.append(t.detach().to(torch.float64).cpu().numpy())
    return out, seen


def to_np(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def rel_fro(a, b) -> float:
    """Relative Frobenius error ||a - b|| / ||b|| of the whole array."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rows(a: np.ndarray, min_len: int) -> np.ndarray:
    """View as (rows, L): trailing axes merged until a row holds at least
    min_len consecutive entries (the whole array when it is smaller)."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 0:
        return a.reshape(1, 1)
    L, ax = 1, a.ndim
    while ax > 0 and L < min_len:
        ax -= 1
        L *= a.shape[ax]
    return a.reshape(-1, max(L, 1))


def row_rel(a, b, min_len: int = 64) -> float:
    """Largest per-row error max_r ||a_r - b_r|| / max(||b_r||, rms_r ||b_r||)
    over rows of at least min_len consecutive entries: a row at least as
    large as the RMS row is measured against its own norm, a smaller row
    against the RMS row norm (the rounding error of a smaller row scales
    with the whole computation's size, not with the row's own value, so its
    own norm would overstate it for low-rank or structured outputs).  Any
    block of wrong entries of the output's typical size moves the rows it
    touches by O(sqrt(block / row)), however large the array."""
    A, B = _rows(a, min_len), _rows(b, min_len)
    assert A.shape == B.shape, (np.shape(a), np.shape(b))
    if B.size == 0:
        return 0.0
    nb = np.linalg.norm(B, axis=1)
    rms = math.sqrt(float(np.mean(nb * nb)))
    den = np.maximum(nb, max(rms, 1e-300))
    return float(np.max(np.linalg.norm(A - B, axis=1) / den))


def rel_err(a, b) -> float:
    """The gate used by every floating-point parity check: the larger of
    the whole-array relative Frobenius error and the largest per-row
    relative error (row_rel)."""
    return max(rel_fro(a, b), row_rel(a, b))


def max_core_rel(got, want) -> float:
    """rel_err of the worst core of a TT (shapes must match core by core)."""
    assert len(got) == len(want)
    return max(rel_err(g, w) for g, w in zip(got, want))


def scalar_err(z_gpu: float, z_ref: float, nx: float, ny: float) -> float:
    """|z - z_ref| / (||X|| ||Y||): the Cauchy-Schwarz scale of an inner product."""
    return abs(z_gpu - z_ref) / max(nx * ny, 1e-300)


def tt_norm(cores) -> float:
    from oracle import tt_oracle as O
    return math.sqrt(max(O.inner_lr(cores, cores), 0.0))


def random_pair(seed, modes, rx, ry):
    x = C.gen_tt_np(seed, 1, C.TTShape(list(modes), list(rx)))
    y = C.gen_tt_np(seed, 2, C.TTShape(list(modes), list(ry)))
    return x, y
