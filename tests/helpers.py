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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_core_rel(got, want) -> float:
    return max(rel_fro(g, w) for g, w in zip(got, want))


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
