"""Counter-based random numbers for the synthetic workloads.

This module holds no part of the contraction arithmetic.  It only draws the
seeded inputs (TT cores, dense matrices, batches) that both the FP64 oracle
and the GPU library consume.

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode.  The
value for counter c under a key k is mix64(k + (c + 1) * GAMMA), where mix64
is the 64-bit finaliser of that paper and GAMMA = 0x9E3779B97F4A7C15.
Keys are derived from (seed, object id, core id) by chained mixing, so every
core of every tensor has an independent substream that does not depend on the
order in which objects are generated.

Uniforms take the top 53 bits: u = (z >> 11) * 2^-53 in [0, 1).
Normals use Box-Muller on the pair of counters (2e, 2e + 1) for element e:
n = sqrt(-2 ln(1 - u0)) * cos(2 pi u1).

BF16 values are the round-to-nearest-even rounding of the FP32 values
(FP64 -> FP32 -> BF16, each step RNE).

Two implementations are provided with identical integer streams: NumPy
(host) and torch (any device, used to fill multi-GB inputs directly in
device memory).  The transcendental step of Box-Muller may differ in the last
bit between the two, so tests always hand the oracle the very tensors that
the GPU consumed (copied to the host), never a regenerated copy.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix64_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (exact 64-bit arithmetic)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def derive_key(seed: int, *ids: int) -> int:
    """Key of the substream for (seed, id0, id1, ...)."""
    k = mix64_int(seed + GAMMA)
    for t in ids:
        k = mix64_int(k ^ ((int(t) + 1) * GAMMA & MASK64))
    return k


# ---------------------------------------------------------------- NumPy side
def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=False)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def raw_np(key: int, start: int, count: int) -> np.ndarray:
    """count consecutive 64-bit outputs for counters start .. start+count-1."""
    c = np.arange(start, start + count, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + c * np.uint64(GAMMA)
        return _mix64_np(z)


def uniform_np(key: int, count: int, start: int = 0) -> np.ndarray:
    z = raw_np(key, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal_np(key: int, count: int) -> np.ndarray:
    """count N(0,1) values in float64 (Box-Muller on counter pairs)."""
    u = uniform_np(key, 2 * count)
    u0 = 1.0 - u[0::2]
    u1 = u[1::2]
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def uniform_int_np(key: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integers uniform on [lo, hi] (inclusive) by floor(u * n)."""
    u = uniform_np(key, count)
    return lo + np.floor(u * (hi - lo + 1)).astype(np.int64)


# ---------------------------------------------------------------- BF16 RNE
def f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round FP32 to BF16 with round-to-nearest-even; returns uint16 bits."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = (b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 -> BF16 (RNE each step), returned as the exact float64 value."""
    return bf16_bits_to_f64(f32_to_bf16_bits(np.asarray(x, dtype=np.float32)))


# ---------------------------------------------------------------- torch side
def _torch():
    import torch
    return torch


def _s64(v: int) -> int:
    """Two's-complement signed view of an unsigned 64-bit constant."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(z, s: int):
    # logical shift right on int64 storage
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix64_t(z):
    z = (z ^ _lsr(z, 30)) * _s64(M1)
    z = (z ^ _lsr(z, 27)) * _s64(M2)
    return z ^ _lsr(z, 31)


def raw_t(key: int, start: int, count: int, device):
    torch = _torch()
    c = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = c * _s64(GAMMA) + _s64(key)
    return _mix64_t(z)


def uniform_t(key: int, count: int, device, start: int = 0):
    torch = _torch()
    z = raw_t(key, start, count, device)
    return _lsr(z, 11).to(torch.float64) * (2.0 ** -53)


def normal_t(key: int, count: int, device):
    torch = _torch()
    u = uniform_t(key, 2 * count, device)
    u0 = 1.0 - u[0::2]
    u1 = u[1::2]
    return torch.sqrt(-2.0 * torch.log(u0)) * torch.cos(2.0 * np.pi * u1)


def f32_to_bf16_t(x32):
    """RNE FP32 -> BF16 on torch tensors (bit arithmetic, any device)."""
    torch = _torch()
    b = x32.contiguous().view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = torch.where(r >= 0x8000, r - 0x10000, r).to(torch.int16)
    return r.view(torch.bfloat16)
