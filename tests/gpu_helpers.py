"""Helpers for the GPU tests: device<->host transfer of uint64 keys and
properties that hold at any size (sortedness, multiset hash)."""
from __future__ import annotations

import numpy as np
import torch

SIGN = -(1 << 63)


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).to(dev).view(torch.uint64)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_host(t: torch.Tensor) -> np.ndarray:
    if t.dtype == torch.uint64:
        return t.view(torch.int64).cpu().numpy().view(np.uint64)
    return t.cpu().numpy()


def signed_order_key(t: torch.Tensor) -> torch.Tensor:
    """int64 whose signed order is the keys' order (totalOrder for float64)."""
    b = t.view(torch.int64)
    if t.dtype == torch.uint64:
        return b ^ SIGN
    return torch.where(b < 0, b ^ 0x7FFFFFFFFFFFFFFF, b)


def is_sorted(t: torch.Tensor) -> bool:
    if t.numel() < 2:
        return True
    k = signed_order_key(t)
    return bool((k[:-1] <= k[1:]).all().item())


def _lsr(z: torch.Tensor, s: int) -> torch.Tensor:
    return (z >> s) & ((1 << (64 - s)) - 1)


def multiset_hash(t: torch.Tensor, salt: int = 0) -> int:
    """Sum over keys of a 64-bit mixing function (wrapping): equal for any
    permutation of the same multiset."""
    z = t.view(torch.int64) ^ salt
    z = (z ^ _lsr(z, 30)) * -4658895280553007687   # 0xBF58476D1CE4E5B9
    z = (z ^ _lsr(z, 27)) * -7723592293110705685   # 0x94D049BB133111EB
    z = z ^ _lsr(z, 31)
    return int(z.sum().item())
