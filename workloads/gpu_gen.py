"""Seeded synthetic inputs generated directly in GPU memory (torch).

The served workload (64 tables of 10 to 200 columns, about 100 GB of
resident main partitions at full size) is too large to create on the host
and copy, so its columns are drawn on the device with a seeded
torch.Generator.  Like workloads.gen, this module only creates inputs:
random sorted dictionaries, uniform codes and their bit packing (the input
layout); it holds no step of the merge.

Value domains (so that torch's signed sort orders them like the column):
  u32   -> values in [0, 2^32), stored as int32 bit patterns
  u64   -> values in [0, 2^63)
  str16 -> bytes in [0x20, 0x7E] (top bit clear in every byte)
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .gen import BASE_SEED


def _sorted_unique_u(g, k, hi, device):
    """k distinct values in [0, hi) sorted, as int64."""
    got = torch.empty(0, dtype=torch.int64, device=device)
    while got.numel() < k:
        need = k - got.numel()
        draw = torch.randint(0, hi, (int(need * 1.02) + 16,), generator=g, device=device,
                             dtype=torch.int64)
        got = torch.unique(torch.cat([got, draw]))
    if got.numel() > k:
        keep = torch.randperm(got.numel(), generator=g, device=device)[:k]
        got = torch.sort(got[keep]).values
    return got


def _sorted_unique_str(g, k, device):
    """k distinct printable 16-byte strings in byte order, shape (k, 16) uint8."""
    got = torch.empty((0, 2), dtype=torch.int64, device=device)
    while got.shape[0] < k:
        need = k - got.shape[0]
        b = torch.randint(0x20, 0x7F, (int(need * 1.02) + 16, 16), generator=g, device=device,
                          dtype=torch.uint8)
        # big-endian halves: for bytes below 0x80 signed order == byte order
        be = b.view(-1, 2, 8).flip(-1).contiguous().view(torch.int64).view(-1, 2)
        got = torch.unique(torch.cat([got, be], dim=0), dim=0)
    if got.shape[0] > k:
        keep = torch.sort(torch.randperm(got.shape[0], generator=g, device=device)[:k]).values
        got = got[keep]
    return got.view(torch.uint8).view(-1, 2, 8).flip(-1).contiguous().view(-1, 16)


def pack_codes_gpu(codes: torch.Tensor, w: int) -> torch.Tensor:
    """Pack int64 codes (< 2^w) LSB-first into int64 words (same layout as
    workloads.gen.pack_codes), in groups of 64 codes = w words."""
    n = codes.numel()
    ngroups = (n + 63) // 64
    nwords = (n * w + 63) // 64
    c = torch.zeros(ngroups * 64, dtype=torch.int64, device=codes.device)
    c[:n] = codes
    c = c.view(ngroups, 64)
    out = torch.zeros((ngroups, w), dtype=torch.int64, device=codes.device)
    for j in range(64):
        off = j * w
        word, sh = off >> 6, off & 63
        out[:, word] |= c[:, j] << sh
        if sh + w > 64:
            out[:, word + 1] |= c[:, j] >> (64 - sh)
    flat = out.view(-1)
    res = torch.empty(max(nwords + (nwords & 1), 2), dtype=torch.int64, device=codes.device)
    res[:nwords] = flat[:nwords]
    res[nwords:] = 0
    return res


def random_values_gpu(g, vtype, n, device):
    if vtype == "u32":
        return torch.randint(0, 2 ** 32, (n,), generator=g, device=device,
                             dtype=torch.int64).to(torch.int32)
    if vtype == "u64":
        return torch.randint(0, 2 ** 63 - 1, (n,), generator=g, device=device, dtype=torch.int64)
    return torch.randint(0x20, 0x7F, (n, 16), generator=g, device=device, dtype=torch.uint8)


def served_shapes(ntables: int = 64, scale: float = 1.0):
    """Per table: (seed, [(vtype, rows, distinct) per column], append rows/s)."""
    out = []
    for t in range(ntables):
        rng = np.random.default_rng(BASE_SEED + 1000 * 5 + t)
        ncols = int(rng.integers(10, 201))
        cols = []
        for _ in range(ncols):
            rows = max(1, int(math.exp(rng.uniform(math.log(1e6), math.log(2e7))) * scale))
            kd = max(1, min(int(math.exp(rng.uniform(math.log(2), math.log(1e7)))), rows))
            vtype = ("u32", "u64", "str16")[int(rng.integers(0, 3))]
            cols.append((vtype, rows, kd))
        rate = math.exp(rng.uniform(math.log(1e4), math.log(1e6))) * scale
        out.append((int(rng.integers(0, 2 ** 62)), cols, rate))
    return out


def served_column(g, vtype, rows, kd, device="cuda"):
    """(vtype, U_M, packed codes, rows, w) generated on the device."""
    w = max(1, int(kd - 1).bit_length()) if kd > 1 else 1
    if vtype == "u32":
        u = _sorted_unique_u(g, kd, 2 ** 32, device).to(torch.int32)
    elif vtype == "u64":
        u = _sorted_unique_u(g, kd, 2 ** 63 - 1, device)
    else:
        u = _sorted_unique_str(g, kd, device)
    codes = torch.randint(0, kd, (rows,), generator=g, device=device, dtype=torch.int64)
    return vtype, u, pack_codes_gpu(codes, w), rows, w
