"""Glue for the GPU tests: run the path through the C ABI and bring results
back as numpy uint32/uint64 arrays."""
from __future__ import annotations

import numpy as np


def u32(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def run_capture(F, mesh, d, cap):
    """Capture on the GPU; returns (head, pool, keys, counter, lists)."""
    import torch
    dm = F.to_device(mesh)
    lists = F.alloc_lists(d, cap)
    F.capture(dm, d, lists)
    torch.cuda.synchronize()
    pool = u32(lists.pool)[:cap] if cap else np.zeros((0, 4), np.uint32)
    kv = lists.keys.detach().cpu().numpy()
    kv = kv.view(np.uint64) if kv.dtype == np.int64 else kv.view(np.uint32)
    keys = kv[:cap] if cap else np.zeros(0, np.uint32)
    return u32(lists.head), pool, keys, int(lists.counter.item()), lists


def run_compact(F, lists, d, cap_occ=None):
    import torch
    out = F.alloc_pofa(lists.capacity, cap_occ)
    F.compact(lists, d, out)
    torch.cuda.synchronize()
    n_occ = int(out.n_occ.item())
    n_frag = int(out.n_frag.item())
    n = min(n_occ, out.cap_occ)
    return {"key": u64(out.oct_key)[:n], "off": u32(out.oct_off)[:n], "cnt": u32(out.oct_cnt)[:n],
            "frag": u32(out.frag)[:n_frag], "n_occ": n_occ, "n_frag": n_frag}, out


def run_splat(F, pofa, d, views):
    import torch
    img = F.splat(pofa, d, views)
    torch.cuda.synchronize()
    return u32(img.rgba), img.depth.cpu().numpy(), img.cov.cpu().numpy()
