"""Helpers for checking fragment lists and arrays, independent of both the
oracle and the GPU path (numpy only)."""
from __future__ import annotations

import numpy as np

NIL = 0xFFFFFFFF


def walk_lists(head: np.ndarray, pool: np.ndarray, counter: int, return_index: bool = False,
               partial: bool = False):
    """Follow every list from its head (vectorised over lists).

    Returns (keys, recs): for every list member its head key and its 16-byte
    record, in walk order (and the pool indices when return_index). Raises AssertionError if an index is out of range,
    a pool slot is reached twice, or the walk does not visit exactly
    min(counter, cap) slots (with partial=True, head covers only some of the
    keys and each slot is visited at most once)."""
    cap = pool.shape[0]
    F = min(counter, cap)
    keys_all = np.nonzero(head != NIL)[0].astype(np.uint64)
    cur = head[keys_all].astype(np.int64)
    seen = np.zeros(F, np.int32)
    out_k, out_i = [], []
    steps = 0
    while cur.size:
        assert np.all(cur < F), "list index beyond the valid pool"
        out_k.append(keys_all)
        out_i.append(cur)
        np.add.at(seen, cur, 1)
        nxt = pool[cur, 3].astype(np.int64)
        live = nxt != NIL
        keys_all, cur = keys_all[live], nxt[live]
        steps += 1
        assert steps <= F + 1, "cycle in a list"
    if partial:
        assert np.all(seen <= 1), "pool slot in more than one list"
    else:
        assert np.all(seen == 1), "pool slot not in exactly one list"
    if not out_k:
        e = (np.zeros(0, np.uint64), np.zeros((0, 4), np.uint32))
        return e + (np.zeros(0, np.int64),) if return_index else e
    k = np.concatenate(out_k)
    i = np.concatenate(out_i)
    return (k, pool[i], i) if return_index else (k, pool[i])


def multiset_leq(a: np.ndarray, b: np.ndarray) -> bool:
    """True when every row of a occurs in b at least as often as in a."""
    if a.shape[0] == 0:
        return True
    ua, ca = np.unique(a, axis=0, return_counts=True)
    ub, cb = np.unique(b, axis=0, return_counts=True)
    allr = np.concatenate([ub, ua])
    _, inv = np.unique(allr, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nb = np.zeros(inv.max() + 1, np.int64)
    np.add.at(nb, inv[:ub.shape[0]], cb)
    return bool(np.all(nb[inv[ub.shape[0]:]] >= ca))


def canonical(keys: np.ndarray, recs: np.ndarray) -> np.ndarray:
    """Rows (key, w0, w1, w2) sorted ascending: the multiset of every list,
    independent of pool order and link values."""
    rows = np.stack([keys.astype(np.uint64), recs[:, 0].astype(np.uint64),
                     recs[:, 1].astype(np.uint64), recs[:, 2].astype(np.uint64)], 1)
    order = np.lexsort((rows[:, 3], rows[:, 2], rows[:, 1], rows[:, 0]))
    return rows[order]


def expected_arrays(keys: np.ndarray, recs: np.ndarray):
    """Per-octant arrays by a textbook sort: records ordered by
    (key, w0, w1, w2); table of distinct keys with offsets and counts; w3 =
    rank of the key among distinct keys."""
    rows = canonical(keys, recs)
    uk, first, cnt = np.unique(rows[:, 0], return_index=True, return_counts=True)
    rank = np.repeat(np.arange(uk.size, dtype=np.uint64), cnt)
    frag = np.stack([rows[:, 1], rows[:, 2], rows[:, 3], rank], 1).astype(np.uint32)
    return uk.astype(np.uint64), first.astype(np.uint32), cnt.astype(np.uint32), frag
