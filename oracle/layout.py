"""Space-filling-curve renumbering and per-mass incidence lists (test infrastructure).

Section "GPU Implementation" keeps the mass<->spring connectivity twice: springs list their
two masses, and every mass lists its connected springs so a per-mass pass can visit them.
Here that per-mass list is a CSR incidence list over a Morton (Z-order) renumbering of the
masses; this module is the plain definition the native builder must reproduce bit-exactly:

* Morton key of integer coordinates q (relative to the body's minimum): bit b of qx goes to
  key bit 3b, of qy to 3b+1, of qz to 3b+2 (21 bits per axis);
* without integer coordinates, positions are quantised per body: ext = largest bbox extent,
  q = min(floor((x - min) * (2^20 / ext)), 2^20 - 1) (q = 0 when ext = 0);
* new order = stable sort by (body, key, input index); perm[new] = old;
* springs renumbered by (min, max) of their new endpoints, sorted ascending;
* CSR row i lists (neighbour, spring id) sorted by neighbour index.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def morton_key(q: np.ndarray) -> np.ndarray:
    """Interleave 21 bits of each of q[:,0], q[:,1], q[:,2] (x lowest)."""
    q = np.asarray(q, dtype=np.uint64)
    key = np.zeros(len(q), dtype=np.uint64)
    for b in range(21):
        for c in range(3):
            bit = (q[:, c] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + c)
    return key


def quantise(x: np.ndarray) -> np.ndarray:
    """Per-body quantisation of float positions to 20-bit integer cells."""
    x = np.asarray(x, dtype=np.float64)
    lo = x.min(axis=0)
    ext = float((x.max(axis=0) - lo).max())
    if ext == 0.0:
        return np.zeros(x.shape, dtype=np.int64)
    scale = 1048576.0 / ext
    q = np.floor((x - lo) * scale).astype(np.int64)
    return np.minimum(q, 1048575)


@dataclasses.dataclass
class Layout:
    perm: np.ndarray      # (N,) new -> old (input) index
    inv: np.ndarray       # (N,) old -> new
    ends: np.ndarray      # (S, 2) new endpoints, (min, max), sorted; row s = new spring s
    spring_perm: np.ndarray  # (S,) new spring -> input spring
    row_ptr: np.ndarray   # (N+1,)
    col: np.ndarray       # (2S,) neighbour (new index)
    sid: np.ndarray       # (2S,) new spring index


def reorder(ends_in: np.ndarray, body_offset: np.ndarray, coords=None, x=None) -> Layout:
    """Renumber masses along the Morton curve and build the incidence CSR."""
    body_offset = np.asarray(body_offset, dtype=np.int64)
    N = int(body_offset[-1])
    body = np.repeat(np.arange(len(body_offset) - 1), np.diff(body_offset))
    key = np.zeros(N, dtype=np.uint64)
    for b in range(len(body_offset) - 1):
        s, e = body_offset[b], body_offset[b + 1]
        if e == s:
            continue
        if coords is not None:
            c = np.asarray(coords[s:e], dtype=np.int64)
            q = c - c.min(axis=0)
        else:
            q = quantise(x[s:e])
        key[s:e] = morton_key(q)
    perm = np.lexsort((np.arange(N), key, body))
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)

    ends_in = np.asarray(ends_in, dtype=np.int64)
    a, b = inv[ends_in[:, 0]], inv[ends_in[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    sorder = np.lexsort((hi, lo))
    ends = np.stack([lo[sorder], hi[sorder]], axis=1)
    S = len(ends)

    rows = np.concatenate([ends[:, 0], ends[:, 1]])
    nbrs = np.concatenate([ends[:, 1], ends[:, 0]])
    sids = np.concatenate([np.arange(S), np.arange(S)])
    o = np.lexsort((nbrs, rows))
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return Layout(perm=perm, inv=inv, ends=ends, spring_perm=sorder,
                  row_ptr=row_ptr, col=nbrs[o], sid=sids[o])
