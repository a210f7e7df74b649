"""Oracle (test infrastructure only): a fill-reducing order from coordinates.

Section 3.3 allows any sigma-independent fill-reducing order Q; inertia does
not depend on it (Sylvester's law), it only affects the oracle's speed.  This
is recursive coordinate bisection: split the vertices at the median of the
widest coordinate, take as separator the boundary vertices of one half
(those with a neighbour in the other half), recurse, and number
[left part, right part, separator].  Periodic bonds simply add their wrap
edges to the boundary.  Independent of the GPU library's graph ordering.
"""
from __future__ import annotations

import numpy as np


def coordinate_nd(rowptr: np.ndarray, col: np.ndarray, coords: np.ndarray | None,
                  leaf: int = 64) -> np.ndarray:
    n = rowptr.size - 1
    if coords is None:
        return np.arange(n, dtype=np.int64)
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    coords = np.asarray(coords, dtype=np.float64)
    out = []
    where = np.full(n, -1, dtype=np.int64)      # label of each vertex in the current split

    # explicit stack of (vertex set, is_separator_to_emit)
    stack = [(np.arange(n, dtype=np.int64), False)]
    while stack:
        verts, emit = stack.pop()
        if emit or verts.size <= leaf:
            out.append(verts)
            continue
        c = coords[verts]
        ext = c.max(axis=0) - c.min(axis=0)
        ax = int(np.argmax(ext))
        if ext[ax] == 0:
            out.append(verts)
            continue
        order = np.lexsort((verts, c[:, ax]))
        half = verts.size // 2
        left, right = verts[order[:half]], verts[order[half:]]
        where[left] = 0
        where[right] = 1
        # boundary vertices of the left half: a neighbour lies in the right half
        starts = rowptr[left]
        lens = rowptr[left + 1] - starts
        tot = int(lens.sum())
        src = np.repeat(np.arange(left.size), lens)
        eidx = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(tot)
        hit = where[col[eidx]] == 1
        sep_mask = np.zeros(n, dtype=bool)
        sep_mask[left[src[hit]]] = True
        sep = left[sep_mask[left]]
        left = left[~sep_mask[left]]
        where[verts] = -1
        # emitted in stack (LIFO) order: left part, right part, separator
        stack.append((sep, True))
        stack.append((right, False))
        stack.append((left, False))
    perm = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    assert perm.size == n and np.unique(perm).size == n
    return perm.astype(np.int64)
