"""FP64 oracle of the Lloyd iterations that cluster camera positions (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
Sec. 3.4 groups the input camera centres with k-means. From given initial centres, each
iteration assigns every point to its nearest centre (squared Euclidean distance, ties to the
lowest centre index; the squared distance is formed as (dx dx + dy dy) + dz dz, so a device that
forms it the same way without fused multiply-add takes the same decisions), stops when no assignment changed (from the second iteration on), and
otherwise moves each centre to the mean of its points; a centre with no points moves to the
point farthest from its assigned centre (distances of that iteration's assignment, ties to the
lowest point index). After max_iter updates the points are assigned once more.
"""
from __future__ import annotations

import numpy as np


def _d2(pos, c):
    """[m][k] squared distances, (dx dx + dy dy) + dz dz."""
    dx = pos[:, None, 0] - c[None, :, 0]
    dy = pos[:, None, 1] - c[None, :, 1]
    dz = pos[:, None, 2] - c[None, :, 2]
    return dx * dx + dy * dy + dz * dz


def lloyd(pos, centres, max_iter: int):
    """pos [m][3], centres [k][3] (initial) -> (centres [k][3], assign [m], iterations)."""
    pos = np.asarray(pos, np.float64)
    c = np.array(centres, np.float64, copy=True)
    k = c.shape[0]
    assign = np.full(pos.shape[0], -1, np.int64)
    it = 0
    for it in range(max(1, max_iter)):
        d2 = _d2(pos, c)
        new = np.argmin(d2, axis=1)  # first minimum: the lowest centre index
        changed = bool(np.any(new != assign))
        assign = new
        if not changed and it > 0:
            return c, assign, it
        dbest = d2[np.arange(pos.shape[0]), assign]
        far = int(np.argmax(dbest))  # first maximum: the lowest point index
        for j in range(k):
            members = pos[assign == j]
            c[j] = members.mean(0) if len(members) else pos[far]
        if it + 1 >= max_iter:
            d2 = _d2(pos, c)
            assign = np.argmin(d2, axis=1)
            return c, assign, it + 1
    return c, assign, it + 1
