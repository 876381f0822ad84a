"""FP64 oracle of the point-set initialisation (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
Sec. 3.2 initialises one Gaussian per point p_i of the initial point set: its isotropic
scale is the distance from p_i to the nearest point of the set at a different position,
s_i = min over {p in P, p != p_i} of ||p_i - p||_2, its opacity 0.1, its rotation the
identity, its view-independent colour the colour given for the point and every higher SH
coefficient 0.

Readings: "p != p_i" compares positions, so coincident copies of p_i are left out like p_i
itself; when no point at another position exists the minimum over the empty set is +inf.
The distance is computed from the FP32 coordinates in FP64 as sqrt((dx*dx + dy*dy) + dz*dz)
(no fused multiply-add) and rounded to FP32 once. The colour enters the SH DC coefficient
as k_DC = (c - 1/2) / Y_00 with Y_00 = 1 / (2 sqrt(pi)), which makes the colour model
max(0, sum k Y + 1/2) return c for any view direction (the paper writes the DC coefficients
as the NeRF colour itself, leaving this offset and scale implicit).
"""
from __future__ import annotations

import numpy as np

OPACITY0 = 0.1
Y00 = 0.5 / np.sqrt(np.pi)


def nn_distance(points: np.ndarray) -> np.ndarray:
    """points [3][n] (FP32 values) -> s [n] float32 by the definition (all pairs, O(n^2))."""
    p = np.asarray(points, np.float64)
    n = p.shape[1]
    out = np.empty(n, np.float64)
    for i in range(n):
        dx, dy, dz = p[0] - p[0, i], p[1] - p[1, i], p[2] - p[2, i]
        d2 = (dx * dx + dy * dy) + dz * dz
        d2 = d2[d2 > 0.0]
        out[i] = np.sqrt(d2.min()) if d2.size else np.inf
    return out.astype(np.float32)


def nn_distance_at(points: np.ndarray, idx) -> np.ndarray:
    """s_i for the listed i only (each against all n points): the definition sampled."""
    p = np.asarray(points, np.float64)
    out = []
    for i in idx:
        dx, dy, dz = p[0] - p[0, i], p[1] - p[1, i], p[2] - p[2, i]
        d2 = (dx * dx + dy * dy) + dz * dz
        d2 = d2[d2 > 0.0]
        out.append(np.sqrt(d2.min()) if d2.size else np.inf)
    return np.asarray(out, np.float64).astype(np.float32)


def init_gaussians(points: np.ndarray, colours=None, sh_degree: int = 3):
    """(mean [3][n], scale [3][n], quat [4][n], opacity [n], sh [(d+1)^2*3][n]), all float32."""
    p = np.asarray(points, np.float32)
    n = p.shape[1]
    s = nn_distance(p)
    scale = np.stack([s, s, s])
    quat = np.zeros((4, n), np.float32)
    quat[0] = 1.0
    opacity = np.full(n, OPACITY0, np.float32)
    sh = np.zeros(((sh_degree + 1) ** 2 * 3, n), np.float32)
    if colours is not None:
        c = np.asarray(colours, np.float32).astype(np.float64)
        sh[0:3] = ((c - 0.5) / Y00).astype(np.float32)
    return p.copy(), scale, quat, opacity, sh
