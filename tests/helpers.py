"""Shared test helpers: GPU availability, the oracle's threshold band, and GPU<->oracle
marshalling of the library's outputs."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenes  # noqa: E402

# Parity bars (see the design notes): images 1e-4 absolute per channel, importance 1e-5,
# gradients 1e-3 relative.
TOL_IMAGE = 1e-4
TOL_H = 1e-5
TOL_GRAD = 1e-3
# Threshold band: the oracle is re-run with the support radius q_max scaled by 1 +- Q_EPS and
# the stop threshold t_min by 1 +- T_EPS. The GPU evaluates the support test in FP64 (only
# FP64 rounding separates it from the oracle, far inside 1e-5); its transmittance is an FP32
# running product whose relative error grows like sqrt(n) * 2^-24 for n composited entries
# (about 1e-6 at n = 300), so a 1e-5 shift of t_min covers its stop decisions.
Q_EPS = 1e-5
T_EPS = 1e-5


def mismatch_limit(n):
    """Entries allowed to differ beyond tolerance (all of them inside the band)."""
    return max(2, int(1e-4 * n))


def check_band(mismatch, band, what=""):
    """No mismatch outside the band; at most mismatch_limit mismatches inside it."""
    outside = int(np.sum(mismatch & ~band))
    inside = int(np.sum(mismatch & band))
    print(f"  {what}: band {int(band.sum())} of {band.size}, mismatches in band {inside}, outside {outside}",
          flush=True)
    assert outside == 0, f"{what}: {outside} entries differ outside the threshold band"
    assert inside <= mismatch_limit(band.size), f"{what}: {inside} entries differ inside the band"


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def band_runs(scene, cam, params, pixels=None, want_h=False):
    """Oracle renders at the nominal thresholds and at the four shifted ones."""
    proj = oracle.project(scene, cam, params)
    runs = []
    for qs, ts in [(1, 1), (1 - Q_EPS, 1), (1 + Q_EPS, 1), (1, 1 - T_EPS), (1, 1 + T_EPS)]:
        runs.append(oracle.render(scene, cam, params, pixels=pixels, proj=proj, qmax_scale=qs, tmin_scale=ts,
                                  want_h=want_h))
    return proj, runs


def image_band(runs, tol=TOL_IMAGE):
    """Pixels whose colour or transmittance moves by more than tol between the runs."""
    nom = runs[0]
    band = np.zeros(nom["T"].shape, bool)
    for r in runs[1:]:
        d = np.abs(r["rgb"] - nom["rgb"])
        d = d.max(0) if d.ndim == 3 else d.max(-1)
        band |= (d > tol) | (np.abs(r["T"] - nom["T"]) > tol)
    return band


def h_band(runs, tol=TOL_H):
    nom = runs[0]["h"]
    band = np.zeros(nom.shape, bool)
    for r in runs[1:]:
        band |= np.abs(r["h"] - nom) > tol
    return band


def splat_table(proj_gpu, v=0):
    """GPU records of view v as a dict of numpy arrays."""
    import torch
    n = proj_gpu.n
    raw = proj_gpu.splat.view(torch.uint8)[v * n * 64:(v + 1) * n * 64].cpu().numpy().reshape(n, 64)
    d = raw[:, :48].copy().view(np.float64).reshape(n, 6)
    f = raw[:, 48:].copy().view(np.float32).reshape(n, 4)
    rect = proj_gpu.rect[v * n:(v + 1) * n].cpu().numpy().view(np.uint64)
    return {
        "u": d[:, 0], "v": d[:, 1], "ca": d[:, 2], "cb": d[:, 3], "cc": d[:, 4], "qmax": d[:, 5],
        "opac": f[:, 0], "rgb": f[:, 1:4],
        "depth": proj_gpu.depth[v * n:(v + 1) * n].cpu().numpy(),
        "count": proj_gpu.count[v * n:(v + 1) * n].cpu().numpy().view(np.uint32),
        "rect": np.stack([(rect >> np.uint64(s)) & np.uint64(0xffff) for s in (0, 16, 32, 48)], 1).astype(np.int64),
    }
