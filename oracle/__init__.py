"""FP64 CPU oracle of the splatting model (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It wraps ``gs_oracle.c`` (plain C, FP64, built with gcc) and shares
no code with the GPU library. See the C file's header for what each routine
computes and which passage of the paper it follows:

  project      per-Gaussian projection (Sec. 3.2: Sigma = R S S^T R^T,
               Sigma' = J M Sigma M^T J^T), SH colour, depth key, tile rectangle
  render       tile-free per-pixel front-to-back compositing (eq. render-gs)
  importance   h_i = max over views and pixels of alpha*T (eq. importance-score)
  prune_mask   m_i = [h_i < t_prune] (Sec. 3.3)
  cluster_bits m_ci = [max over views of cluster c of alpha*T > t_cluster]
               (eq. importance-score-vis)
  render_bwd   exact a.e. gradient of the image w.r.t. all Gaussian parameters
  pairs        the (tile, depth, index) key list the binning step must produce

The training loss of Sec. 3.2 ((1 - lambda) L2 + lambda D-SSIM) and its gradient are in
``oracle.loss`` (numpy, FP64); the initialisation of Sec. 3.2 (nearest-neighbour scales,
opacity, rotation and DC colour of one Gaussian per point) is in ``oracle.init``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_SO = os.path.join(_HERE, "libgs_oracle.so")

# projection table fields (must follow the enum in gs_oracle.c)
FIELDS = ["vis", "x", "y", "z", "u", "v", "sxx", "sxy", "syy", "ca", "cb", "cc", "qmax", "hx", "hy", "r", "g", "b",
          "rawr", "rawg", "rawb", "depth32", "tx0", "ty0", "tx1", "ty1", "count", "opac", "dx", "dy", "dz", "dlen"]
F = {name: k for k, name in enumerate(FIELDS)}
NG2 = 9

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GS_ORACLE_LIB")  # another build of gs_oracle.c (the sanitizer run's)
        if not path:
            path = _SO
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        L.or_project.argtypes = [dp, dp, dp, dp, dp, i64, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.or_render.argtypes = [dp, i64, dp, ip, ip, i64, ctypes.c_double, ctypes.c_double, dp, dp, ip, lp, dp]
        L.or_render_bwd_2d.argtypes = [dp, i64, dp, ip, ip, i64, dp, dp]
        L.or_project_bwd.argtypes = [dp, dp, dp, dp, i64, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.or_sh_basis.argtypes = [ctypes.c_int, dp, i64, dp]
        L.or_sh_basis_grad.argtypes = [ctypes.c_int, dp, i64, dp]
        assert L.or_nproj() == len(FIELDS), "field table out of date"
        assert L.or_ng2() == NG2
        _lib = L
    return _lib


def _p(a, ctype=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _d(a) -> np.ndarray:
    """FP32 (or any) array widened exactly to a C-contiguous FP64 array."""
    return np.ascontiguousarray(np.asarray(a).astype(np.float64))


def cam_array(cam) -> np.ndarray:
    a = np.zeros(20, np.float64)
    a[0:9] = np.asarray(cam.R, np.float32).reshape(-1)
    a[9:12] = np.asarray(cam.t, np.float32)
    a[12:16] = np.float32([cam.fx, cam.fy, cam.cx, cam.cy])
    a[16] = cam.width
    a[17] = cam.height
    a[18] = np.float32(cam.znear)
    return a


def params_array(p) -> np.ndarray:
    a = np.zeros(9, np.float64)
    a[0:6] = np.float32([p.lowpass, p.kappa, p.alpha_min, p.alpha_max, p.t_min, p.guard])
    a[6:9] = np.float32(p.bg)
    return a


def sh_basis(degree: int, dirs: np.ndarray) -> np.ndarray:
    """Real orthonormal SH (Condon-Shortley phase) at unit directions [m][3] -> [m][(d+1)^2]."""
    dirs = _d(dirs).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], (degree + 1) ** 2))
    lib().or_sh_basis(degree, _p(dirs), dirs.shape[0], _p(out))
    return out


def sh_basis_grad(degree: int, dirs: np.ndarray) -> np.ndarray:
    dirs = _d(dirs).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], (degree + 1) ** 2, 3))
    lib().or_sh_basis_grad(degree, _p(dirs), dirs.shape[0], _p(out))
    return out


def project(scene, cam, params, tile=(16, 16)) -> np.ndarray:
    """Projection table [n][len(FIELDS)] of one view."""
    n = scene.n
    out = np.zeros((n, len(FIELDS)), np.float64)
    mean, scale, quat, op, sh = (_d(scene.mean), _d(scene.scale), _d(scene.quat), _d(scene.opacity), _d(scene.sh))
    lib().or_project(_p(mean), _p(scale), _p(quat), _p(op), _p(sh), n, scene.sh_degree, _p(cam_array(cam)),
                     _p(params_array(params)), int(tile[0]), int(tile[1]), _p(out))
    return out


def all_pixels(cam):
    py, px = np.meshgrid(np.arange(cam.height, dtype=np.int32), np.arange(cam.width, dtype=np.int32), indexing="ij")
    return px.reshape(-1).copy(), py.reshape(-1).copy()


def render(scene, cam, params, pixels=None, proj=None, qmax_scale=1.0, tmin_scale=1.0, want_h=False,
           fingerprint=False) -> Dict[str, np.ndarray]:
    """Render pixels of one view. pixels = (px, py) int arrays, or None for the whole image.

    Returns rgb [m][3] (or [3][H][W] for a whole image), T [m], ncomp [m], optionally h [n]
    (max weight per Gaussian over these pixels) and fp (decision fingerprint per pixel)."""
    if proj is None:
        proj = project(scene, cam, params)
    whole = pixels is None
    if whole:
        px, py = all_pixels(cam)
    else:
        px = np.ascontiguousarray(pixels[0], np.int32)
        py = np.ascontiguousarray(pixels[1], np.int32)
    m = px.shape[0]
    rgb = np.zeros((m, 3))
    T = np.zeros(m)
    nc = np.zeros(m, np.int32)
    fp = np.zeros(m, np.int64) if fingerprint else None
    h = np.zeros(scene.n) if want_h else None
    lib().or_render(_p(proj), scene.n, _p(params_array(params)), _p(px, ctypes.c_int32), _p(py, ctypes.c_int32), m,
                    float(qmax_scale), float(tmin_scale), _p(rgb), _p(T), _p(nc, ctypes.c_int32),
                    _p(fp, ctypes.c_int64), _p(h))
    out = {"rgb": rgb, "T": T, "ncomp": nc}
    if whole:
        out["rgb"] = rgb.reshape(cam.height, cam.width, 3).transpose(2, 0, 1).copy()
        out["T"] = T.reshape(cam.height, cam.width)
        out["ncomp"] = nc.reshape(cam.height, cam.width)
    if want_h:
        out["h"] = h
    if fingerprint:
        out["fp"] = fp if not whole else fp.reshape(cam.height, cam.width)
    return out


def importance(scene, cams: Sequence, params, pixels_per_view=None) -> np.ndarray:
    """h_i = max over the given views (all pixels, or the listed ones) of alpha*T (eq. importance-score)."""
    h = np.zeros(scene.n)
    for v, cam in enumerate(cams):
        pix = None if pixels_per_view is None else pixels_per_view[v]
        h = np.maximum(h, render(scene, cam, params, pixels=pix, want_h=True)["h"])
    return h


def prune_mask(h: np.ndarray, t_prune: float) -> np.ndarray:
    """m_i = 1(h_i < t_prune): True means the Gaussian is removed (Sec. 3.3)."""
    return h < t_prune


def cluster_bits(scene, cams: Sequence, view_cluster: Sequence[int], k: int, params, t_cluster: float) -> np.ndarray:
    """bits[c][i] = [max over views assigned to c of alpha*T > t_cluster] (eq. importance-score-vis)."""
    hc = np.zeros((k, scene.n))
    for v, cam in enumerate(cams):
        c = int(view_cluster[v])
        hc[c] = np.maximum(hc[c], render(scene, cam, params, want_h=True)["h"])
    return hc > t_cluster


def render_bwd(scene, cam, params, dl_drgb, pixels=None, proj=None) -> Dict[str, np.ndarray]:
    """Gradient of sum(dl_drgb * image) w.r.t. mean, scale, quat, opacity, sh (SoA like the scene).

    dl_drgb is [3][H][W] for a whole image or [m][3] for listed pixels."""
    if proj is None:
        proj = project(scene, cam, params)
    if pixels is None:
        px, py = all_pixels(cam)
        g = _d(np.asarray(dl_drgb).reshape(3, -1).T)
    else:
        px = np.ascontiguousarray(pixels[0], np.int32)
        py = np.ascontiguousarray(pixels[1], np.int32)
        g = _d(dl_drgb).reshape(-1, 3)
    n = scene.n
    g2 = np.zeros((n, NG2))
    L = lib()
    L.or_render_bwd_2d(_p(proj), n, _p(params_array(params)), _p(px, ctypes.c_int32), _p(py, ctypes.c_int32),
                       px.shape[0], _p(g), _p(g2))
    out = {"mean": np.zeros((3, n)), "scale": np.zeros((3, n)), "quat": np.zeros((4, n)),
           "opacity": np.zeros(n), "sh": np.zeros(scene.sh.shape)}
    L.or_project_bwd(_p(_d(scene.mean)), _p(_d(scene.scale)), _p(_d(scene.quat)), _p(_d(scene.sh)), n,
                     scene.sh_degree, _p(cam_array(cam)), _p(proj), _p(g2), _p(out["mean"]), _p(out["scale"]),
                     _p(out["quat"]), _p(out["opacity"]), _p(out["sh"]))
    out["g2d"] = g2
    return out


def pairs(depth32: Sequence[np.ndarray], rects: Sequence[np.ndarray], sizes: Sequence, tile=(16, 16)):
    """The sorted (key, value) list binning must produce, for views v = 0, 1, ...

    Tiles of view v are numbered off_v + ty * tiles_x + tx, where off_v is the number of
    tiles of all earlier views (tiles_x = ceil(W / tile_w), tiles_y = ceil(H / tile_h)).
    For view v and Gaussian i with FP32 depth d and inclusive tile rectangle
    (tx0, ty0, tx1, ty1) (rows of rects[v]; empty when tx1 < tx0 or ty1 < ty0), every tile
    of the rectangle gives key = tile << 32 | bits(d) and value = i. The list is sorted by
    key, then value."""
    keys, vals = [], []
    off = 0
    for v, (d, r) in enumerate(zip(depth32, rects)):
        W, H = int(sizes[v][0]), int(sizes[v][1])
        tiles_x = (W + tile[0] - 1) // tile[0]
        tiles_y = (H + tile[1] - 1) // tile[1]
        d = np.asarray(d, np.float32)
        r = np.asarray(r, np.int64).reshape(-1, 4)
        bits = d.view(np.uint32).astype(np.uint64)
        for i in np.nonzero((r[:, 2] >= r[:, 0]) & (r[:, 3] >= r[:, 1]))[0]:
            tx = np.arange(r[i, 0], r[i, 2] + 1)
            ty = np.arange(r[i, 1], r[i, 3] + 1)
            tid = (ty[:, None] * tiles_x + tx[None, :]).reshape(-1) + off
            keys.append((tid.astype(np.uint64) << np.uint64(32)) | bits[i])
            vals.append(np.full(tid.shape, i, np.uint32))
        off += tiles_x * tiles_y
    if not keys:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    k = np.concatenate(keys)
    v = np.concatenate(vals)
    order = np.lexsort((v, k))
    return k[order], v[order]


def rects_of(proj: np.ndarray) -> np.ndarray:
    """Inclusive tile rectangles [n][4] from a projection table; culled Gaussians get an empty one."""
    r = proj[:, [F["tx0"], F["ty0"], F["tx1"], F["ty1"]]].astype(np.int64)
    empty = (proj[:, F["vis"]] == 0) | (proj[:, F["count"]] == 0)
    r[empty] = (0, 0, -1, -1)
    return r
