"""Python binding of the splatting library: buffers come from PyTorch (device memory and
streams), every computation is a call into libgs_hip.so (include/gs.h).

  Gaussians, ViewBatch          device-side inputs (structure of arrays; batched views)
  preprocess / bin_sort /       the C-ABI calls, one to one
  render_fwd / render_bwd /
  importance / cluster_visibility / bits_to_list
  render / render_batch         the plain path for one view batch (images per view)
  render_filtered               a test view with its nearest cluster's visibility list
  Renderer                      persistent buffers for repeated frames (fixed capacity,
                                no host synchronisation per frame)
  GSRender                      torch.autograd.Function over render_fwd / render_bwd
  kmeans / nearest_centre       camera clustering (Sec. 3.4): host, or host seeding + device Lloyd
  kmeans_seed / kmeans_lloyd    the two halves of the device clustering
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

DEFAULT_TILE = (16, 32)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(device):
    return torch.device(device if device is not None else "cuda")


def _check_f32(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")


def make_params(p=None) -> L.gs_params:
    """gs_params from any object with lowpass, kappa, alpha_min, alpha_max, t_min, guard, bg."""
    s = L.gs_params()
    if p is None:
        s.lowpass, s.kappa, s.alpha_min, s.alpha_max, s.t_min, s.guard = 0.3, 3.0, 1.0 / 255.0, 0.99, 1e-4, 1.3
        s.bg[:] = [0.0, 0.0, 0.0]
        return s
    s.lowpass, s.kappa, s.alpha_min, s.alpha_max = p.lowpass, p.kappa, p.alpha_min, p.alpha_max
    s.t_min, s.guard = p.t_min, p.guard
    s.bg[:] = list(p.bg)
    return s


@dataclass
class Gaussians:
    mean: torch.Tensor      # [3][n] float32
    scale: torch.Tensor     # [3][n]
    quat: torch.Tensor      # [4][n]
    opacity: torch.Tensor   # [n]
    sh: torch.Tensor        # [(d+1)^2*3][n]
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    @classmethod
    def from_arrays(cls, mean, scale, quat, opacity, sh, sh_degree, device=None) -> "Gaussians":
        dev = _dev(device)
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a) if isinstance(a, np.ndarray) else a,
                                      dtype=torch.float32).to(dev).contiguous()
        return cls(f(mean), f(scale), f(quat), f(opacity), f(sh), int(sh_degree))

    @classmethod
    def from_scene(cls, scene, device=None) -> "Gaussians":
        return cls.from_arrays(scene.mean, scene.scale, scene.quat, scene.opacity, scene.sh, scene.sh_degree, device)

    def struct(self) -> L.gs_gaussians:
        for t in (self.mean, self.scale, self.quat, self.opacity, self.sh):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError("Gaussian parameters must be contiguous float32 device tensors")
        return L.gs_gaussians(_ptr(self.mean), _ptr(self.scale), _ptr(self.quat), _ptr(self.opacity), _ptr(self.sh),
                              self.n, self.sh_degree)


def camera_struct(cam) -> L.gs_camera:
    c = L.gs_camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).reshape(-1)]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32)]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(cam.znear)
    c.reserved = 0
    return c


class ViewBatch:
    """Views rendered in one call: cameras, tile size and the global tile/pixel layout."""

    def __init__(self, cams: Sequence, tile: Tuple[int, int] = DEFAULT_TILE, device=None, batch_depth: int = 1,
                 lpt: bool = False, pixels_per_lane: int = 0):
        lib = L.load()
        self.cams = list(cams)
        self.n_views = len(self.cams)
        self.tile = (int(tile[0]), int(tile[1]))
        self.batch_depth = int(batch_depth)
        self.lpt = bool(lpt)  # traversals take tiles longest list first
        self.pixels_per_lane = int(pixels_per_lane)  # reverse traversal; 0 = the library's default
        self.device = _dev(device)
        arr = (L.gs_camera * self.n_views)(*[camera_struct(c) for c in self.cams])
        toff = (ctypes.c_int32 * (self.n_views + 1))()
        poff = (ctypes.c_int64 * (self.n_views + 1))()
        L.check(lib.gs_view_layout(arr, self.n_views, self.tile[0], self.tile[1], toff, poff))
        self.tile_offset_host = np.array(toff[:], np.int64)
        self.pixel_offset_host = np.array(poff[:], np.int64)
        self.n_tiles = int(self.tile_offset_host[-1])
        self.max_view_tiles = int(np.diff(self.tile_offset_host).max()) if self.n_views else 0
        self.n_pixels = int(self.pixel_offset_host[-1])
        raw = bytes(arr)
        self.cams_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        self.tile_offset = torch.tensor(self.tile_offset_host, dtype=torch.int32, device=self.device)
        self.pixel_offset = torch.tensor(self.pixel_offset_host, dtype=torch.int64, device=self.device)
        self.sizes = [(int(c.width), int(c.height)) for c in self.cams]

    def struct(self) -> L.gs_views:
        return L.gs_views(_ptr(self.cams_dev), _ptr(self.tile_offset), _ptr(self.pixel_offset), self.n_views,
                          self.tile[0], self.tile[1], self.n_tiles, self.n_pixels, self.batch_depth,
                          int(self.lpt), self.pixels_per_lane, self.max_view_tiles)

    def image(self, rgb: torch.Tensor, v: int) -> torch.Tensor:
        """View v's planar [3][H][W] image inside a global rgb buffer."""
        W, H = self.sizes[v]
        o = int(self.pixel_offset_host[v])
        return rgb[3 * o:3 * o + 3 * W * H].view(3, H, W)

    def plane(self, buf: torch.Tensor, v: int) -> torch.Tensor:
        """View v's [H][W] slice of a per-pixel buffer (t_final, n_last)."""
        W, H = self.sizes[v]
        o = int(self.pixel_offset_host[v])
        return buf[o:o + W * H].view(H, W)

    def pack_images(self, images: Sequence) -> torch.Tensor:
        """Concatenate per-view [3][H][W] images into the global rgb layout."""
        return torch.cat([torch.as_tensor(im, dtype=torch.float32).reshape(-1) for im in images]).to(self.device)


class Projected:
    def __init__(self, n: int, n_views: int, device):
        self.n = int(n)
        self.n_views = int(n_views)
        vn = max(self.n * self.n_views, 1)
        self.splat = torch.empty(vn * L.SPLAT_BYTES, dtype=torch.uint8, device=device)
        self.depth = torch.empty(vn, dtype=torch.float32, device=device)
        self.rect = torch.empty(vn, dtype=torch.int64, device=device)
        self.count = torch.empty(vn, dtype=torch.int32, device=device)

    def struct(self) -> L.gs_projected:
        return L.gs_projected(_ptr(self.splat), _ptr(self.depth), _ptr(self.rect), _ptr(self.count), self.n)

    def splat_fields(self):
        """Records as float64 [V*n][8] (u, v, ca, cb, cc, qmax, opacity|r, g|b bits)."""
        return self.splat.view(torch.float64).view(-1, 8)


class Bins:
    """Sorted pairs and tile ranges. `queue` (the longest-first tile order) is only built
    when asked for (views with lpt need it); `entry_offset` (the emission slot of every
    (view, entry), which the backward needs) only when entries > 0. `overflow_sticky`
    collects the overflow word of every bin_sort since construction (or the last clear)."""

    def __init__(self, capacity: int, n_tiles: int, device, queue: bool = True, entries: int = 0):
        self.capacity = int(capacity)
        cap = max(self.capacity, 1)
        self.keys = torch.empty(cap, dtype=torch.int64, device=device)
        self.vals = torch.empty(cap, dtype=torch.int32, device=device)
        self.ranges = torch.empty(max(2 * n_tiles, 2), dtype=torch.int32, device=device)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        self.overflow_sticky = torch.zeros(1, dtype=torch.int32, device=device)
        self.queue = torch.empty(max(n_tiles, 1), dtype=torch.int32, device=device) if queue else None
        self.entries = int(entries)
        self.entry_offset = (torch.empty(self.entries, dtype=torch.int32, device=device) if self.entries > 0
                             else None)

    def struct(self) -> L.gs_bins:
        return L.gs_bins(_ptr(self.keys), _ptr(self.vals), _ptr(self.ranges), self.capacity, _ptr(self.n_pairs),
                         _ptr(self.overflow), _ptr(self.queue), _ptr(self.entry_offset), _ptr(self.overflow_sticky))


def workspace_bytes(n: int, n_views: int, capacity: int, n_tiles: int) -> int:
    return int(L.load().gs_workspace_bytes(int(n), int(n_views), int(capacity), int(n_tiles)))


def alloc_workspace(n, n_views, capacity, n_tiles, device) -> torch.Tensor:
    return torch.empty(max(workspace_bytes(n, n_views, capacity, n_tiles), 256), dtype=torch.uint8, device=device)


def preprocess(g: Gaussians, views: ViewBatch, params=None, subset: Optional[torch.Tensor] = None,
               want_color: bool = True, out: Optional[Projected] = None) -> Projected:
    lib = L.load()
    n = g.n if subset is None else int(subset.shape[0])
    if out is None:
        out = Projected(n, views.n_views, views.device)
    if subset is not None and not (subset.dtype == torch.int32 and subset.is_cuda and subset.is_contiguous()):
        raise ValueError("subset must be a contiguous int32 device tensor")
    p = make_params(params)
    L.check(lib.gs_preprocess(ctypes.byref(g.struct()), ctypes.byref(views.struct()), ctypes.byref(p),
                              _ptr(subset), n, int(bool(want_color)), ctypes.byref(out.struct()), _stream(views.device)))
    return out


def bin_sort(proj: Projected, views: ViewBatch, capacity: Optional[int] = None, bins: Optional[Bins] = None,
             ws: Optional[torch.Tensor] = None, grow: bool = True, backward: bool = False) -> Bins:
    """Bin and sort. With grow=True the pair count is read back (one host sync) and the call
    is repeated with a larger buffer when the capacity was too small. backward=True keeps the
    entries' emission slots, which render_bwd needs."""
    lib = L.load()
    entries = proj.n * views.n_views if backward else 0
    if bins is None:
        if capacity is None:
            capacity = max(1 << 16, 4 * proj.n * views.n_views)
        bins = Bins(capacity, views.n_tiles, views.device, queue=views.lpt, entries=entries)
    for _ in range(3):
        need = workspace_bytes(proj.n, views.n_views, bins.capacity, views.n_tiles)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=views.device)
        L.check(lib.gs_bin_sort(ctypes.byref(proj.struct()), ctypes.byref(views.struct()), ctypes.byref(bins.struct()),
                                _ptr(ws), ws.numel(), _stream(views.device)))
        if not grow:
            return bins
        if int(bins.overflow.item()) == 0:
            return bins
        need_pairs = int(bins.n_pairs.item())
        bins = Bins(int(need_pairs * 1.125) + 4096, views.n_tiles, views.device, queue=bins.queue is not None,
                    entries=bins.entries)
    raise RuntimeError("bin_sort: capacity growth did not converge")


def render_fwd(proj: Projected, views: ViewBatch, bins: Bins, params=None, rgb=None, t_final=None, n_last=None,
               n_contrib=None):
    lib = L.load()
    dev = views.device
    if rgb is None:
        rgb = torch.empty(3 * max(views.n_pixels, 1), dtype=torch.float32, device=dev)
        t_final = torch.empty(max(views.n_pixels, 1), dtype=torch.float32, device=dev)
        n_last = torch.empty(max(views.n_pixels, 1), dtype=torch.int32, device=dev)
    p = make_params(params)
    L.check(lib.gs_render_fwd(ctypes.byref(proj.struct()), ctypes.byref(views.struct()), ctypes.byref(bins.struct()),
                              ctypes.byref(p), _ptr(rgb), _ptr(t_final), _ptr(n_last), _ptr(n_contrib), _stream(dev)))
    return rgb, t_final, n_last


def l1_loss_grad(rgb: torch.Tensor, target: torch.Tensor, dl_drgb: Optional[torch.Tensor] = None,
                 loss: Optional[torch.Tensor] = None, scale: Optional[float] = None):
    """L1 loss (mean over elements by default) and its gradient, both on the device."""
    n = rgb.numel()
    if dl_drgb is None:
        dl_drgb = torch.empty_like(rgb)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=rgb.device)
    s = 1.0 / max(n, 1) if scale is None else scale
    L.check(L.load().gs_l1_loss_grad(_ptr(rgb), _ptr(target), n, float(s), _ptr(dl_drgb), _ptr(loss),
                                     _stream(rgb.device)))
    return loss, dl_drgb


SSIM_LAMBDA = 0.2


def ssim_workspace_bytes(n_planes: int, height: int, width: int) -> int:
    return int(L.load().gs_ssim_workspace_bytes(n_planes, height, width))


def ssim_loss_grad(img: torch.Tensor, target: torch.Tensor, dl_dimg: Optional[torch.Tensor] = None,
                   loss: Optional[torch.Tensor] = None, lam: float = SSIM_LAMBDA, n_norm: Optional[int] = None,
                   ws: Optional[torch.Tensor] = None):
    """The Sec. 3.2 training loss (1 - lam) L2 + lam D-SSIM of img against target, both
    [..., H, W] stacks of planes, and its gradient, on the device. n_norm is the element count
    the means run over (img.numel() by default; the batch total when views of different
    sizes are passed one call each). Returns (loss, dl_dimg); loss accumulates (+=)."""
    _check_f32(img, "img")
    _check_f32(target, "target")
    if img.shape != target.shape or img.dim() < 2:
        raise ValueError("img and target must be [..., H, W] stacks of the same shape")
    h, w = int(img.shape[-2]), int(img.shape[-1])
    planes = img.numel() // max(h * w, 1)
    if dl_dimg is None:
        dl_dimg = torch.empty_like(img)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=img.device)
    need = ssim_workspace_bytes(planes, h, w)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=img.device)
    n = img.numel() if n_norm is None else int(n_norm)
    L.check(L.load().gs_ssim_loss_grad(_ptr(img), _ptr(target), planes, h, w, n, float(lam), _ptr(dl_dimg),
                                       _ptr(loss), _ptr(ws), ws.numel(), _stream(img.device)))
    return loss, dl_dimg


def render(g: Gaussians, views: ViewBatch, params=None, subset=None, capacity=None, backward: bool = True):
    """Plain path: preprocess -> bin_sort (growing the pair buffer if needed) -> render_fwd.
    backward=True keeps what render_bwd needs (the emission slots of the pairs)."""
    proj = preprocess(g, views, params, subset=subset)
    bins = bin_sort(proj, views, capacity, backward=backward and subset is None)
    rgb, t, last = render_fwd(proj, views, bins, params)
    return {"rgb": rgb, "t_final": t, "n_last": last, "proj": proj, "bins": bins}


def render_batch(g: Gaussians, cams: Sequence, params=None, tile: Tuple[int, int] = DEFAULT_TILE,
                 batch_depth: int = 1, lpt: bool = False, device=None) -> List[torch.Tensor]:
    """Every view of cams in one launch per stage (views of uneven size share one global tile
    space); returns each view's planar [3][H][W] image, a view of the batch's rgb buffer."""
    views = ViewBatch(cams, tile, _dev(device), batch_depth, lpt)
    out = render(g, views, params, backward=False)
    return [views.image(out["rgb"], v) for v in range(len(cams))]


def render_filtered(g: Gaussians, cam, lists: Sequence[torch.Tensor], centres: np.ndarray, params=None,
                    tile: Tuple[int, int] = DEFAULT_TILE, device=None) -> torch.Tensor:
    """A test view rendered with the visibility list of the cluster centre nearest to its camera
    centre (Sec. 3.4; ties to the lowest centre): planar [3][H][W] image."""
    c = nearest_centre(centres, cam.position)
    views = ViewBatch([cam], tile, _dev(device))
    return views.image(render(g, views, params, subset=lists[c])["rgb"], 0)


def importance(g: Gaussians, views: ViewBatch, params=None, h: Optional[torch.Tensor] = None, capacity=None):
    """h = max(h, importance over the views' pixels) (eq. importance-score); h starts at 0."""
    lib = L.load()
    if h is None:
        h = torch.zeros(max(g.n, 1), dtype=torch.float32, device=views.device)
    proj = preprocess(g, views, params, want_color=False)
    bins = bin_sort(proj, views, capacity)
    p = make_params(params)
    L.check(lib.gs_importance(ctypes.byref(proj.struct()), ctypes.byref(views.struct()), ctypes.byref(bins.struct()),
                              ctypes.byref(p), _ptr(h), _stream(views.device)))
    return h


def prune_mask(h: torch.Tensor, t_prune: float) -> torch.Tensor:
    """m_i = 1(h_i < t_prune): True marks a Gaussian to remove (Sec. 3.3)."""
    _check_f32(h, "h")
    mask = torch.empty(h.numel(), dtype=torch.uint8, device=h.device)
    L.check(L.load().gs_prune_mask(_ptr(h), h.numel(), float(t_prune), _ptr(mask), _stream(h.device)))
    return mask.bool()


def prune(h: torch.Tensor, t_prune: float, planes: Sequence[torch.Tensor]):
    """Remove the Gaussians with h < t_prune from every per-Gaussian FP32 plane (Sec. 3.3):
    returns (compacted planes, kept indices). A plane is a tensor whose last dimension has
    length n (for example mean [3, n], sh [48, n], or an optimizer moment shaped like a
    parameter). Reads the kept count back (one host synchronisation)."""
    _check_f32(h, "h")
    n = h.numel()
    dev = h.device
    rows_in, shapes = [], []
    for t in planes:
        _check_f32(t, "plane")
        if t.shape[-1] != n:
            raise ValueError(f"plane of shape {tuple(t.shape)} does not end in n = {n}")
        r = t.reshape(-1, n)
        rows_in.extend(r[k] for k in range(r.shape[0]))
        shapes.append(tuple(t.shape[:-1]))
    outs = [torch.empty((int(np.prod(sh, dtype=np.int64)), n), dtype=torch.float32, device=dev) for sh in shapes]
    rows_out = [o[k] for o in outs for k in range(o.shape[0])]
    kept = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    n_kept = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = alloc_workspace(n, 1, 0, 0, dev)
    vp = ctypes.c_void_p * max(len(rows_in), 1)
    pin = vp(*[r.data_ptr() for r in rows_in])
    pout = vp(*[r.data_ptr() for r in rows_out])
    L.check(L.load().gs_prune(_ptr(h), n, float(t_prune), pin, pout, len(rows_in), _ptr(kept), _ptr(n_kept), _ptr(ws),
                              ws.numel(), _stream(dev)))
    nk = int(n_kept.item())
    res = [o[:, :nk].reshape(*sh, nk).clone() if nk else o[:, :0].reshape(*sh, 0) for o, sh in zip(outs, shapes)]
    return res, kept[:nk]


def prune_gaussians(g: "Gaussians", h: torch.Tensor, t_prune: float, extra: Sequence[torch.Tensor] = ()):
    """Pruned copy of the Gaussians (and of any per-Gaussian state in `extra`), plus the kept
    indices."""
    planes = [g.mean, g.scale, g.quat, g.opacity, g.sh, *extra]
    out, kept = prune(h, t_prune, planes)
    pg = Gaussians(out[0], out[1], out[2], out[3], out[4], g.sh_degree)
    return pg, kept, out[5:]


def gather(index: torch.Tensor, planes: Sequence[torch.Tensor], n_src: Optional[int] = None):
    """out[..., k] = plane[..., index[k]] for every per-Gaussian FP32 plane (last dimension n_src):
    compact copies of a Gaussian subset, such as a visibility list (Sec. 3.4). No host
    synchronisation."""
    if not (index.is_cuda and index.dtype == torch.int32 and index.is_contiguous() and index.dim() == 1):
        raise ValueError("index must be a contiguous 1D int32 device tensor")
    m = index.numel()
    n = planes[0].shape[-1] if n_src is None else int(n_src)
    rows_in, outs = [], []
    for t in planes:
        _check_f32(t, "plane")
        if t.shape[-1] != n:
            raise ValueError(f"plane of shape {tuple(t.shape)} does not end in n = {n}")
        r = t.reshape(-1, n)
        rows_in.extend(r[k] for k in range(r.shape[0]))
        outs.append(torch.empty((*t.shape[:-1], m), dtype=torch.float32, device=index.device))
    rows_out = [r for o in outs for r in o.reshape(int(np.prod(o.shape[:-1], dtype=np.int64)), m)]
    vp = ctypes.c_void_p * max(len(rows_in), 1)
    L.check(L.load().gs_gather(_ptr(index), m, n, vp(*[r.data_ptr() for r in rows_in]),
                               vp(*[r.data_ptr() for r in rows_out]), len(rows_in), _stream(index.device)))
    return outs


def gather_gaussians(g: "Gaussians", index: torch.Tensor, extra: Sequence[torch.Tensor] = ()):
    """Compact copy of the Gaussians listed in index (and of any per-Gaussian state in extra).
    With an increasing index list the copy keeps the subset's order, so its renders equal the
    renders of the subset."""
    out = gather(index, [g.mean, g.scale, g.quat, g.opacity, g.sh, *extra], g.n)
    return Gaussians(out[0], out[1], out[2], out[3], out[4], g.sh_degree), out[5:]


def nn_distance(points: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Distance from each point of points [3][n] to the nearest point at another position
    (the initial isotropic scale of Sec. 3.2); +inf without such a point."""
    _check_f32(points, "points")
    if points.dim() != 2 or points.shape[0] != 3:
        raise ValueError("points must be [3, n]")
    n = int(points.shape[1])
    dist = torch.empty(n, dtype=torch.float32, device=points.device)
    need = int(L.load().gs_nn_workspace_bytes(n))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=points.device)
    L.check(L.load().gs_nn_distance(_ptr(points), n, _ptr(dist), _ptr(ws), ws.numel(), _stream(points.device)))
    return dist


def init_gaussians(points: torch.Tensor, colours: Optional[torch.Tensor] = None, sh_degree: int = 3) -> "Gaussians":
    """Gaussians initialised from a point set (Sec. 3.2): mean = points, isotropic scale = the
    nearest-neighbour distance, identity rotation, opacity 0.1, DC colour = colours [3][n]
    (1/2 when None), higher SH 0."""
    _check_f32(points, "points")
    if points.dim() != 2 or points.shape[0] != 3:
        raise ValueError("points must be [3, n]")
    if colours is not None:
        _check_f32(colours, "colours")
        if colours.shape != points.shape:
            raise ValueError("colours must be shaped like points")
    n, dev = int(points.shape[1]), points.device
    e = lambda r: torch.empty((r, n), dtype=torch.float32, device=dev)
    g = Gaussians(e(3), e(3), e(4), torch.empty(n, dtype=torch.float32, device=dev), e((sh_degree + 1) ** 2 * 3),
                  int(sh_degree))
    need = int(L.load().gs_nn_workspace_bytes(n))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    L.check(L.load().gs_init_gaussians(_ptr(points), _ptr(colours), n, int(sh_degree), _ptr(g.mean), _ptr(g.scale),
                                       _ptr(g.quat), _ptr(g.opacity), _ptr(g.sh), _ptr(ws), ws.numel(), _stream(dev)))
    return g


ADAM_MODES = {"linear": L.GS_ADAM_LINEAR, "log": L.GS_ADAM_LOG, "logit": L.GS_ADAM_LOGIT}


def adam_step(groups: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor, float, str]], step: int,
              betas: Tuple[float, float] = (0.9, 0.999), eps: float = 1e-15, zero_grad: bool = True):
    """One fused Adam step (gs_adam_step) over groups (param, grad, m, v, lr, mode) of
    contiguous FP32 device tensors; mode is "linear", "log" or "logit". Clears the gradients
    when zero_grad is set. No allocation on the device, no host synchronisation."""
    arr = (L.gs_adam_group * max(len(groups), 1))()
    dev = None
    for k, (x, g, m, v, lr, mode) in enumerate(groups):
        for t in (x, g, m, v):
            _check_f32(t, "Adam buffer")
        if not (x.numel() == g.numel() == m.numel() == v.numel()):
            raise ValueError("param, grad and moments must have the same number of elements")
        arr[k] = L.gs_adam_group(_ptr(x), _ptr(g), _ptr(m), _ptr(v), x.numel(), float(lr), ADAM_MODES[mode])
        dev = x.device
    if not groups:
        return
    L.check(L.load().gs_adam_step(arr, len(groups), float(betas[0]), float(betas[1]), float(eps), int(step),
                                  int(bool(zero_grad)), _stream(dev)))


def cluster_visibility(g: Gaussians, views: ViewBatch, view_cluster: Sequence[int], k: int, t_cluster: float,
                       params=None, bits: Optional[torch.Tensor] = None, capacity=None) -> torch.Tensor:
    """OR into bits [k][ceil(n/32)] the per-cluster indicator lists (eq. importance-score-vis)."""
    lib = L.load()
    words = (g.n + 31) // 32
    ids = np.asarray(view_cluster, np.int64).reshape(-1)
    if k < 1 or ids.shape[0] != views.n_views or (ids.size and (ids.min() < 0 or ids.max() >= k)):
        raise ValueError(f"view_cluster must hold one id in [0, {k}) per view")
    if bits is None:
        bits = torch.zeros(max(k * words, 1), dtype=torch.int32, device=views.device)
    elif bits.dtype != torch.int32 or not bits.is_cuda or bits.numel() < k * words:
        raise ValueError(f"bits must be an int32 device tensor of at least k * ceil(n / 32) = {k * words} words")
    vc = torch.as_tensor(ids.astype(np.int32), device=views.device)
    proj = preprocess(g, views, params, want_color=False)
    bins = bin_sort(proj, views, capacity)
    p = make_params(params)
    L.check(lib.gs_cluster_visibility(ctypes.byref(proj.struct()), ctypes.byref(views.struct()),
                                      ctypes.byref(bins.struct()), ctypes.byref(p), _ptr(vc), int(k), float(t_cluster),
                                      _ptr(bits), _stream(views.device)))
    return bits


def bits_to_list(bits_row: torch.Tensor, n: int) -> torch.Tensor:
    """Sorted indices of the set bits of one visibility row (device int32 tensor)."""
    lib = L.load()
    dev = bits_row.device
    out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = alloc_workspace(n, 1, 0, 0, dev)
    L.check(lib.gs_bits_to_list(_ptr(bits_row), int(n), _ptr(out), _ptr(cnt), _ptr(ws), ws.numel(), _stream(dev)))
    return out[:int(cnt.item())]


def render_bwd(g: Gaussians, views: ViewBatch, proj: Projected, bins: Bins, t_final, n_last, dl_drgb, params=None,
               grad: Optional[Gaussians] = None, ws: Optional[torch.Tensor] = None,
               overwrite: Optional[bool] = None) -> Gaussians:
    """dL/dparams (given dL/drgb in the global image layout): added into grad, or written into it
    with overwrite=True (every entry, no clearing needed). With grad None, new buffers are
    written (overwrite is then always on)."""
    lib = L.load()
    dev = views.device
    if grad is None:
        grad = Gaussians(torch.empty_like(g.mean), torch.empty_like(g.scale), torch.empty_like(g.quat),
                         torch.empty_like(g.opacity), torch.empty_like(g.sh), g.sh_degree)
        overwrite = True
    if bins.entry_offset is None:
        raise ValueError("render_bwd needs bins made with backward=True (the pairs' emission slots)")
    need = workspace_bytes(g.n, views.n_views, bins.capacity, views.n_tiles)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    gg = L.gs_gaussians_grad(_ptr(grad.mean), _ptr(grad.scale), _ptr(grad.quat), _ptr(grad.opacity), _ptr(grad.sh),
                             g.n, g.sh_degree, int(bool(overwrite)))
    p = make_params(params)
    dl = dl_drgb.contiguous()
    L.check(lib.gs_render_bwd(ctypes.byref(g.struct()), ctypes.byref(views.struct()), ctypes.byref(proj.struct()),
                              ctypes.byref(bins.struct()), ctypes.byref(p), _ptr(t_final), _ptr(n_last), _ptr(dl),
                              ctypes.byref(gg), _ptr(ws), ws.numel(), _stream(dev)))
    return grad


class GSRender(torch.autograd.Function):
    """Differentiable render of a view batch: (mean, scale, quat, opacity, sh) -> rgb in the
    global image layout. The backward is the hand-written reverse traversal."""

    @staticmethod
    def forward(ctx, mean, scale, quat, opacity, sh, views: ViewBatch, sh_degree: int, params=None):
        g = Gaussians(mean.detach().contiguous(), scale.detach().contiguous(), quat.detach().contiguous(),
                      opacity.detach().contiguous(), sh.detach().contiguous(), sh_degree)
        out = render(g, views, params)
        ctx.state = (g, views, out["proj"], out["bins"], out["t_final"], out["n_last"], params)
        return out["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        g, views, proj, bins, t, last, params = ctx.state
        grad = render_bwd(g, views, proj, bins, t, last, grad_rgb, params)
        return grad.mean, grad.scale, grad.quat, grad.opacity, grad.sh, None, None, None


def kmeans(pos: np.ndarray, k: int, seed: int = 3, max_iter: int = 100, device=None):
    """FP64 k-means on camera positions [m][3] -> (centres [k][3], assignment [m]), host arrays.
    With a device, the seeding runs on the host and the Lloyd iterations on that GPU
    (kmeans_lloyd): the same clustering up to the last bits of the centres."""
    if device is not None:
        pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
        cen = torch.as_tensor(kmeans_seed(pos, k, seed), device=device)
        asg, _ = kmeans_lloyd(torch.as_tensor(pos, device=device), cen, max(1, int(max_iter)))
        return cen.cpu().numpy(), asg.cpu().numpy()
    lib = L.load()
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    m = pos.shape[0]
    cen = np.zeros((k, 3), np.float64)
    asg = np.zeros(m, np.int32)
    L.check(lib.gs_kmeans(pos.ctypes.data_as(ctypes.c_void_p), m, int(k), int(seed), int(max_iter),
                          cen.ctypes.data_as(ctypes.c_void_p), asg.ctypes.data_as(ctypes.c_void_p)))
    return cen, asg


def kmeans_seed(pos: np.ndarray, k: int, seed: int = 3) -> np.ndarray:
    """The k-means++ seeding of kmeans() alone: initial centres [k][3] (host, FP64)."""
    lib = L.load()
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    cen = np.zeros((k, 3), np.float64)
    L.check(lib.gs_kmeans_seed(pos.ctypes.data_as(ctypes.c_void_p), pos.shape[0], int(k), int(seed),
                               cen.ctypes.data_as(ctypes.c_void_p)))
    return cen


def kmeans_lloyd(pos: torch.Tensor, centres: torch.Tensor, max_iter: int = 100,
                 ws: Optional[torch.Tensor] = None):
    """Device FP64 Lloyd iterations from the given centres (Sec. 3.4 camera clustering, for large
    camera sets). pos: device [m][3] float64; centres: device [k][3] float64, updated in place.
    Returns (assignment [m] int32, iterations [1] int32), both on the device; nothing waits."""
    if pos.dtype != torch.float64 or centres.dtype != torch.float64:
        raise TypeError("pos and centres must be float64")
    if pos.device.type != "cuda" or centres.device != pos.device:
        raise ValueError("pos and centres must be on the same GPU")
    if pos.dim() != 2 or pos.shape[1] != 3 or centres.dim() != 2 or centres.shape[1] != 3:
        raise ValueError("pos must be [m, 3] and centres [k, 3]")
    if not (pos.is_contiguous() and centres.is_contiguous()):
        raise ValueError("pos and centres must be contiguous")
    m, k = int(pos.shape[0]), int(centres.shape[0])
    lib = L.load()
    assign = torch.empty(m, dtype=torch.int32, device=pos.device)
    iters = torch.zeros(1, dtype=torch.int32, device=pos.device)
    need = int(lib.gs_kmeans_workspace_bytes(m, k, int(max_iter)))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=pos.device)
    L.check(lib.gs_kmeans_lloyd(_ptr(pos), m, k, int(max_iter), _ptr(centres), _ptr(assign), _ptr(iters), _ptr(ws),
                                ws.numel(), _stream(pos.device)))
    return assign, iters


def nearest_centre(centres: np.ndarray, x) -> int:
    lib = L.load()
    c = np.ascontiguousarray(centres, np.float64)
    xx = np.ascontiguousarray(x, np.float64)
    return int(lib.gs_nearest_centre(c.ctypes.data_as(ctypes.c_void_p), c.shape[0], xx.ctypes.data_as(ctypes.c_void_p)))


class Renderer:
    """Repeated frames of one view batch with persistent buffers: no allocation and no host
    synchronisation per frame. The pair capacity is fixed at construction (from a first
    sized run); check() reports whether any frame since construction (or the last
    clear_overflow()) overflowed it. backward=False leaves out the pairs' emission slots,
    which only backward() reads."""

    def __init__(self, g: Gaussians, views: ViewBatch, params=None, capacity: Optional[int] = None,
                 want_color: bool = True, headroom: float = 1.25, subset: Optional[torch.Tensor] = None,
                 backward: bool = True):
        self.g, self.views, self.params = g, views, params
        self.p = make_params(params)
        dev = views.device
        self.subset = subset
        self.n_entries = g.n if subset is None else int(subset.shape[0])
        self.proj = Projected(self.n_entries, views.n_views, dev)
        preprocess(g, views, params, subset=subset, want_color=want_color, out=self.proj)
        if capacity is None:
            b = bin_sort(self.proj, views)
            capacity = int(int(b.n_pairs.item()) * headroom) + 4096
        self.backward_ok = bool(backward) and subset is None
        self.bins = Bins(capacity, views.n_tiles, dev, queue=views.lpt,
                         entries=self.n_entries * views.n_views if self.backward_ok else 0)
        self.ws = alloc_workspace(self.n_entries, views.n_views, capacity, views.n_tiles, dev)
        self.rgb = torch.empty(3 * max(views.n_pixels, 1), dtype=torch.float32, device=dev)
        self.t_final = torch.empty(max(views.n_pixels, 1), dtype=torch.float32, device=dev)
        self.n_last = torch.empty(max(views.n_pixels, 1), dtype=torch.int32, device=dev)
        self.want_color = want_color
        self._sg = g.struct()
        self._sv = views.struct()
        self._sp = self.proj.struct()
        self._sb = self.bins.struct()

    def _pre(self, stream):
        lib = L.load()
        L.check(lib.gs_preprocess(ctypes.byref(self._sg), ctypes.byref(self._sv), ctypes.byref(self.p),
                                  _ptr(self.subset), self.n_entries, int(self.want_color), ctypes.byref(self._sp),
                                  stream))
        L.check(lib.gs_bin_sort(ctypes.byref(self._sp), ctypes.byref(self._sv), ctypes.byref(self._sb),
                                _ptr(self.ws), self.ws.numel(), stream))

    def forward(self):
        s = _stream(self.views.device)
        lib = L.load()
        L.check(lib.gs_preprocess(ctypes.byref(self._sg), ctypes.byref(self._sv), ctypes.byref(self.p),
                                  _ptr(self.subset), self.n_entries, int(self.want_color), ctypes.byref(self._sp), s))
        # binning, and each tile's sort inside the compositing launch
        L.check(lib.gs_bin_sort_render_fwd(ctypes.byref(self._sp), ctypes.byref(self._sv), ctypes.byref(self._sb),
                                           ctypes.byref(self.p), _ptr(self.rgb), _ptr(self.t_final),
                                           _ptr(self.n_last), None, _ptr(self.ws), self.ws.numel(), s))
        return self.rgb

    def render_only(self, s=None, n_contrib: Optional[torch.Tensor] = None):
        """Compositing pass alone over the current bins (after forward() or _pre())."""
        s = _stream(self.views.device) if s is None else s
        L.check(L.load().gs_render_fwd(ctypes.byref(self._sp), ctypes.byref(self._sv), ctypes.byref(self._sb),
                                       ctypes.byref(self.p), _ptr(self.rgb), _ptr(self.t_final), _ptr(self.n_last),
                                       _ptr(n_contrib), s))

    def importance(self, h: torch.Tensor):
        s = _stream(self.views.device)
        lib = L.load()
        L.check(lib.gs_preprocess(ctypes.byref(self._sg), ctypes.byref(self._sv), ctypes.byref(self.p),
                                  _ptr(self.subset), self.n_entries, int(self.want_color), ctypes.byref(self._sp), s))
        # binning, and each tile's sort inside the importance launch
        L.check(lib.gs_bin_sort_importance(ctypes.byref(self._sp), ctypes.byref(self._sv), ctypes.byref(self._sb),
                                           ctypes.byref(self.p), _ptr(h), _ptr(self.ws), self.ws.numel(), s))
        return h

    def importance_split(self, h: torch.Tensor):
        """importance() with the binning's own sort launch, then the importance pass."""
        s = _stream(self.views.device)
        self._pre(s)
        L.check(L.load().gs_importance(ctypes.byref(self._sp), ctypes.byref(self._sv), ctypes.byref(self._sb),
                                       ctypes.byref(self.p), _ptr(h), s))
        return h

    def backward(self, dl_drgb: torch.Tensor, grad: Gaussians, overwrite: bool = False):
        """dL/dparams of the last forward(): added into grad, or written into every entry of it
        with overwrite=True (then grad needs no clearing)."""
        if not self.backward_ok:
            raise ValueError("this Renderer was built without the backward (a subset, or backward=False)")
        s = _stream(self.views.device)
        gg = L.gs_gaussians_grad(_ptr(grad.mean), _ptr(grad.scale), _ptr(grad.quat), _ptr(grad.opacity),
                                 _ptr(grad.sh), self.g.n, self.g.sh_degree, int(bool(overwrite)))
        L.check(L.load().gs_render_bwd(ctypes.byref(self._sg), ctypes.byref(self._sv), ctypes.byref(self._sp),
                                       ctypes.byref(self._sb), ctypes.byref(self.p), _ptr(self.t_final),
                                       _ptr(self.n_last), _ptr(dl_drgb), ctypes.byref(gg), _ptr(self.ws),
                                       self.ws.numel(), s))
        return grad

    def check(self) -> Tuple[bool, int]:
        """(some frame since construction or the last clear_overflow() overflowed the pair
        capacity, pairs of the last frame); synchronises."""
        return bool(int(self.bins.overflow_sticky.item())), int(self.bins.n_pairs.item())

    def clear_overflow(self):
        self.bins.overflow_sticky.zero_()


@dataclass
class PinholeCamera:
    """A camera in the form the binding reads (world -> camera p_c = R p + t)."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def position(self) -> np.ndarray:
        return -(np.asarray(self.R, np.float64).T @ np.asarray(self.t, np.float64))


def _camera_at(position, yaw, pitch, like) -> PinholeCamera:
    """Camera at `position` looking along (yaw, pitch) (y down), intrinsics copied from `like`."""
    fwd = np.array([np.cos(pitch) * np.sin(yaw), -np.sin(pitch), np.cos(pitch) * np.cos(yaw)])
    down = np.array([0.0, 1.0, 0.0])
    y = down - np.dot(down, fwd) * fwd
    y /= np.linalg.norm(y)
    x = np.cross(y, fwd)
    R = np.stack([x, y, fwd]).astype(np.float32)
    t = (-R.astype(np.float64) @ np.asarray(position, np.float64)).astype(np.float32)
    return PinholeCamera(R, t, like.fx, like.fy, like.cx, like.cy, like.width, like.height, like.znear)


class VisibilityFilter:
    """Viewpoint-based visibility filtering (Sec. 3.4): k-means clusters of the training
    camera positions; per cluster, the indicator list of the Gaussians composited with weight
    above t_cluster in some view of the cluster (eq. importance-score-vis); a test view is
    rendered with the list of the cluster centre nearest to its camera centre.

    extra_per_cluster random cameras are added to every cluster's views, as the method does
    for robustness to test views. With extra_placement="jitter" each sits at a random member
    camera's position moved by a uniform offset in a ball of radius `jitter`; with "cell" it is
    drawn uniformly from the part of the cluster centre's Voronoi cell (the positions whose
    nearest centre is this one, so the test views that will use this list) inside the box of
    the member cameras widened by `cell_margin` in x and z, at a member's height. Either way it
    looks in a random direction (yaw uniform, pitch uniform in +-max_pitch) and copies a
    member's intrinsics.

    The Lloyd iterations run on the GPU from DEVICE_KMEANS_CAMERAS cameras on (device_kmeans=None),
    or as asked; the host and device clusterings follow the same steps."""

    DEVICE_KMEANS_CAMERAS = 4096

    def __init__(self, g: Gaussians, train_cams: Sequence, k: int = 64, t_cluster: float = 0.001, params=None,
                 chunk: int = 8, tile: Tuple[int, int] = DEFAULT_TILE, seed: int = 3, device=None,
                 extra_per_cluster: int = 0, jitter: float = 1.0, max_pitch: float = np.deg2rad(30.0),
                 materialize: bool = False, device_kmeans: Optional[bool] = None, extra_placement: str = "jitter",
                 cell_margin: float = 6.0):
        if extra_placement not in ("jitter", "cell"):
            raise ValueError('extra_placement must be "jitter" or "cell"')
        dev = _dev(device)
        self.g, self.k, self.t_cluster, self.params, self.tile, self.device = g, k, t_cluster, params, tile, dev
        pos = np.stack([c.position for c in train_cams])
        if device_kmeans is None:
            device_kmeans = len(train_cams) >= self.DEVICE_KMEANS_CAMERAS
        self.centres, self.assign = kmeans(pos, k, seed=seed, device=dev if device_kmeans else None)
        views, owner = list(train_cams), list(self.assign)
        if extra_per_cluster > 0:
            rng = np.random.default_rng(seed)
            for c in range(k):
                members = np.nonzero(self.assign == c)[0]
                if members.size == 0:
                    continue
                if extra_placement == "cell":
                    spots = self._cell_positions(pos, members, c, extra_per_cluster, cell_margin, rng)
                for e in range(extra_per_cluster):
                    m = train_cams[int(rng.choice(members))]
                    if extra_placement == "cell":
                        where = spots[e]
                    else:
                        off = rng.standard_normal(3)
                        off *= jitter * rng.uniform() ** (1.0 / 3.0) / max(np.linalg.norm(off), 1e-12)
                        where = m.position + off
                    views.append(_camera_at(where, rng.uniform(0, 2 * np.pi), rng.uniform(-max_pitch, max_pitch), m))
                    owner.append(c)
        self.views_used = len(views)
        self.cluster_views, self.view_owner = views, np.asarray(owner, np.int32)  # every view and its cluster
        words = (g.n + 31) // 32
        self.bits = torch.zeros(max(k * words, 1), dtype=torch.int32, device=dev)
        owner = np.asarray(owner, np.int32)
        for c0 in range(0, len(views), chunk):
            vb = ViewBatch(views[c0:c0 + chunk], tile, dev)
            cluster_visibility(g, vb, owner[c0:c0 + chunk], k, t_cluster, params, bits=self.bits)
        self.lists = [bits_to_list(self.bits[c * words:(c + 1) * words], g.n) for c in range(k)]
        # materialised lists: each cluster's Gaussians copied into compact planes (memory for
        # coalesced loads: a filtered render then reads rows instead of gathering by index)
        self.copies = [gather_gaussians(g, lst)[0] for lst in self.lists] if materialize else None

    def _cell_positions(self, pos, members, c, count, margin, rng, tries=64):
        """count positions drawn uniformly from the Voronoi cell of centre c inside the box of
        the member cameras widened by margin in x and z, at member heights (rejection sampling;
        members' own positions fill in if the cell is too thin to hit)."""
        lo, hi = pos[members].min(0), pos[members].max(0)
        lo = lo - np.array([margin, 0.0, margin])
        hi = hi + np.array([margin, 0.0, margin])
        out = []
        for _ in range(tries):
            cand = rng.uniform(lo, hi, (4 * count, 3))
            cand[:, 1] = pos[rng.choice(members, 4 * count), 1]
            d = ((cand[:, None, :] - self.centres[None, :, :]) ** 2).sum(-1)
            out.extend(cand[np.argmin(d, 1) == c])
            if len(out) >= count:
                return np.asarray(out[:count])
        out.extend(pos[rng.choice(members, count)])
        return np.asarray(out[:count])

    def materialize(self):
        if self.copies is None:
            self.copies = [gather_gaussians(self.g, lst)[0] for lst in self.lists]
        return self

    def copy_bytes(self) -> int:
        return 0 if self.copies is None else sum(4 * (11 + c.sh.shape[0]) * c.n for c in self.copies)

    def cluster_of(self, cam) -> int:
        return nearest_centre(self.centres, cam.position)

    def list_for(self, cam) -> torch.Tensor:
        return self.lists[self.cluster_of(cam)]

    def copy_for(self, cam) -> "Gaussians":
        if self.copies is None:
            raise ValueError("the lists are not materialised (materialize=True or materialize())")
        return self.copies[self.cluster_of(cam)]

    def render(self, cam, capacity=None):
        views = ViewBatch([cam], self.tile, self.device)
        if self.copies is not None:
            return render(self.copy_for(cam), views, self.params, capacity=capacity)
        return render(self.g, views, self.params, subset=self.list_for(cam), capacity=capacity)


class PathRenderer:
    """Frames of a camera path (all of one resolution) rendered with persistent buffers and no
    host synchronisation per frame: the cameras of every frame are uploaded once and each
    frame points the view batch at its own camera. A frame may render only a subset of the
    Gaussians (a visibility list). The pair capacity is fixed; ok() reports overflows.

    pipeline = k > 1 keeps k buffer sets and k streams (default priority): frame f runs on
    stream f mod k, so the projection and binning of one frame overlap the compositing of the
    previous one. Its result stays valid until frame f + k is enqueued; call sync() before
    reading it on the current stream."""

    def __init__(self, g: Gaussians, cams: Sequence, params=None, tile: Tuple[int, int] = DEFAULT_TILE,
                 capacity: Optional[int] = None, max_entries: Optional[int] = None, device=None,
                 lpt: bool = False, batch_depth: int = 1, pipeline: int = 1):
        dev = _dev(device)
        self.g, self.params, self.device = g, params, dev
        self.p = make_params(params)
        self.views = ViewBatch([cams[0]], tile, dev, batch_depth, lpt)
        if any((c.width, c.height) != (cams[0].width, cams[0].height) for c in cams):
            raise ValueError("every frame of a path must have the same resolution")
        arr = (L.gs_camera * len(cams))(*[camera_struct(c) for c in cams])
        self.cams_all = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(dev)
        self.n_frames = len(cams)
        self.max_entries = g.n if max_entries is None else int(max_entries)
        self.proj = Projected(self.max_entries, 1, dev)
        if capacity is None:
            preprocess(g, self.views, params, out=self._proj_n(g.n))
            b = bin_sort(self._proj_n(g.n), self.views)
            capacity = int(int(b.n_pairs.item()) * 2.0) + 65536
        self.bins = Bins(capacity, self.views.n_tiles, dev, queue=self.views.lpt)
        self.ws = alloc_workspace(self.max_entries, 1, capacity, self.views.n_tiles, dev)
        self.rgb = torch.empty(3 * self.views.n_pixels, dtype=torch.float32, device=dev)
        self.t_final = torch.empty(self.views.n_pixels, dtype=torch.float32, device=dev)
        self.n_last = torch.empty(self.views.n_pixels, dtype=torch.int32, device=dev)
        self._sg = g.struct()
        self._sb = self.bins.struct()
        self._sets = [(self.proj, self.bins, self._sb, self.ws, self.rgb, self.t_final, self.n_last)]
        for _ in range(1, max(1, int(pipeline))):
            bins = Bins(capacity, self.views.n_tiles, dev, queue=self.views.lpt)
            self._sets.append((Projected(self.max_entries, 1, dev), bins, bins.struct(),
                               alloc_workspace(self.max_entries, 1, capacity, self.views.n_tiles, dev),
                               torch.empty_like(self.rgb), torch.empty_like(self.t_final),
                               torch.empty_like(self.n_last)))
        self.streams = [torch.cuda.Stream(device=dev) for _ in self._sets] if len(self._sets) > 1 else None

    def _proj_n(self, n):
        self.proj.n = n
        return self.proj

    def sync(self):
        """Make the current stream wait for every frame enqueued so far."""
        if self.streams:
            cur = torch.cuda.current_stream(self.device)
            for st in self.streams:
                cur.wait_stream(st)

    def frame(self, f: int, subset: Optional[torch.Tensor] = None, g: Optional["Gaussians"] = None):
        """Enqueue frame f (optionally with only the listed Gaussians, or with another set of
        Gaussians g such as a materialised visibility list); returns the rgb buffer."""
        lib = L.load()
        if g is not None and subset is not None:
            raise ValueError("pass a subset or a Gaussian set, not both")
        src = self._sg if g is None else g.struct()
        n = (self.g.n if g is None else g.n) if subset is None else int(subset.shape[0])
        if n > self.max_entries:
            raise ValueError("subset larger than max_entries")
        sv = self.views.struct()
        sv.cams = ctypes.c_void_p(self.cams_all.data_ptr() + ctypes.sizeof(L.gs_camera) * f)
        k = f % len(self._sets)
        proj, _, sb, ws, rgb, t_final, n_last = self._sets[k]
        proj.n = n
        sp = proj.struct()
        if self.streams:
            st = self.streams[k]
            st.wait_stream(torch.cuda.current_stream(self.device))  # inputs made on the caller's stream
            s = ctypes.c_void_p(st.cuda_stream)
        else:
            s = _stream(self.device)
        L.check(lib.gs_preprocess(ctypes.byref(src), ctypes.byref(sv), ctypes.byref(self.p), _ptr(subset), n, 1,
                                  ctypes.byref(sp), s))
        L.check(lib.gs_bin_sort_render_fwd(ctypes.byref(sp), ctypes.byref(sv), ctypes.byref(sb), ctypes.byref(self.p),
                                           _ptr(rgb), _ptr(t_final), _ptr(n_last), None, _ptr(ws), ws.numel(), s))
        return rgb

    def ok(self) -> bool:
        """True when no frame since construction overflowed its pair buffer (synchronises)."""
        self.sync()
        return all(int(b.overflow_sticky.item()) == 0 for _, b, *_ in self._sets)
