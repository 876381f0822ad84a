"""Batched training step (forward + loss + backward over many views of uneven size) as
one captured hipGraph, and the autotuner that picks its launch configuration. The loss is
L1 (loss="l1") or the Sec. 3.2 training loss 0.8 L2 + 0.2 D-SSIM (loss="l2_dssim", one
gs_ssim_loss_grad call per view with the batch's element count, sharing one workspace).

  StepConfig      tile size, batch depth (records staged per lane), tile order (longest
                  list first, or tile order) and pixels per lane of the traversals
  FwdBwdStep      preallocated buffers, an eager step, capture into a hipGraph, replay
  autotune        times every candidate configuration on the actual scene and views and
                  keeps the fastest; results are cached as JSON keyed by device, scene size
                  and the set of view resolutions
  Trainer         the optimisation loop: one drawn view per step, the Sec. 3.2 loss, a fused
                  Adam step, pruning of parameters and Adam moments at the scheduled steps

The step enqueues only calls of the C ABI plus zero fills of the accumulating outputs; it
allocates nothing and never synchronises with the host, so it can be captured and replayed.
"""
from __future__ import annotations

import ctypes
import json
import os
import time
from dataclasses import asdict, dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from .splat import SSIM_LAMBDA, Gaussians, Renderer, ViewBatch, l1_loss_grad, ssim_loss_grad, ssim_workspace_bytes


@dataclass(frozen=True)
class StepConfig:
    tile_w: int = 16
    tile_h: int = 16
    batch_depth: int = 1
    lpt: bool = False
    pixels_per_lane: int = 0  # 0: the library's default for the tile size

    @property
    def tile(self):
        return (self.tile_w, self.tile_h)


CANDIDATES = ([StepConfig(tw, th, 1, lpt) for (tw, th) in [(16, 16), (16, 8), (8, 8), (32, 8), (32, 16), (16, 32)]
               for lpt in (False, True)]
              + [StepConfig(tw, th, 2, True) for (tw, th) in [(16, 16), (32, 16), (16, 32)]]
              + [StepConfig(tw, th, 1, True, ppl) for (tw, th) in [(16, 16), (32, 16), (16, 32)] for ppl in (1, 2, 4)]
              + [StepConfig(32, 32, 1, False)])


def zero_grads(g: Gaussians) -> Gaussians:
    return Gaussians(torch.zeros_like(g.mean), torch.zeros_like(g.scale), torch.zeros_like(g.quat),
                     torch.zeros_like(g.opacity), torch.zeros_like(g.sh), g.sh_degree)


LOSSES = ("l1", "l2_dssim")


class FwdBwdStep:
    """Forward, loss against per-view targets, and backward for a batch of views."""

    def __init__(self, g: Gaussians, cams: Sequence, targets: Sequence, params=None, cfg: StepConfig = StepConfig(),
                 capacity: Optional[int] = None, device=None, loss: str = "l1"):
        if loss not in LOSSES:
            raise ValueError(f"loss must be one of {LOSSES}")
        dev = torch.device(device if device is not None else "cuda")
        self.cfg = cfg
        self.loss_kind = loss
        self.views = ViewBatch(cams, cfg.tile, dev, cfg.batch_depth, cfg.lpt, cfg.pixels_per_lane)
        self.r = Renderer(g, self.views, params, capacity)
        self.target = self.views.pack_images(targets)
        self.grad = zero_grads(g)
        self.dl = torch.empty_like(self.target)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self._npx3 = self.target.numel()
        self._planes = []
        self.ws = None
        if loss == "l2_dssim":
            need = 1
            for v, (w, h) in enumerate(self.views.sizes):
                o = 3 * int(self.views.pixel_offset_host[v])
                self._planes.append((o, o + 3 * w * h, (3, h, w)))
                need = max(need, ssim_workspace_bytes(3, h, w))
            self.ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def enqueue(self):
        """Enqueue one step on the current stream (no allocation, no host synchronisation). The
        reverse call writes every gradient, so the gradient buffers are not cleared."""
        self.loss.zero_()
        rgb = self.r.forward()
        if self.loss_kind == "l1":
            l1_loss_grad(rgb[:self._npx3], self.target, self.dl, self.loss)
        else:
            for a, b, shape in self._planes:
                ssim_loss_grad(rgb[a:b].view(shape), self.target[a:b].view(shape), self.dl[a:b].view(shape),
                               self.loss, SSIM_LAMBDA, self._npx3, self.ws)
        self.r.backward(self.dl, self.grad, overwrite=True)

    def capture(self, warmup: int = 2):
        s = torch.cuda.Stream(device=self.views.device)
        s.wait_stream(torch.cuda.current_stream(self.views.device))
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.enqueue()
        torch.cuda.current_stream(self.views.device).wait_stream(s)
        torch.cuda.synchronize(self.views.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.enqueue()
        torch.cuda.synchronize(self.views.device)
        return self

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.enqueue()

    def ok(self) -> bool:
        """True when no step since construction overflowed the pair buffer (synchronises)."""
        return not self.r.check()[0]


def _cache_path():
    return os.environ.get("GS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gs_autotune.json"))


def _key(g: Gaussians, cams: Sequence, device) -> str:
    name = torch.cuda.get_device_name(device)
    sizes = sorted((int(c.width), int(c.height)) for c in cams)
    return f"{name}|n2^{int(np.log2(max(g.n, 1)))}|{sizes}"


def time_step(step: FwdBwdStep, reps: int = 5) -> float:
    """Mean milliseconds per replayed (or eager) step."""
    step.run()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        step.run()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def autotune(g: Gaussians, cams: Sequence, targets: Sequence, params=None, candidates: Sequence = CANDIDATES,
             reps: int = 5, use_cache: bool = True, graph: bool = True, device=None, log=None) -> StepConfig:
    """Fastest StepConfig for this scene and view set (fwd + loss + bwd per replay)."""
    dev = torch.device(device if device is not None else "cuda")
    key = _key(g, cams, dev)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return StepConfig(**cache[key]["config"])
    best, best_ms, table = None, float("inf"), []
    for cfg in candidates:
        step = FwdBwdStep(g, cams, targets, params, cfg, device=dev)
        if graph:
            step.capture()
        ms = time_step(step, reps)
        if not step.ok():
            continue
        table.append({"config": asdict(cfg), "ms": ms})
        if log:
            log(f"  autotune {cfg}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = cfg, ms
        del step
    if use_cache:
        cache[key] = {"config": asdict(best), "ms": best_ms, "table": table, "time": time.time()}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return best


# ---------------------------------------------------------------------------------------------
# Optimisation with pruning (Sec. 3.2, Sec. 3.3)
# ---------------------------------------------------------------------------------------------

@dataclass
class TrainConfig:
    """Schedule and optimiser settings. The paper gives the loss (lambda = 0.2), the pruning
    rule and when it is applied (twice during optimisation; t_prune 0.01 for the default model,
    0.25 for the light one); the optimiser and its learning rates are those of 3D Gaussian
    splatting: Adam, positions at 1.6e-4 x the camera extent decaying exponentially to 1.6e-6 x
    over the run, SH DC 2.5e-3, higher SH bands 2.5e-3 / 20 enabled one band every 1000 steps,
    opacity 0.05 in logit space, scales 5e-3 in log space, rotations 1e-3."""
    steps: int = 30000
    prune_steps: Tuple[int, ...] = (16000, 24000)
    t_prune: float = 0.01
    lam: float = 0.2
    lr_mean: float = 1.6e-4
    lr_mean_final: float = 1.6e-6
    lr_sh_dc: float = 2.5e-3
    lr_sh_rest: float = 2.5e-3 / 20
    lr_opacity: float = 0.05
    lr_scale: float = 5e-3
    lr_quat: float = 1e-3
    sh_band_every: int = 1000
    betas: Tuple[float, float] = (0.9, 0.999)
    eps: float = 1e-15
    seed: int = 0
    headroom: float = 2.0
    check_every: int = 1000
    lpt: bool = True  # the traversals take the step view's tiles longest list first

    @classmethod
    def light(cls, **kw) -> "TrainConfig":
        """The lightweight variant: t_prune = 0.25 (the default model uses 0.01)."""
        return cls(t_prune=0.25, **kw)


def camera_extent(cams: Sequence) -> float:
    """1.1 x the largest distance of a camera centre from the centroid of the centres."""
    pos = np.stack([np.asarray(c.position, np.float64) for c in cams])
    return float(1.1 * np.max(np.linalg.norm(pos - pos.mean(0), axis=1))) or 1.0


class Trainer:
    """Optimises Gaussians against per-view targets (the radiance field's renders in the
    paper) with the Sec. 3.2 loss, one uniformly drawn training view per step, a fused Adam
    step on the device, and pruning at cfg.prune_steps: the importance of every Gaussian over
    all training views (eq. importance-score), then the Gaussians with h < t_prune removed
    from the parameters and from both Adam moments by one compaction (Sec. 3.3).

    All training views share one resolution. Nothing is allocated per step; a step does not
    synchronise with the host (pruning does, to size the new arrays). The pair capacity is
    sized from the most demanding training view times cfg.headroom; a step that overflows it
    renders nothing and takes an Adam step without Gaussian gradients, so the overflow flag
    (sticky over steps) is read before every pruning and every cfg.check_every steps, and an
    overflow raises."""

    def __init__(self, g: Gaussians, cams: Sequence, targets: Sequence, params=None,
                 cfg: TrainConfig = TrainConfig(), tile=None, device=None):
        from .splat import DEFAULT_TILE, camera_struct
        from . import _lib as L
        dev = torch.device(device if device is not None else "cuda")
        if any((c.width, c.height) != (cams[0].width, cams[0].height) for c in cams):
            raise ValueError("every training view must have the same resolution")
        self.cfg, self.params, self.device = cfg, params, dev
        self.cams = list(cams)
        self.tile = DEFAULT_TILE if tile is None else tile
        self.extent = camera_extent(self.cams)
        arr = (L.gs_camera * len(cams))(*[camera_struct(c) for c in cams])
        self.cams_all = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(dev)
        self._cam_bytes = ctypes.sizeof(L.gs_camera)
        w, h = cams[0].width, cams[0].height
        self.targets = torch.stack([torch.as_tensor(np.asarray(t, np.float32).reshape(3, h, w)) for t in targets]).to(dev)
        self.dl = torch.empty((3, h, w), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.ws_loss = torch.empty(max(ssim_workspace_bytes(3, h, w), 1), dtype=torch.uint8, device=dev)
        self.rng = np.random.default_rng(cfg.seed)
        self.it = 0
        self.history: List[dict] = []
        self._set_gaussians(g, zero_grads(g), zero_grads(g))

    def _set_gaussians(self, g: Gaussians, m: Gaussians, v: Gaussians):
        self.g, self.m, self.v = g, m, v
        self.grad = zero_grads(g)
        self.view = ViewBatch([self.cams[0]], self.tile, self.device, lpt=self.cfg.lpt)
        self.r = Renderer(g, self.view, self.params, capacity=self._capacity(g))

    def _capacity(self, g: Gaussians) -> int:
        """Pairs of the most demanding training view times the headroom."""
        from .splat import bin_sort, preprocess
        most = 0
        for cam in self.cams:
            one = ViewBatch([cam], self.tile, self.device)
            most = max(most, int(bin_sort(preprocess(g, one, self.params), one).n_pairs.item()))
        return int(most * self.cfg.headroom) + 4096

    def lr_mean(self) -> float:
        c = self.cfg
        t = min(self.it / max(c.steps, 1), 1.0)
        return self.extent * float(np.exp((1 - t) * np.log(c.lr_mean) + t * np.log(c.lr_mean_final)))

    def groups(self):
        c, g, gr, m, v = self.cfg, self.g, self.grad, self.m, self.v
        out = [(g.mean, gr.mean, m.mean, v.mean, self.lr_mean(), "linear"),
               (g.scale, gr.scale, m.scale, v.scale, c.lr_scale, "log"),
               (g.quat, gr.quat, m.quat, v.quat, c.lr_quat, "linear"),
               (g.opacity, gr.opacity, m.opacity, v.opacity, c.lr_opacity, "logit"),
               (g.sh[0:3], gr.sh[0:3], m.sh[0:3], v.sh[0:3], c.lr_sh_dc, "linear")]
        for band in range(1, g.sh_degree + 1):
            rows = slice(3 * band * band, 3 * (band + 1) * (band + 1))
            lr = c.lr_sh_rest if self.it >= band * c.sh_band_every else 0.0
            out.append((g.sh[rows], gr.sh[rows], m.sh[rows], v.sh[rows], lr, "linear"))
        return out

    def step(self):
        """One optimisation step on a uniformly drawn training view; pruning when due."""
        from .splat import adam_step
        i = int(self.rng.integers(len(self.cams)))
        self.r._sv.cams = ctypes.c_void_p(self.cams_all.data_ptr() + self._cam_bytes * i)
        rgb = self.r.forward()
        self.loss.zero_()
        shape = self.dl.shape
        ssim_loss_grad(rgb[:self.dl.numel()].view(shape), self.targets[i], self.dl, self.loss, self.cfg.lam, None,
                       self.ws_loss)
        self.r.backward(self.dl.view(-1), self.grad, overwrite=True)
        self.it += 1
        adam_step(self.groups(), self.it, self.cfg.betas, self.cfg.eps, zero_grad=False)
        if self.it in self.cfg.prune_steps:
            self.prune()
        elif self.cfg.check_every > 0 and self.it % self.cfg.check_every == 0:
            self.check_capacity()
        return i

    def check_capacity(self):
        """Raise if some step since the last check overflowed the pair capacity (synchronises)."""
        if not self.ok():
            raise RuntimeError(f"a training step before step {self.it} overflowed the pair capacity "
                               f"({self.r.bins.capacity} pairs); use a larger TrainConfig.headroom")

    def importance(self) -> torch.Tensor:
        from .splat import importance
        h = torch.zeros(max(self.g.n, 1), dtype=torch.float32, device=self.device)
        for c0 in range(0, len(self.cams), 8):
            importance(self.g, ViewBatch(self.cams[c0:c0 + 8], self.tile, self.device), self.params, h=h)
        return h

    def prune(self, t_prune: Optional[float] = None):
        """Remove the Gaussians with h < t_prune from the parameters and the Adam moments."""
        from .splat import prune_gaussians
        t = self.cfg.t_prune if t_prune is None else t_prune
        self.check_capacity()
        h = self.importance()
        m, v = self.m, self.v
        before = self.g.n
        pg, kept, rest = prune_gaussians(self.g, h, t, [m.mean, m.scale, m.quat, m.opacity, m.sh,
                                                         v.mean, v.scale, v.quat, v.opacity, v.sh])
        deg = self.g.sh_degree
        pm = Gaussians(rest[0], rest[1], rest[2], rest[3], rest[4], deg)
        pv = Gaussians(rest[5], rest[6], rest[7], rest[8], rest[9], deg)
        self._set_gaussians(pg, pm, pv)
        self.history.append({"step": self.it, "t_prune": t, "before": before, "after": pg.n})
        return kept

    def ok(self) -> bool:
        """True when no step on the current Gaussians overflowed the pair capacity (synchronises)."""
        return not self.r.check()[0]
