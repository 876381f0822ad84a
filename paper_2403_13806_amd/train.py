"""Batched training step (forward + loss + backward over many views of uneven size) as
one captured hipGraph, and the autotuner that picks its launch configuration. The loss is
L1 (loss="l1") or the Sec. 3.2 training loss 0.8 L2 + 0.2 D-SSIM (loss="l2_dssim", one
gs_ssim_loss_grad call per view with the batch's element count, sharing one workspace).

  StepConfig      tile size, batch depth (records staged per lane) and persistent launch
  FwdBwdStep      preallocated buffers, an eager step, capture into a hipGraph, replay
  autotune        times every candidate configuration on the actual scene and views and
                  keeps the fastest; results are cached as JSON keyed by device, scene size
                  and the set of view resolutions

The step enqueues only calls of the C ABI plus zero fills of the accumulating outputs; it
allocates nothing and never synchronises with the host, so it can be captured and replayed.
"""
from __future__ import annotations

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
    persistent: bool = False

    @property
    def tile(self):
        return (self.tile_w, self.tile_h)


CANDIDATES = ([StepConfig(tw, th, d, p) for (tw, th) in [(16, 16), (16, 8), (8, 8), (32, 8), (32, 16)]
               for d in (1, 2) for p in (False, True)] + [StepConfig(32, 32, 1, False)])


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
        self.views = ViewBatch(cams, cfg.tile, dev, cfg.batch_depth, cfg.persistent)
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
        """Enqueue one step on the current stream (no allocation, no host synchronisation)."""
        for t in (self.grad.mean, self.grad.scale, self.grad.quat, self.grad.opacity, self.grad.sh, self.loss):
            t.zero_()
        rgb = self.r.forward()
        if self.loss_kind == "l1":
            l1_loss_grad(rgb[:self._npx3], self.target, self.dl, self.loss)
        else:
            for a, b, shape in self._planes:
                ssim_loss_grad(rgb[a:b].view(shape), self.target[a:b].view(shape), self.dl[a:b].view(shape),
                               self.loss, SSIM_LAMBDA, self._npx3, self.ws)
        self.r.backward(self.dl, self.grad)

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
        """True when no frame since construction overflowed the pair buffer (synchronises)."""
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
