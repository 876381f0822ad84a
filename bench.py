"""Benchmark of the splatting hot path on one MI355X.

Headline: forward frames/s of the plain path (preprocess -> bin/sort -> composite) on a
1M-Gaussian SH-3 scene (mixture of 32 anisotropic clusters, random storage order) at
1256x828, cycling over 8 orbit views. Also reported: per-stage kernel times and their
algorithmic rates, fwd+bwd views/s (200k Gaussians, one 1256x828 view; and 1M Gaussians,
8 views of uneven size, batched vs one view at a time), importance views/s, the FP64
oracle timed on the host cores on a bounded sample, and the roofline of the dominant
kernel (compositing), measured with HIP events on the stream the kernels run on.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s fwd (1M Gaussians, 1256x828) + fwd+bwd views/s vs plain; % HBM roofline"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 VALU lane-operations/s (FP32 or
# FP64, one FMA = one lane-op; the 157.3 TFLOP/s FP32 figure counts FMA = 2 and packed = 2)
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
# algorithmic lane-ops of one composited (pixel, Gaussian) evaluation: FP64 support test
# (2 sub, 3 mul, 2 fma, 1 cmp = 8) + opacity and blend in FP32 (cvt, scale, exp = 4 slots,
# mul, min, weight, 3 fma colour, 1 - alpha, transmittance, stop test = 15)
OPS_PER_COMPOSITE = 23
# importance / visibility: support test 8, opacity 8, weight 1, transmittance and stop 3 = 20;
# reverse: support test 8, opacity 8, transmittance recovery 5, weight and colour sums 7,
# dL/dalpha 9, the nine 2D-gradient terms 10 = 47 (per composited evaluation)
OPS_PER_IMPORTANCE = 20
OPS_PER_BACKWARD = 47
TILE = (16, 32)  # tile of the headline frames (fastest measured: fewer pairs to sort than 16x16)
LPT = True  # longest list first: the compositing tiles' order (its queue is built inside the binning)
PX = 2 if TILE[0] >= 16 and TILE[0] * TILE[1] >= 512 else 1  # pixels per lane the library picks for it
RENDER_KERNEL = f"k_render<{TILE[0]},{TILE[1]},1,0,{PX}>"
SPLAT = 64


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--only", choices=["batched", "importance", "house", "training", "kmeans"], default=None,
                    help="run one secondary workload alone (for profiling) and print its numbers")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every gs_* call is enqueued on)."""

    def __init__(self, torch):
        self.t = torch
        self.s = torch.cuda.Event(enable_timing=True)
        self.e = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.s.record()
        return self

    def __exit__(self, *a):
        self.e.record()

    def ms(self):
        self.e.synchronize()
        return self.s.elapsed_time(self.e)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path shards over views "
              "with one all-reduce per pass and is not run across GPUs here", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2403_13806_amd as gs
    import scenes

    dev = torch.device("cuda:0")
    P = scenes.Params()
    K, W = args.steps, args.warmup
    if args.only:
        if args.only == "batched":
            sc = scenes.mixture_scene(1_000_000, seed=0, sh_degree=3)
            g = gs.Gaussians.from_scene(sc, dev)
            res = fwd_bwd_and_batched(torch, gs, scenes, P, dev, g, sc, K, W, tune=False)
        elif args.only == "importance":
            res = importance_pass(torch, gs, scenes, P, dev)
        elif args.only == "training":
            sc = scenes.mixture_scene(1_000_000, seed=0, sh_degree=3)
            g = gs.Gaussians.from_scene(sc, dev)
            res = trainer_pass(torch, gs, scenes, P, dev, g, scenes.orbit_views(8), steps=K)
        elif args.only == "kmeans":
            res = kmeans_pass(torch, gs, scenes, dev)
        else:
            res = filtered_pass(torch, gs, scenes, P, dev)
        print(json.dumps({"only": args.only, **res}), flush=True)
        return

    copy_gbps = calib_copy(torch, dev)
    log(f"device copy of 256 MiB: {copy_gbps:.0f} GB/s (read + write)")
    log("scene: 1M Gaussians, mixture-32, SH degree 3")
    sc = scenes.mixture_scene(1_000_000, seed=0, sh_degree=3)
    cams = scenes.orbit_views(8)
    g = gs.Gaussians.from_scene(sc, dev)
    # forward-only frames: the pairs' emission slots (the backward's input) are not kept
    rs = [gs.Renderer(g, gs.ViewBatch([c], TILE, dev, lpt=LPT), P, backward=False) for c in cams]
    torch.cuda.synchronize()

    # ---------------- headline: plain forward frames/s ----------------
    for i in range(W):
        rs[i % 8].forward()
    torch.cuda.synchronize()
    log(f"timing {K} forward frames")
    t0 = time.perf_counter()
    with Timer(torch) as tm:
        for i in range(K):
            rs[i % 8].forward()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = tm.ms()
    for r in rs:
        ovf, _ = r.check()
        assert not ovf, "pair capacity overflowed during the timed frames"
    fps = K / wall
    log(f"forward: {fps:.1f} frames/s (wall), {K / ev_ms * 1e3:.1f} frames/s (events)")

    # ---------------- per-stage kernel times (events around each call) ----------------
    # (the stages are timed as separate calls: binning with its own tile sort, then compositing
    # alone; the headline frames above sort each tile inside the compositing launch instead)
    import ctypes
    from paper_2403_13806_amd import _lib as L
    from paper_2403_13806_amd.splat import _ptr, _stream
    lib = L.load()
    stages = {"preprocess": [], "bin_sort": [], "render_fwd": [], "importance": [], "visibility": [], "backward": []}
    pairs, composites, tested, visible = [], [], [], []
    ncontrib = torch.empty(rs[0].views.n_pixels, dtype=torch.int32, device=dev)
    h_buf = torch.zeros(g.n, dtype=torch.float32, device=dev)
    bits_buf = torch.zeros((g.n + 31) // 32, dtype=torch.int32, device=dev)
    one_cluster = torch.zeros(1, dtype=torch.int32, device=dev)
    from paper_2403_13806_amd.train import zero_grads
    gbuf = zero_grads(g)
    # the reverse call as a training step makes it: every gradient written (no clearing before it)
    gg = L.gs_gaussians_grad(_ptr(gbuf.mean), _ptr(gbuf.scale), _ptr(gbuf.quat), _ptr(gbuf.opacity), _ptr(gbuf.sh),
                             g.n, g.sh_degree, 1)
    dl_buf = torch.full((3 * rs[0].views.n_pixels,), 1e-6, dtype=torch.float32, device=dev)
    reps = max(3, K // 8)
    for r, cam0 in zip(rs, cams):
        s = _stream(dev)
        # the reverse call runs on a renderer that keeps the emission slots, after its forward
        rb = gs.Renderer(g, gs.ViewBatch([cam0], TILE, dev, lpt=LPT), P, capacity=r.bins.capacity)
        rb.forward()
        for _ in range(reps):
            with Timer(torch) as a:
                L.check(lib.gs_preprocess(ctypes.byref(r._sg), ctypes.byref(r._sv), ctypes.byref(r.p), None, r.g.n, 1,
                                          ctypes.byref(r._sp), s))
            with Timer(torch) as b:
                L.check(lib.gs_bin_sort(ctypes.byref(r._sp), ctypes.byref(r._sv), ctypes.byref(r._sb), _ptr(r.ws),
                                        r.ws.numel(), s))
            with Timer(torch) as c:  # the plain compositing kernel (the roofline's)
                r.render_only(s)
            # the traversals built on the same lists: importance, cluster visibility, reverse
            with Timer(torch) as d:
                L.check(lib.gs_importance(ctypes.byref(r._sp), ctypes.byref(r._sv), ctypes.byref(r._sb),
                                          ctypes.byref(r.p), _ptr(h_buf), s))
            with Timer(torch) as e:
                L.check(lib.gs_cluster_visibility(ctypes.byref(r._sp), ctypes.byref(r._sv), ctypes.byref(r._sb),
                                                  ctypes.byref(r.p), _ptr(one_cluster), 1, 0.01, _ptr(bits_buf), s))
            with Timer(torch) as f:
                L.check(lib.gs_render_bwd(ctypes.byref(rb._sg), ctypes.byref(rb._sv), ctypes.byref(rb._sp),
                                          ctypes.byref(rb._sb), ctypes.byref(rb.p), _ptr(rb.t_final), _ptr(rb.n_last),
                                          _ptr(dl_buf), ctypes.byref(gg), _ptr(rb.ws), rb.ws.numel(), s))
            stages["preprocess"].append(a.ms())
            stages["bin_sort"].append(b.ms())
            stages["render_fwd"].append(c.ms())
            stages["importance"].append(d.ms())
            stages["visibility"].append(e.ms())
            stages["backward"].append(f.ms())
        # work counts of this view (the counting instance of the compositing kernel, untimed)
        r.render_only(s, ncontrib)
        npairs = int(r.bins.n_pairs.item())
        pairs.append(npairs)
        composites.append(int(ncontrib.sum().item()))
        visible.append(int((r.proj.count > 0).sum().item()))
        cam = r.views.cams[0]
        tx = (cam.width + TILE[0] - 1) // TILE[0]
        py, px = torch.meshgrid(torch.arange(cam.height, device=dev), torch.arange(cam.width, device=dev),
                                indexing="ij")
        tile = ((py // TILE[1]) * tx + px // TILE[0]).reshape(-1)
        rg = r.bins.ranges.view(-1, 2).long()
        st, en = rg[tile, 0], rg[tile, 1]
        stopped = r.t_final < P.t_min
        tested.append(int(torch.where(stopped, r.n_last.long() - st, en - st).sum().item()))
    avg = {k: float(np.mean(v)) for k, v in stages.items()}
    npx = rs[0].views.n_pixels
    n = g.n
    mp, mc, mt, mv = (float(np.mean(x)) for x in (pairs, composites, tested, visible))
    n_tiles = rs[0].views.n_tiles
    buckets = n_tiles <= 8192  # pairs emitted straight into per-view tile buckets, else onesweep radix passes
    passes = 1 if buckets else max(1, (int(np.ceil(np.log2(n_tiles))) + 7) // 8)
    bytes_pre = 4 * n * (3 + 3 + 4 + 1 + 48) + 4 * n + mv * (SPLAT + 4 + 8)
    # buckets: two walks over the entries (count per entry, rectangle per visible entry, and in
    # the second the depth too), one row of tile counts per 4096 entries (written, scanned in
    # place, read by the emission: 4 passes of 4 B per tile), 8 B per pair into its tile's range.
    # Entry order: block sums (count in), emission (count per entry, rect + depth per visible
    # entry, 12 B per pair out), digit histogram (4 B per pair), passes (12 B in + 12 B out per
    # pair each), ranges (4 B per pair). Then the per-tile sort (8 B in, 12 B out per pair) and
    # the ranges
    if buckets:
        stride = (n_tiles + 15) // 16 * 16
        bytes_sort = 8 * n + 24 * mv + 16 * stride * np.ceil(n / 4096) + mp * (8 + 20) + n_tiles * 12
    else:
        bytes_sort = (4 + 8) * n + 12 * mv + mp * (12 + 20) + mp * (4 + passes * 24 + 4) + n_tiles * 8
    bytes_render = mp * (4 + SPLAT) + npx * (12 + 4 + 4) + rs[0].views.n_tiles * 8
    ops_render = OPS_PER_COMPOSITE * mc
    ops_imp, ops_bwd = OPS_PER_IMPORTANCE * mc, OPS_PER_BACKWARD * mc
    stage_rows = {
        "preprocess": {"ms": avg["preprocess"], "alg_GBps": bytes_pre / avg["preprocess"] / 1e6,
                       "hbm_frac": bytes_pre / avg["preprocess"] / 1e-3 / PEAK_HBM},
        "bin_sort": {"ms": avg["bin_sort"], "alg_GBps": bytes_sort / avg["bin_sort"] / 1e6,
                     "hbm_frac": bytes_sort / avg["bin_sort"] / 1e-3 / PEAK_HBM,
                     "grouping": "tile buckets (per-view LDS histograms, no grouping pass)" if buckets
                     else f"{passes} onesweep radix passes"},
        "render_fwd": {"ms": avg["render_fwd"], "alg_Tops": ops_render / avg["render_fwd"] / 1e9,
                       "alu_frac": ops_render / avg["render_fwd"] / 1e-3 / PEAK_LANE_OPS,
                       "alg_GBps": bytes_render / avg["render_fwd"] / 1e6,
                       "hbm_frac": bytes_render / avg["render_fwd"] / 1e-3 / PEAK_HBM},
        # same composited evaluations as the forward (the stop rule is the same)
        "importance": {"ms": avg["importance"], "alg_Tops": ops_imp / avg["importance"] / 1e9,
                       "alu_frac": ops_imp / avg["importance"] / 1e-3 / PEAK_LANE_OPS},
        "visibility": {"ms": avg["visibility"], "alg_Tops": ops_imp / avg["visibility"] / 1e9,
                       "alu_frac": ops_imp / avg["visibility"] / 1e-3 / PEAK_LANE_OPS},
        # the whole reverse call: 2D-gradient traversal plus the parameter chains
        "backward": {"ms": avg["backward"], "alg_Tops": ops_bwd / avg["backward"] / 1e9,
                     "alu_frac": ops_bwd / avg["backward"] / 1e-3 / PEAK_LANE_OPS},
    }
    work = {"visible_per_view": mv, "pairs_per_view": mp, "composited_per_view": mc,
            "tested_per_view": mt, "composited_per_pixel": mc / npx, "tested_per_composited": mt / max(mc, 1)}
    log(f"stages (ms): {json.dumps({k: round(v, 4) for k, v in avg.items()})}; work {json.dumps(work)}")
    roofline = {"bound": "alu", "kernel": RENDER_KERNEL, "achieved": ops_render / avg["render_fwd"] / 1e9,
                "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-ops/s",
                "frac": ops_render / avg["render_fwd"] / 1e-3 / PEAK_LANE_OPS, "traffic": recorded_traffic(RENDER_KERNEL),
                "traffic_unit": "bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated)",
                "alg_bytes_per_launch": bytes_render,
                "hbm_frac": bytes_render / avg["render_fwd"] / 1e-3 / PEAK_HBM,
                "per_unit": f"{OPS_PER_COMPOSITE} lane-ops per composited (pixel, Gaussian)",
                "units_per_launch": mc, "avg_launch_ms": avg["render_fwd"]}

    # the same frames with two buffer sets on two streams (PathRenderer(pipeline=2)): the
    # projection and binning of one frame overlap the compositing of the previous one. Not in
    # the quick run, whose kernel trace must time single-stream launches only
    pipelined_fps = None
    if not args.quick:
        pipelined_fps = pipelined_frames(torch, gs, P, dev, g, cams, K, W)

    extra = {"stages": stage_rows, "work": work, "events_frames_per_s": K / ev_ms * 1e3,
             "pipelined_2_streams_frames_per_s": pipelined_fps,
             "copy_256MiB_GBps": copy_gbps}
    extra["prune"] = prune_pass(torch, gs, g, h_buf, dev)
    extra["loss_l2_dssim"] = loss_pass(torch, gs, scenes, dev)
    extra["init_1M_points"] = init_pass(torch, gs, scenes, dev)

    if not args.quick:
        extra.update(fwd_bwd_and_batched(torch, gs, scenes, P, dev, g, sc, K, W))
        extra["importance"] = importance_rate(torch, gs, rs, n, dev, K)
        del rs
        extra["importance_150_views"] = importance_pass(torch, gs, scenes, P, dev)
        extra["house_filtering"] = filtered_pass(torch, gs, scenes, P, dev)
        extra["training_loop"] = trainer_pass(torch, gs, scenes, P, dev, g, cams)
        extra["kmeans_131072_cameras"] = kmeans_pass(torch, gs, scenes, dev)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc, cams[0], P)

    line = {
        "metric": METRIC, "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "1M Gaussians (mixture of 32 clusters, SH degree 3), 1256x828, 8 orbit views, "
                               "plain forward per frame", "gaussians": n, "width": 1256, "height": 828,
                   "views": 8, "tile": f"{TILE[0]}x{TILE[1]}",
                   "tile_order": "longest-first" if LPT else "tile index",
                   "tile_sort": "in the compositing launch (gs_bin_sort_render_fwd)", "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "render_fwd_1M_1256x828_traffic.md")
TRAFFIC_SOURCES = ("paper_2403_13806_amd/csrc/gs_render.hip", "paper_2403_13806_amd/csrc/gs_device.hpp",
                   "include/gs.h")


def recorded_traffic(kernel):
    """HBM bytes per compositing launch from the committed counter record, or None when the
    compositing sources changed since the counters were taken or the record is of another
    kernel instance."""
    import hashlib
    try:
        rec = dict(l.split(": ", 1) for l in open(TRAFFIC_RECORD).read().splitlines() if ": " in l)
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in TRAFFIC_SOURCES)).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != h or rec.get("kernel") != kernel:
        return None
    return float(rec["traffic_bytes_per_launch"])


def prune_pass(torch, gs, g, h, dev, t_prune=0.01, reps=5):
    """Pruning as a training loop would run it: the Gaussian parameters and two optimizer
    moments per parameter (177 FP32 planes at SH-3) compacted by h >= t_prune."""
    import ctypes
    from paper_2403_13806_amd import _lib as L
    from paper_2403_13806_amd.splat import _ptr, _stream, alloc_workspace
    n = g.n
    planes = [g.mean, g.scale, g.quat, g.opacity, g.sh]
    moments = [torch.zeros_like(t) for t in planes for _ in range(2)]
    rows_in = [r for t in planes + moments for r in t.reshape(-1, n)]
    outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in rows_in]
    kept = torch.empty(n, dtype=torch.int32, device=dev)
    n_kept = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = alloc_workspace(n, 1, 0, 0, dev)
    vp = ctypes.c_void_p * len(rows_in)
    pin, pout = vp(*[r.data_ptr() for r in rows_in]), vp(*[o.data_ptr() for o in outs])
    call = lambda: L.check(L.load().gs_prune(_ptr(h), n, t_prune, pin, pout, len(rows_in), _ptr(kept), _ptr(n_kept),
                                             _ptr(ws), ws.numel(), _stream(dev)))
    call()
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(reps):
            call()
    ms = tm.ms() / reps
    nk = int(n_kept.item())
    alg = 4 * n + nk * (4 + 8 * len(rows_in))  # h in; per kept Gaussian its index and each plane in + out
    # as a stream compaction: every plane read whole (a kept fraction this size touches every
    # cache line in random storage order), the kept part written
    stream = 4 * n + 4 * len(rows_in) * (n + nk)
    log(f"prune: {len(rows_in)} planes, kept {nk} of {n}, {ms:.3f} ms, {alg / ms / 1e6:.0f} GB/s kept-only, "
        f"{stream / ms / 1e6:.0f} GB/s as a stream")
    return {"planes": len(rows_in), "gaussians": n, "kept": nk, "t_prune": t_prune, "ms": ms,
            "alg_GBps": alg / ms / 1e6, "hbm_frac": alg / ms / 1e-3 / PEAK_HBM,
            "stream_GBps": stream / ms / 1e6, "stream_hbm_frac": stream / ms / 1e-3 / PEAK_HBM}


def pipelined_frames(torch, gs, P, dev, g, cams, K, W):
    """The headline frames rendered by PathRenderer(pipeline=2)."""
    from paper_2403_13806_amd.splat import PathRenderer
    pipe = PathRenderer(g, cams, P, tile=TILE, device=dev, lpt=LPT, pipeline=2)
    for k in range(W):
        pipe.frame(k % len(cams))
    pipe.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        pipe.frame(k % len(cams))
    pipe.sync()
    torch.cuda.synchronize()
    fps = K / (time.perf_counter() - t0)
    assert pipe.ok()
    log(f"pipelined (2 streams, 2 buffer sets): {fps:.1f} frames/s")
    return fps


def loss_pass(torch, gs, scenes, dev, reps=20):
    """The Sec. 3.2 training loss (1 - 0.2) L2 + 0.2 D-SSIM and its gradient for one
    1256 x 828 view (three planes): two HBM-bound launches, 44 algorithmic bytes per pixel
    and plane (8 read and 12 written by the statistics launch, 20 read and 4 written by the
    gradient launch)."""
    x, y = scenes.image_pair(3, 828, 1256)
    xt, yt = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
    dl = torch.empty_like(xt)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(gs.ssim_workspace_bytes(3, 828, 1256), dtype=torch.uint8, device=dev)
    gs.ssim_loss_grad(xt, yt, dl, loss, ws=ws)
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(reps):
            gs.ssim_loss_grad(xt, yt, dl, loss, ws=ws)
    ms = tm.ms() / reps
    alg = 44 * x.size
    log(f"loss (L2 + D-SSIM): 3 x 828 x 1256, {ms:.4f} ms, {alg / ms / 1e6:.0f} GB/s algorithmic")
    return {"planes": 3, "height": 828, "width": 1256, "ms": ms, "alg_bytes": alg,
            "alg_GBps": alg / ms / 1e6, "hbm_frac": alg / ms / 1e-3 / PEAK_HBM}


def init_pass(torch, gs, scenes, dev, reps=5):
    """Initialisation of the point representation (Sec. 3.2) from 1M points (the means of the
    house scene: mostly on walls and floors, storage order random): exact nearest-neighbour
    scales on the cell grid plus the constant parameters."""
    sc = scenes.house_scene(1_000_000, seed=6, sh_degree=0)
    pts = torch.as_tensor(np.ascontiguousarray(sc.mean), device=dev)
    col = torch.rand((3, pts.shape[1]), device=dev)
    gs.init_gaussians(pts, col, 3)
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(reps):
            g = gs.init_gaussians(pts, col, 3)
    ms = tm.ms() / reps
    log(f"init: 1M house points, {ms:.3f} ms (nearest-neighbour scales + constants)")
    return {"points": int(pts.shape[1]), "ms": ms, "points_per_s": pts.shape[1] / ms * 1e3}


def kmeans_pass(torch, gs, scenes, dev, reps=3):
    """Camera clustering (Sec. 3.4) of a large camera set: 131072 camera centres drawn over the
    12 house rooms, 64 clusters, at most 100 Lloyd iterations on the device from the host
    k-means++ seeding; the host FP64 k-means on the same set timed once beside it."""
    pos = scenes.house_camera_positions(131072)
    t0 = time.perf_counter()
    init = gs.kmeans_seed(pos, 64, seed=3)
    seed_ms = (time.perf_counter() - t0) * 1e3
    pos_d = torch.as_tensor(pos, device=dev)
    init_d = torch.as_tensor(init, device=dev)
    cen = init_d.clone()
    ws = torch.empty(int(gs.load().gs_kmeans_workspace_bytes(131072, 64, 100)), dtype=torch.uint8, device=dev)
    gs.kmeans_lloyd(pos_d, cen, 100, ws)
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(reps):
            cen.copy_(init_d)
            _, iters = gs.kmeans_lloyd(pos_d, cen, 100, ws)
    ms = tm.ms() / reps
    it = int(iters.item())
    t0 = time.perf_counter()
    gs.kmeans(pos, 64, seed=3)
    host_ms = (time.perf_counter() - t0) * 1e3
    log(f"kmeans: 131072 cameras, 64 clusters, {it} iterations: device Lloyd {ms:.3f} ms, host seeding "
        f"{seed_ms:.1f} ms, host k-means {host_ms:.1f} ms")
    return {"cameras": 131072, "clusters": 64, "iterations": it, "device_lloyd_ms": ms, "host_seed_ms": seed_ms,
            "host_kmeans_ms": host_ms}


def trainer_pass(torch, gs, scenes, P, dev, g, cams, steps=20):
    """The optimisation loop on the 1M-Gaussian scene and its eight 1256x828 views: one drawn
    view per step, the Sec. 3.2 loss, the fused Adam step over all parameter groups, and one
    pruning event (importance over the eight views, compaction of parameters and both Adam
    moments). The Adam step moves 32 bytes per element (parameter, gradient and both moments
    read; parameter, moments and the cleared gradient written)."""
    from paper_2403_13806_amd.train import TrainConfig, Trainer
    g0 = gs.Gaussians(g.mean.clone(), g.scale.clone(), g.quat.clone(), g.opacity.clone(), g.sh.clone(), g.sh_degree)
    tg = scenes.target_images(cams)
    cfg = TrainConfig(steps=30000, prune_steps=(), t_prune=0.01)
    tr = Trainer(g0, cams, tg, P, cfg, device=dev)
    for _ in range(3):
        tr.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) / steps * 1e3
    # the Adam step alone: ten calls back to back (one call would also time its host-side setup)
    groups = tr.groups()
    with Timer(torch) as tm:
        for k in range(10):
            gs.adam_step(groups, tr.it + 1 + k, cfg.betas, cfg.eps)
    adam_ms = tm.ms() / 10
    n_elem = sum(t[0].numel() for t in tr.groups())
    t0 = time.perf_counter()
    tr.prune(0.01)
    torch.cuda.synchronize()
    prune_s = time.perf_counter() - t0
    before, after = tr.history[-1]["before"], tr.history[-1]["after"]
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.step()
    torch.cuda.synchronize()
    step_ms_after = (time.perf_counter() - t0) / steps * 1e3
    assert tr.ok()
    log(f"training loop: {step_ms:.3f} ms/step ({1e3 / step_ms:.0f} steps/s) at {before} Gaussians, Adam "
        f"{adam_ms:.3f} ms ({32 * n_elem / adam_ms / 1e6:.0f} GB/s over {n_elem} elements); pruning to {after} "
        f"in {prune_s:.3f} s; then {step_ms_after:.3f} ms/step")
    return {"gaussians": before, "steps_per_s": 1e3 / step_ms, "ms_per_step": step_ms, "adam_ms": adam_ms,
            "adam_GBps": 32 * n_elem / adam_ms / 1e6, "adam_hbm_frac": 32 * n_elem / adam_ms / 1e-3 / PEAK_HBM,
            "prune_event_s": prune_s, "kept": after, "steps_per_s_after_prune": 1e3 / step_ms_after}


def calib_copy(torch, dev, nbytes=256 << 20, reps=5):
    """A plain device-to-device copy of known size: its measured rate is the practical HBM
    ceiling, and its hardware byte counters calibrate the counters of the other kernels."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    with Timer(torch) as tm:
        for _ in range(reps):
            dst.copy_(src)
    return 2 * nbytes * reps / (tm.ms() * 1e-3) / 1e9


def fwd_bwd_and_batched(torch, gs, scenes, P, dev, g1m, sc1m, K, W, tune=True):
    out = {}
    # --- 200k Gaussians, one 1256x828 view, forward + L1 + backward ---
    log("fwd+bwd: 200k Gaussians, 1256x828")
    sc = scenes.mixture_scene(200_000, seed=0, sh_degree=3, log_scale_mu=-4.0)
    cam = scenes.orbit_camera(0.0, np.deg2rad(15.0), 4.0, 1256, 828)
    g = gs.Gaussians.from_scene(sc, dev)
    r = gs.Renderer(g, gs.ViewBatch([cam], (16, 16), dev), P)
    tgt = torch.as_tensor(scenes.target_images([cam])[0].reshape(-1), device=dev)
    grad = gs.Gaussians(torch.zeros_like(g.mean), torch.zeros_like(g.scale), torch.zeros_like(g.quat),
                        torch.zeros_like(g.opacity), torch.zeros_like(g.sh), 3)
    dl = torch.empty_like(tgt)
    loss = torch.zeros(1, device=dev)

    def step():
        rgb = r.forward()
        gs.l1_loss_grad(rgb[:tgt.numel()], tgt, dl, loss)
        r.backward(dl, grad, overwrite=True)

    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    out["fwd_bwd_200k_1view_views_per_s"] = K / (time.perf_counter() - t0)
    log(f"  {out['fwd_bwd_200k_1view_views_per_s']:.1f} views/s")

    # --- 1M Gaussians, 8 uneven views: batched vs one view at a time ---
    from paper_2403_13806_amd.train import FwdBwdStep, StepConfig, autotune, time_step
    log("fwd+bwd: 1M Gaussians, 8 uneven views; plain = 8 sequential per-view steps at 16x16")
    cams = scenes.uneven_views()
    tg = scenes.target_images(cams)
    gradb = gs.Gaussians(torch.zeros_like(g1m.mean), torch.zeros_like(g1m.scale), torch.zeros_like(g1m.quat),
                         torch.zeros_like(g1m.opacity), torch.zeros_like(g1m.sh), 3)
    lb = torch.zeros(1, device=dev)
    singles = []
    for v, c in enumerate(cams):
        rv = gs.Renderer(g1m, gs.ViewBatch([c], (16, 16), dev), P)
        tv = torch.as_tensor(tg[v].reshape(-1), device=dev)
        singles.append((rv, tv, torch.empty_like(tv)))

    def plain():
        # the first view writes the gradients, the others add into them
        for v, (rv, tv, dv) in enumerate(singles):
            rgb = rv.forward()
            gs.l1_loss_grad(rgb[:tv.numel()], tv, dv, lb)
            rv.backward(dv, gradb, overwrite=v == 0)

    kk = max(3, K // 8)
    for _ in range(2):
        plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(kk):
        plain()
    torch.cuda.synchronize()
    out["fwd_bwd_1M_8uneven_plain_views_per_s"] = 8 * kk / (time.perf_counter() - t0)
    log(f"  plain per-view: {out['fwd_bwd_1M_8uneven_plain_views_per_s']:.1f} views/s")
    del singles
    # batched, same default launch, not captured
    eager = FwdBwdStep(g1m, cams, tg, P, StepConfig(16, 16, 1, False), device=dev)
    out["fwd_bwd_1M_8uneven_batched_views_per_s"] = 8 / (time_step(eager, kk) * 1e-3)
    log(f"  batched, 16x16, eager: {out['fwd_bwd_1M_8uneven_batched_views_per_s']:.1f} views/s")
    assert eager.ok()
    del eager
    # batched, autotuned launch configuration, captured in a hipGraph and replayed
    if tune:
        log("  autotuning the batched step")
        cfg = autotune(g1m, cams, tg, P, reps=3, use_cache=False, device=dev, log=log)
    else:
        cfg = StepConfig(16, 16, 1, False)
    step = FwdBwdStep(g1m, cams, tg, P, cfg, device=dev).capture()
    t0 = time.perf_counter()
    for _ in range(kk):
        step.run()
    torch.cuda.synchronize()
    out["fwd_bwd_1M_8uneven_batched_graph_views_per_s"] = 8 * kk / (time.perf_counter() - t0)
    out["fwd_bwd_1M_8uneven_batched_graph_config"] = {"tile": list(cfg.tile), "batch_depth": cfg.batch_depth,
                                                      "lpt": cfg.lpt, "pixels_per_lane": cfg.pixels_per_lane}
    log(f"  batched, {cfg}, hipGraph: {out['fwd_bwd_1M_8uneven_batched_graph_views_per_s']:.1f} views/s")
    assert step.ok()
    del step
    # the same step with the Sec. 3.2 loss (0.8 L2 + 0.2 D-SSIM) in place of L1
    step = FwdBwdStep(g1m, cams, tg, P, cfg, device=dev, loss="l2_dssim").capture()
    t0 = time.perf_counter()
    for _ in range(kk):
        step.run()
    torch.cuda.synchronize()
    out["fwd_bwd_1M_8uneven_batched_graph_l2_dssim_views_per_s"] = 8 * kk / (time.perf_counter() - t0)
    log(f"  batched, {cfg}, hipGraph, L2 + D-SSIM loss: "
        f"{out['fwd_bwd_1M_8uneven_batched_graph_l2_dssim_views_per_s']:.1f} views/s")
    assert step.ok()
    return out


def importance_rate(torch, gs, rs, n, dev, K):
    h = torch.zeros(n, device=dev)
    for r in rs:
        r.importance(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        rs[i % 8].importance(h)
    torch.cuda.synchronize()
    v = K / (time.perf_counter() - t0)
    log(f"importance: {v:.1f} views/s (1M Gaussians, 1256x828)")
    return {"views_per_s_1M_1256x828": v}


def importance_pass(torch, gs, scenes, P, dev, chunk=10):
    """Pruning score over all training rays: 500k Gaussians (mixture, SH-3), 150 orbit views
    at 1256x828 in batches of `chunk` views, longest-first tile order; h = max over all
    pixels of all views of alpha*T, mask h < 0.01."""
    log("importance: 500k Gaussians, 150 views at 1256x828")
    sc = scenes.mixture_scene(500_000, seed=0, sh_degree=3)
    cams = scenes.orbit_views(150)
    g = gs.Gaussians.from_scene(sc, dev)
    rs = [gs.Renderer(g, gs.ViewBatch(cams[i:i + chunk], TILE, dev, lpt=True), P, want_color=False,
                      backward=False)
          for i in range(0, len(cams), chunk)]
    h = torch.zeros(g.n, device=dev)
    for r in rs:
        r.importance(h)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        h.zero_()
        for r in rs:
            r.importance(h)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    assert all(not r.check()[0] for r in rs)
    # kept-vs-threshold curve from the prune-mask kernel (mask = h < t)
    kept = {str(t): int(g.n - gs.prune_mask(h, t).sum().item()) for t in (0.001, 0.005, 0.01, 0.03, 0.1, 0.25)}
    hh = h.cpu().numpy()
    out = {"views_per_s": len(cams) / dt, "ms_all_views": dt * 1e3, "gaussians": g.n,
           "kept_at_t_prune": kept, "pruned_at_0.01": g.n - kept["0.01"], "never_composited": int((hh == 0).sum())}
    log(f"  {out['views_per_s']:.0f} views/s, kept at 0.01: {kept['0.01']} of {g.n}")
    return out


def path_quality(torch, pr, path, ref, lists, cluster_of):
    """Filtered against unfiltered frames over the whole path: PSNR (peak 1) and max |diff| per
    frame; the fraction of frames equal within the image tolerance 1e-4 and at 40 dB or more;
    the worst frames with their cluster."""
    ps, mx = [], []
    for f in range(len(path)):
        d = (ref[f] - pr.frame(f, lists[f])).abs()
        mx.append(float(d.max()))
        ps.append(10 * np.log10(1.0 / max(float((d * d).mean()), 1e-20)))
    assert pr.ok()
    ps, mx = np.array(ps), np.array(mx)
    worst = np.argsort(ps)[:5]
    return {"frames": len(path), "psnr_min": float(ps.min()), "psnr_mean": float(ps.mean()),
            "psnr_median": float(np.median(ps)), "frac_psnr_ge_40": float(np.mean(ps >= 40)),
            "frac_equal_1e-4": float(np.mean(mx <= 1e-4)), "max_abs": float(mx.max()),
            "worst_frames": [[int(f), round(float(ps[f]), 2), int(cluster_of(path[f]))] for f in worst]}


def filtered_pass(torch, gs, scenes, P, dev, n=5_000_000, k=64, t_cluster=0.01, extra=32):
    """Test-time visibility filtering at house scale: 5M Gaussians in 12 rooms, 640 training
    cameras at 1920x1080 clustered into 64 by k-means, per-cluster lists at h > t_cluster, a
    300-frame 1920x1080 path rendered without the lists, with them (gathered by index), and
    from the lists materialised as compact per-cluster copies (bitwise the same frames). Every
    filtered rate comes with the quality of its frames against the unfiltered ones."""
    from paper_2403_13806_amd.splat import PathRenderer
    log(f"house: {n} Gaussians, 640 training views + {extra} random views per cluster, k={k}, "
        f"t_cluster={t_cluster}")
    sc = scenes.house_scene(n)
    train = scenes.house_training_views(640)
    path = scenes.house_test_path(300)
    g = gs.Gaussians.from_scene(sc, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vf = gs.VisibilityFilter(g, train, k=k, t_cluster=t_cluster, params=P, chunk=8, device=dev,
                             extra_per_cluster=extra)
    torch.cuda.synchronize()
    t_vis = time.perf_counter() - t0
    sizes = np.array([int(x.shape[0]) for x in vf.lists])
    frame_lists = [vf.list_for(c) for c in path]
    pr = PathRenderer(g, path, P, device=dev, max_entries=g.n)
    # the lists materialised as compact per-cluster copies (memory for coalesced loads)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vf.materialize()
    torch.cuda.synchronize()
    t_mat = time.perf_counter() - t0
    frame_copies = [vf.copy_for(c) for c in path]

    def rate(lists, copies):
        for f in range(3):
            pr.frame(f, lists[f], copies[f])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(len(path)):
            pr.frame(f, lists[f], copies[f])
        torch.cuda.synchronize()
        return len(path) / (time.perf_counter() - t0)

    none = [None] * len(path)
    rates = {"unfiltered": rate(none, none), "filtered": rate(frame_lists, none),
             "filtered_materialized": rate(none, frame_copies)}
    # the materialised frames pipelined over two streams
    pr2 = PathRenderer(g, path, P, device=dev, max_entries=g.n, pipeline=2, capacity=pr.bins.capacity)
    for f in range(3):
        pr2.frame(f, None, frame_copies[f])
    pr2.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(len(path)):
        pr2.frame(f, None, frame_copies[f])
    pr2.sync()
    torch.cuda.synchronize()
    rates["filtered_materialized_pipelined"] = len(path) / (time.perf_counter() - t0)
    assert pr2.ok()
    del pr2
    # untimed: every unfiltered frame kept on the device (7.5 GB) as the quality reference;
    # the copies render like the lists, bit for bit
    ref = [pr.frame(f, None).clone() for f in range(len(path))]
    assert pr.ok()
    for f in range(0, len(path), 25):
        assert torch.equal(pr.frame(f, frame_lists[f]), pr.frame(f, g=frame_copies[f])) and pr.ok()
    quality = path_quality(torch, pr, path, ref, frame_lists, vf.cluster_of)
    out = {"gaussians": n, "train_views": len(train), "extra_views_per_cluster": extra, "extra_placement": "jitter",
           "k": k, "t_cluster": t_cluster, "visibility_pass_s": t_vis, "views_per_s": vf.views_used / t_vis,
           "list_size_mean": float(sizes.mean()), "list_size_max": int(sizes.max()),
           "unfiltered_fps": rates["unfiltered"], "filtered_fps": rates["filtered"],
           "speedup": rates["filtered"] / rates["unfiltered"],
           "filtered_materialized_fps": rates["filtered_materialized"],
           "filtered_materialized_pipelined_fps": rates["filtered_materialized_pipelined"],
           "speedup_materialized": rates["filtered_materialized"] / rates["unfiltered"],
           "materialize_s": t_mat, "materialized_bytes": vf.copy_bytes(), "quality": quality}
    log(f"  lists mean {sizes.mean():.0f}; unfiltered {rates['unfiltered']:.0f} fps, filtered "
        f"{rates['filtered']:.0f} fps, filtered from materialised copies {rates['filtered_materialized']:.0f} fps "
        f"({rates['filtered_materialized_pipelined']:.0f} pipelined over two streams) "
        f"({vf.copy_bytes() / 1e9:.2f} GB, built in {t_mat:.2f} s); PSNR over {len(path)} frames: min "
        f"{quality['psnr_min']:.1f}, median {quality['psnr_median']:.1f} dB, {100 * quality['frac_psnr_ge_40']:.0f}% "
        f">= 40 dB")
    del vf, frame_copies
    # the paper's own threshold, t_cluster = 0.001 (larger lists, same path), and denser extra
    # cameras drawn in each cluster centre's Voronoi cell (the region whose test views use it)
    for key, kw in (("at_t_cluster_0.001", dict(t_cluster=0.001, extra_per_cluster=extra)),
                    ("cell_128_at_t_cluster_0.01", dict(t_cluster=0.01, extra_per_cluster=128,
                                                        extra_placement="cell"))):
        vf = gs.VisibilityFilter(g, train, k=k, params=P, chunk=8, device=dev, materialize=True, **kw)
        lists = [vf.list_for(c) for c in path]
        copies = [vf.copy_for(c) for c in path]
        res = {**{k_: v for k_, v in kw.items()}, "extra_placement": kw.get("extra_placement", "jitter"),
               "list_size_mean": float(np.mean([int(x.shape[0]) for x in vf.lists])),
               "filtered_fps": rate(lists, none), "filtered_materialized_fps": rate(none, copies)}
        res["speedup"] = res["filtered_fps"] / rates["unfiltered"]
        res["speedup_materialized"] = res["filtered_materialized_fps"] / rates["unfiltered"]
        res["quality"] = path_quality(torch, pr, path, ref, lists, vf.cluster_of)
        out[key] = res
        log(f"  {key}: lists mean {res['list_size_mean']:.0f}; filtered {res['filtered_fps']:.0f} fps, from copies "
            f"{res['filtered_materialized_fps']:.0f} fps; PSNR min {res['quality']['psnr_min']:.1f}, median "
            f"{res['quality']['psnr_median']:.1f} dB, {100 * res['quality']['frac_psnr_ge_40']:.0f}% >= 40 dB")
        del vf, copies
    del ref
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, cam, P, m=8192, runs=3):
    """The FP64 oracle on the host: projection of all Gaussians for one view plus m random
    pixels, timed `runs` times after one warm-up run; the median frame time is extrapolated
    linearly in the pixel count."""
    import oracle
    log(f"cpu baseline: oracle, 1 view projection + {m} pixels, median of {runs} after a warm-up")
    rng = np.random.default_rng(0)
    px = rng.integers(0, cam.width, m).astype(np.int32)
    py = rng.integers(0, cam.height, m).astype(np.int32)
    frames, parts = [], []
    for k in range(runs + 1):
        t0 = time.perf_counter()
        proj = oracle.project(sc, cam, P)
        t1 = time.perf_counter()
        oracle.render(sc, cam, P, pixels=(px, py), proj=proj)
        t2 = time.perf_counter()
        del proj
        if k == 0:
            continue  # warm-up
        frames.append((t1 - t0) + (t2 - t1) * (cam.width * cam.height) / m)
        parts.append((t1 - t0, t2 - t1))
    i = int(np.argsort(frames)[len(frames) // 2])
    frame = frames[i]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = cpu_model()
    log(f"  projection {parts[i][0]:.2f} s, {m} pixels {parts[i][1]:.2f} s -> {1 / frame:.3g} frames/s ({model})")
    return {"value": 1.0 / frame, "unit": "frames/s", "cores": cores, "cpu_model": model, "kind": "oracle",
            "runs": runs, "frame_s_runs": frames,
            "sample": f"1M-Gaussian projection of view 0 ({parts[i][0]:.2f} s) + {m} random pixels "
                      f"({parts[i][1]:.2f} s), median of {runs} runs after a warm-up, frame time extrapolated "
                      f"to {cam.width * cam.height} pixels"}


if __name__ == "__main__":
    main()
