"""MI355X (gfx950) Gaussian-splatting hot path of RadSplat (arXiv 2403.13806).

The computation lives in libgs_hip.so (C ABI in include/gs.h, HIP kernels in csrc/);
this package only marshals PyTorch device buffers into those calls.

Typical use (all tensors on the GPU):

    g = init_gaussians(points, colours)                  # Sec. 3.2 initialisation
    views = ViewBatch(cams)                              # one or more pinhole views
    rgb = render(g, views)["rgb"]                        # preprocess, bin, sort, composite
    tr = train.Trainer(g, cams, targets)                 # loss, Adam, pruning at 16k / 24k
    for _ in range(30000):
        tr.step()
    h = importance(tr.g, ViewBatch(cams))                # eq. importance-score
    vf = VisibilityFilter(tr.g, cams, k=64, materialize=True)   # Sec. 3.4 lists
    frame = vf.render(test_cam)["rgb"]

Renderer and PathRenderer keep their buffers between frames (no allocation per frame);
train.FwdBwdStep captures a batched forward + loss + backward in a hipGraph.
"""
from ._lib import GSError, load  # noqa: F401
from .splat import (Bins, Gaussians, GSRender, Projected, Renderer, ViewBatch, VisibilityFilter,  # noqa: F401
                    adam_step, alloc_workspace,
                    bin_sort, bits_to_list, cluster_visibility, gather, gather_gaussians, importance, kmeans,
                    kmeans_lloyd, kmeans_seed, init_gaussians, l1_loss_grad, make_params, nearest_centre, nn_distance,
                    preprocess, prune, prune_gaussians, prune_mask, render, render_batch, render_bwd, render_filtered,
                    render_fwd,
                    ssim_loss_grad, ssim_workspace_bytes, workspace_bytes)
