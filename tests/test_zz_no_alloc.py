"""gs_bin_sort_noalloc (the workspace-free variant of gs_bin_sort, whose scratch is a static
device array) against gs_bin_sort: bit-exact pairs, ranges, counts and emission slots on two
calls in a row, the second with a smaller input, and the same image rendered from both."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2403_13806_amd as gs
import scenes
from paper_2403_13806_amd import _lib as L
from paper_2403_13806_amd.splat import _ptr, _stream

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
P = scenes.Params()


def _noalloc(proj, views, bins):
    lib = L.load()
    return lib.gs_bin_sort_noalloc(ctypes.byref(proj.struct()), ctypes.byref(views.struct()),
                                   ctypes.byref(bins.struct()), _stream(DEV))


def test_bin_sort_noalloc_matches_bin_sort():
    cases = [(scenes.mixture_scene(300_000, seed=0, sh_degree=3), scenes.orbit_views(2)[1], (16, 32)),
             (scenes.mixture_scene(20_000, seed=4, sh_degree=1), scenes.orbit_camera(1.0, 0.2, 4.0, 320, 240),
              (16, 16))]
    for k, (sc, cam, tile) in enumerate(cases):  # the second call is the smaller one
        print(f"noalloc case {k}: {sc.n} Gaussians, {cam.width}x{cam.height}, tile {tile}", flush=True)
        g = gs.Gaussians.from_scene(sc, DEV)
        views = gs.ViewBatch([cam], tile, DEV)
        proj = gs.preprocess(g, views, P)
        ref = gs.bin_sort(proj, views, backward=True)
        torch.cuda.synchronize()
        n_pairs = int(ref.n_pairs.item())
        assert int(ref.overflow.item()) == 0 and n_pairs > 1000
        bins = gs.Bins(ref.capacity, views.n_tiles, DEV, queue=False, entries=proj.n)
        bins.keys.fill_(-1)
        bins.vals.fill_(-1)
        L.check(_noalloc(proj, views, bins))
        torch.cuda.synchronize()
        assert int(bins.overflow.item()) == 0 and int(bins.n_pairs.item()) == n_pairs
        assert torch.equal(bins.keys[:n_pairs], ref.keys[:n_pairs])
        assert torch.equal(bins.vals[:n_pairs], ref.vals[:n_pairs])
        assert torch.equal(bins.ranges[:2 * views.n_tiles], ref.ranges[:2 * views.n_tiles])
        assert torch.equal(bins.entry_offset, ref.entry_offset)
        a = gs.render_fwd(proj, views, ref, P)
        b = gs.render_fwd(proj, views, bins, P)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def test_bin_sort_noalloc_rejects_frames_beyond_its_scratch():
    sc = scenes.uniform_cube_scene(100, seed=1)
    g = gs.Gaussians.from_scene(sc, DEV)
    views = gs.ViewBatch([scenes.plain_view()], (16, 16), DEV)
    proj = gs.preprocess(g, views, P)
    bins = gs.Bins(4096, views.n_tiles, DEV, queue=False)
    bins.capacity = 1 << 28  # 25 bytes of scratch per pair of capacity: far beyond 64 MiB
    code = _noalloc(proj, views, bins)
    assert code == L.GS_ERR_UNSUPPORTED
    assert b"scratch" in L.load().gs_last_error()
