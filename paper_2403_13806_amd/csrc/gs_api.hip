// C ABI entry points (include/gs.h): argument checking, workspace layout and launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "gs_device.hpp"
#include "gs_tile_sort.hpp"

namespace gs {

static thread_local char g_err[512] = "";

gs_status set_error(gs_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

gs_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return GS_OK;
}

// launchers defined next to their kernels
gs_status launch_preprocess(const gs_gaussians*, const gs_views*, const gs_params*, const int32_t*, int64_t, int,
                            gs_projected*, hipStream_t);
gs_status launch_preprocess_bwd(const gs_gaussians*, const gs_views*, const gs_params*, const gs_projected*,
                                const gs_bins*, const float*, float*, gs_gaussians_grad*, hipStream_t);
gs_status launch_bin_sort(const gs_projected*, const gs_views*, gs_bins*, void*, hipStream_t, TileSortArgs*);
gs_status launch_render_fwd_sorted(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, float*,
                                   float*, uint32_t*, uint32_t*, const TileSortArgs&, hipStream_t);
gs_status launch_importance_sorted(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, float*,
                                   const TileSortArgs&, hipStream_t);
gs_status launch_visibility_sorted(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*,
                                   const int32_t*, int32_t, float, uint32_t*, const TileSortArgs&, hipStream_t);
size_t sort_workspace_bytes(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles);
size_t list_workspace_bytes(int64_t n);
gs_status launch_bits_to_list(const uint32_t*, int64_t, int32_t*, int64_t*, void*, hipStream_t);
size_t prune_workspace_bytes(int64_t n);
gs_status launch_prune_mask(const float*, int64_t, float, uint8_t*, hipStream_t);
gs_status launch_prune(const float*, int64_t, float, const float* const*, float* const*, int32_t, int32_t*, int64_t*,
                       void*, size_t, hipStream_t);
gs_status launch_gather(const int32_t*, int64_t, int64_t, const float* const*, float* const*, int32_t, hipStream_t);
gs_status launch_fill_f32(float*, int64_t, float, hipStream_t);
size_t nn_workspace_bytes(int64_t);
int32_t kmeans_max_centres();
size_t kmeans_workspace_bytes(int64_t, int32_t, int32_t);
gs_status launch_kmeans_lloyd(const double*, int64_t, int32_t, int32_t, double*, int32_t*, int32_t*, void*,
                              hipStream_t);
gs_status launch_adam(const gs_adam_group*, int32_t, double, double, double, int64_t, int32_t, hipStream_t);
gs_status launch_nn_distance(const float*, int64_t, float*, void*, hipStream_t);
gs_status launch_init_gaussians(const float*, const float*, int64_t, int32_t, float*, float*, float*, float*, float*,
                                void*, hipStream_t);
gs_status launch_render_fwd(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, float*, float*,
                            uint32_t*, uint32_t*, hipStream_t);
gs_status launch_l1(const float*, const float*, int64_t, float, float*, float*, hipStream_t);
size_t ssim_workspace_bytes(int32_t, int32_t, int32_t);
gs_status launch_ssim_loss_grad(const float*, const float*, int32_t, int32_t, int32_t, int64_t, float, float*, float*,
                                void*, hipStream_t);
gs_status launch_importance(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, float*,
                            hipStream_t);
gs_status launch_visibility(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, const int32_t*,
                            int32_t, float, uint32_t*, hipStream_t);
gs_status launch_render_bwd(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, const float*,
                            const uint32_t*, const float*, float*, hipStream_t);

// nine FP32 partial gradients per pair slot, then their nine sums per (view, entry)
static size_t bwd_slots_bytes(uint64_t capacity) { return (sizeof(float) * 9 * (size_t)capacity + 255) & ~(size_t)255; }
static size_t bwd_workspace_bytes(uint64_t capacity, int64_t n, int32_t n_views) {
    return bwd_slots_bytes(capacity) + sizeof(float) * 9 * (size_t)n * (size_t)n_views;
}

static bool tile_ok(int tw, int th) {
    auto ok = [](int x) { return x == 8 || x == 16 || x == 32; };
    return ok(tw) && ok(th);
}

static gs_status check_views(const gs_views* v) {
    if (!v) return set_error(GS_ERR_INVALID_ARG, "views is NULL");
    if (v->n_views < 1) return set_error(GS_ERR_INVALID_ARG, "n_views must be >= 1 (got %d)", v->n_views);
    if (v->n_views > 65535) return set_error(GS_ERR_UNSUPPORTED, "at most 65535 views per call (got %d)", v->n_views);
    if (!v->cams || !v->tile_offset || !v->pixel_offset)
        return set_error(GS_ERR_INVALID_ARG, "views has a NULL device table");
    if (!tile_ok(v->tile_w, v->tile_h))
        return set_error(GS_ERR_UNSUPPORTED, "tile %dx%d: each side must be 8, 16 or 32", v->tile_w, v->tile_h);
    if (v->n_tiles < 0 || v->n_pixels < 0) return set_error(GS_ERR_INVALID_ARG, "negative tile or pixel count");
    if (v->batch_depth != 1 && v->batch_depth != 2)
        return set_error(GS_ERR_UNSUPPORTED, "batch_depth must be 1 or 2 (got %d)", v->batch_depth);
    if (v->batch_depth == 2 && v->tile_w * v->tile_h > 512)
        return set_error(GS_ERR_UNSUPPORTED, "batch_depth 2 needs a tile of at most 512 pixels (LDS)");
    if (v->lpt != 0 && v->lpt != 1) return set_error(GS_ERR_INVALID_ARG, "lpt must be 0 or 1 (got %d)", v->lpt);
    const int ppl = v->pixels_per_lane;
    if (ppl != 0 && ppl != 1 && ppl != 2 && ppl != 4)
        return set_error(GS_ERR_UNSUPPORTED, "pixels_per_lane must be 0, 1, 2 or 4 (got %d)", ppl);
    if ((ppl >= 2 && v->tile_w < 16) || (ppl == 4 && v->tile_h < 16))
        return set_error(GS_ERR_UNSUPPORTED, "pixels_per_lane %d needs a tile of at least %dx%d", ppl, 16,
                         ppl == 4 ? 16 : 8);
    if (v->max_view_tiles < 0 || v->max_view_tiles > v->n_tiles)
        return set_error(GS_ERR_INVALID_ARG, "max_view_tiles must be in [0, n_tiles] (got %d)", v->max_view_tiles);
    return GS_OK;
}

static gs_status check_queue(const gs_views* v, const gs_bins* b) {
    if (v->lpt && !b->queue)
        return set_error(GS_ERR_INVALID_ARG, "the longest-first order needs bins->queue (built by gs_bin_sort)");
    return GS_OK;
}

static gs_status check_params(const gs_params* p) {
    if (!p) return set_error(GS_ERR_INVALID_ARG, "params is NULL");
    if (!(p->alpha_min > 0.f) || !(p->alpha_max > 0.f) || !(p->alpha_max < 1.f) || !(p->t_min >= 0.f) ||
        !(p->kappa > 0.f) || !(p->lowpass >= 0.f) || !(p->guard > 0.f))
        return set_error(GS_ERR_INVALID_ARG, "params out of range (need alpha_min > 0, 0 < alpha_max < 1, "
                                             "t_min >= 0, kappa > 0, lowpass >= 0, guard > 0)");
    return GS_OK;
}

static gs_status check_gaussians(const gs_gaussians* g) {
    if (!g) return set_error(GS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0) return set_error(GS_ERR_INVALID_ARG, "negative Gaussian count");
    if (g->n >= (int64_t)1 << 31) return set_error(GS_ERR_UNSUPPORTED, "at most 2^31-1 Gaussians");
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return set_error(GS_ERR_UNSUPPORTED, "sh_degree %d not in 0..3", g->sh_degree);
    if (g->n > 0 && (!g->mean || !g->scale || !g->quat || !g->opacity))
        return set_error(GS_ERR_INVALID_ARG, "Gaussian parameter pointer is NULL");
    return GS_OK;
}

static gs_status check_projected(const gs_projected* p, bool need_splat) {
    if (!p) return set_error(GS_ERR_INVALID_ARG, "projected is NULL");
    if (p->n < 0) return set_error(GS_ERR_INVALID_ARG, "negative entry count");
    if (p->n > 0 && (!p->count || !p->rect || !p->depth || (need_splat && !p->splat)))
        return set_error(GS_ERR_INVALID_ARG, "projected buffer pointer is NULL");
    return GS_OK;
}

static gs_status check_bins(const gs_bins* b) {
    if (!b) return set_error(GS_ERR_INVALID_ARG, "bins is NULL");
    if (!b->ranges || !b->n_pairs || !b->overflow || (b->capacity > 0 && (!b->keys || !b->vals)))
        return set_error(GS_ERR_INVALID_ARG, "bins buffer pointer is NULL");
    if (b->capacity >= ((uint64_t)1 << 32)) return set_error(GS_ERR_UNSUPPORTED, "capacity must be < 2^32");
    return GS_OK;
}

// Scratch of gs_bin_sort_noalloc: one copy per GPU the library runs on, held until the process
// ends. In host code `scratch` names a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, on the first call made with that device current.
static __device__ __align__(256) unsigned char scratch[GS_BIN_SORT_NOALLOC_BYTES];

static gs_status noalloc_scratch(void** out) {
    static std::mutex mu;
    static std::map<int, void*> ptrs;
    int dev = 0;
    const hipError_t e0 = hipGetDevice(&dev);
    if (e0 != hipSuccess) return set_error(GS_ERR_HIP, "gs_bin_sort_noalloc: hipGetDevice: %s", hipGetErrorString(e0));
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptrs.find(dev);
    if (it == ptrs.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return set_error(GS_ERR_HIP, "gs_bin_sort_noalloc: hipGetSymbolAddress of the scratch on device %d: %s",
                             dev, hipGetErrorString(e));
        it = ptrs.emplace(dev, ptr).first;
    }
    *out = it->second;
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

const char* gs_last_error(void) { return g_err; }

gs_status gs_view_layout(const gs_camera* cams, int32_t n_views, int32_t tile_w, int32_t tile_h,
                         int32_t* tile_offset, int64_t* pixel_offset) {
    if (!cams || !tile_offset || !pixel_offset || n_views < 1)
        return set_error(GS_ERR_INVALID_ARG, "gs_view_layout: NULL table or n_views < 1");
    if (!tile_ok(tile_w, tile_h)) return set_error(GS_ERR_UNSUPPORTED, "gs_view_layout: unsupported tile size");
    int64_t tiles = 0, pix = 0;
    for (int v = 0; v < n_views; ++v) {
        const int W = cams[v].width, H = cams[v].height;
        if (W < 1 || H < 1 || W > 65535 * 8 || H > 65535 * 8)
            return set_error(GS_ERR_INVALID_ARG, "view %d: bad size %dx%d", v, W, H);
        tile_offset[v] = (int32_t)tiles;
        pixel_offset[v] = pix;
        tiles += (int64_t)div_up(W, tile_w) * div_up(H, tile_h);
        pix += (int64_t)W * H;
        if (tiles >= ((int64_t)1 << 31)) return set_error(GS_ERR_UNSUPPORTED, "more than 2^31 tiles in a batch");
    }
    tile_offset[n_views] = (int32_t)tiles;
    pixel_offset[n_views] = pix;
    return GS_OK;
}

size_t gs_workspace_bytes(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles) {
    if (n < 0 || n_views < 0) return 0;
    size_t b = sort_workspace_bytes(n, n_views, capacity, n_tiles);
    b = std::max(b, bwd_workspace_bytes(capacity, n, n_views));
    b = std::max(b, list_workspace_bytes(n));
    b = std::max(b, prune_workspace_bytes(n) + list_workspace_bytes(n));
    return b;
}

gs_status gs_preprocess(const gs_gaussians* g, const gs_views* views, const gs_params* p, const int32_t* subset,
                        int64_t n_subset, int32_t want_color, gs_projected* out, void* stream) {
    gs_status st;
    if ((st = check_gaussians(g)) || (st = check_views(views)) || (st = check_params(p)) ||
        (st = check_projected(out, true)))
        return st;
    const int64_t n = subset ? n_subset : g->n;
    if (subset && (n_subset < 0 || n_subset > g->n))
        return set_error(GS_ERR_INVALID_ARG, "n_subset %lld outside [0, %lld]", (long long)n_subset, (long long)g->n);
    if (out->n != n)
        return set_error(GS_ERR_INVALID_ARG, "projected->n = %lld but %lld entries per view are produced",
                         (long long)out->n, (long long)n);
    if (want_color && g->n > 0 && !g->sh) return set_error(GS_ERR_INVALID_ARG, "sh is NULL with want_color");
    return launch_preprocess(g, views, p, subset, n, want_color, out, (hipStream_t)stream);
}

gs_status gs_bin_sort(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* ws, size_t ws_bytes,
                      void* stream) {
    gs_status st;
    if ((st = check_projected(proj, false)) || (st = check_views(views)) || (st = check_bins(bins))) return st;
    const size_t need = sort_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    return launch_bin_sort(proj, views, bins, ws, (hipStream_t)stream, nullptr);
}

gs_status gs_bin_sort_noalloc(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, false)) || (st = check_views(views)) || (st = check_bins(bins))) return st;
    const size_t need = sort_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles);
    if (need > (size_t)GS_BIN_SORT_NOALLOC_BYTES)
        return set_error(GS_ERR_UNSUPPORTED,
                         "gs_bin_sort_noalloc: this call needs %zu bytes of scratch, the static scratch holds %zu "
                         "(use gs_bin_sort with a workspace)", need, (size_t)GS_BIN_SORT_NOALLOC_BYTES);
    void* ws = nullptr;
    if ((st = noalloc_scratch(&ws))) return st;
    return launch_bin_sort(proj, views, bins, ws, (hipStream_t)stream, nullptr);
}

gs_status gs_render_fwd(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                        float* rgb, float* t_final, uint32_t* n_last, uint32_t* n_contrib, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if ((st = check_queue(views, bins))) return st;
    if (views->n_pixels > 0 && (!rgb || !t_final || !n_last))
        return set_error(GS_ERR_INVALID_ARG, "output image pointer is NULL");
    return launch_render_fwd(proj, views, bins, p, rgb, t_final, n_last, n_contrib, (hipStream_t)stream);
}

gs_status gs_bin_sort_render_fwd(const gs_projected* proj, const gs_views* views, gs_bins* bins, const gs_params* p,
                                 float* rgb, float* t_final, uint32_t* n_last, uint32_t* n_contrib, void* ws,
                                 size_t ws_bytes, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if ((st = check_queue(views, bins))) return st;
    const size_t need = sort_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    if (views->n_pixels > 0 && (!rgb || !t_final || !n_last))
        return set_error(GS_ERR_INVALID_ARG, "output image pointer is NULL");
    TileSortArgs ta;
    if ((st = launch_bin_sort(proj, views, bins, ws, (hipStream_t)stream, &ta))) return st;
    return launch_render_fwd_sorted(proj, views, bins, p, rgb, t_final, n_last, n_contrib, ta, (hipStream_t)stream);
}

gs_status gs_l1_loss_grad(const float* rgb, const float* target, int64_t n, float scale, float* dl_drgb,
                          float* loss_accum, void* stream) {
    if (n < 0 || (n > 0 && (!rgb || !target || !dl_drgb)))
        return set_error(GS_ERR_INVALID_ARG, "gs_l1_loss_grad: bad arguments");
    return launch_l1(rgb, target, n, scale, dl_drgb, loss_accum, (hipStream_t)stream);
}

size_t gs_ssim_workspace_bytes(int32_t n_planes, int32_t height, int32_t width) {
    return ssim_workspace_bytes(n_planes, height, width);
}

gs_status gs_ssim_loss_grad(const float* img, const float* target, int32_t n_planes, int32_t height, int32_t width,
                            int64_t n_norm, float lambda, float* dl_dimg, float* loss_accum, void* ws,
                            size_t ws_bytes, void* stream) {
    if (n_planes < 0 || n_planes > 65535)
        return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: n_planes must be in [0, 65535]");
    if (n_planes == 0) return GS_OK;
    if (height < 1 || width < 1) return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: height and width must be >= 1");
    if ((int64_t)height * width > INT32_MAX || width > (INT32_MAX - 128) / 32)
        return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: a plane must hold fewer than 2^31 pixels");
    if (n_norm < 1) return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: n_norm must be >= 1");
    if (!(lambda >= 0.f && lambda <= 1.f))
        return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: lambda must be in [0, 1]");
    if (!img || !target || !dl_dimg) return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: NULL image pointer");
    if (dl_dimg == img || dl_dimg == target)
        return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: dl_dimg aliases an input image");
    const size_t need = ssim_workspace_bytes(n_planes, height, width);
    if (!ws || ws_bytes < need)
        return set_error(GS_ERR_INVALID_ARG, "gs_ssim_loss_grad: workspace of %zu bytes needed, %zu given", need,
                         ws ? ws_bytes : (size_t)0);
    return launch_ssim_loss_grad(img, target, n_planes, height, width, n_norm, lambda, dl_dimg, loss_accum, ws,
                                 (hipStream_t)stream);
}

gs_status gs_render_bwd(const gs_gaussians* g, const gs_views* views, const gs_projected* proj, const gs_bins* bins,
                        const gs_params* p, const float* t_final, const uint32_t* n_last, const float* dl_drgb,
                        gs_gaussians_grad* grad, void* ws, size_t ws_bytes, void* stream) {
    gs_status st;
    if ((st = check_gaussians(g)) || (st = check_views(views)) || (st = check_projected(proj, true)) ||
        (st = check_bins(bins)) || (st = check_params(p)))
        return st;
    if (!grad || grad->n != g->n || grad->sh_degree != g->sh_degree)
        return set_error(GS_ERR_INVALID_ARG, "grad buffers missing or shaped unlike the Gaussians");
    if (grad->overwrite != 0 && grad->overwrite != 1)
        return set_error(GS_ERR_INVALID_ARG, "grad->overwrite must be 0 or 1 (got %d)", grad->overwrite);
    if (g->n > 0 && (!grad->mean || !grad->scale || !grad->quat || !grad->opacity || !grad->sh || !g->sh))
        return set_error(GS_ERR_INVALID_ARG, "gradient or SH pointer is NULL");
    if (proj->n != g->n)
        return set_error(GS_ERR_INVALID_ARG, "backward needs a projection of all Gaussians (no subset)");
    if ((st = check_queue(views, bins))) return st;
    if (views->n_pixels > 0 && (!t_final || !n_last || !dl_drgb))
        return set_error(GS_ERR_INVALID_ARG, "t_final, n_last or dl_drgb is NULL");
    if (g->n > 0 && !bins->entry_offset)
        return set_error(GS_ERR_INVALID_ARG, "the backward needs bins->entry_offset (written by gs_bin_sort)");
    const size_t need = bwd_workspace_bytes(bins->capacity, g->n, views->n_views);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    float* slots = (float*)ws;
    float* g2 = (float*)((char*)ws + bwd_slots_bytes(bins->capacity));
    if ((st = launch_render_bwd(proj, views, bins, p, t_final, n_last, dl_drgb, slots, s))) return st;
    return launch_preprocess_bwd(g, views, p, proj, bins, slots, g2, grad, s);
}

gs_status gs_importance(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                        float* h_accum, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if (proj->n > 0 && !h_accum) return set_error(GS_ERR_INVALID_ARG, "h_accum is NULL");
    if ((st = check_queue(views, bins))) return st;
    return launch_importance(proj, views, bins, p, h_accum, (hipStream_t)stream);
}

gs_status gs_cluster_visibility(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                                const gs_params* p, const int32_t* view_cluster, int32_t k, float t_cluster,
                                uint32_t* bits_accum, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if (k < 1) return set_error(GS_ERR_INVALID_ARG, "k must be >= 1 (got %d)", k);
    if (!view_cluster || (proj->n > 0 && !bits_accum))
        return set_error(GS_ERR_INVALID_ARG, "view_cluster or bits_accum is NULL");
    if (!(t_cluster >= 0.f)) return set_error(GS_ERR_INVALID_ARG, "t_cluster must be >= 0");
    if ((st = check_queue(views, bins))) return st;
    return launch_visibility(proj, views, bins, p, view_cluster, k, t_cluster, bits_accum, (hipStream_t)stream);
}

gs_status gs_bin_sort_importance(const gs_projected* proj, const gs_views* views, gs_bins* bins, const gs_params* p,
                                 float* h_accum, void* ws, size_t ws_bytes, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if (proj->n > 0 && !h_accum) return set_error(GS_ERR_INVALID_ARG, "h_accum is NULL");
    if ((st = check_queue(views, bins))) return st;
    const size_t need = sort_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    TileSortArgs ta;
    if ((st = launch_bin_sort(proj, views, bins, ws, (hipStream_t)stream, &ta))) return st;
    return launch_importance_sorted(proj, views, bins, p, h_accum, ta, (hipStream_t)stream);
}

gs_status gs_bin_sort_cluster_visibility(const gs_projected* proj, const gs_views* views, gs_bins* bins,
                                         const gs_params* p, const int32_t* view_cluster, int32_t k, float t_cluster,
                                         uint32_t* bits_accum, void* ws, size_t ws_bytes, void* stream) {
    gs_status st;
    if ((st = check_projected(proj, true)) || (st = check_views(views)) || (st = check_bins(bins)) ||
        (st = check_params(p)))
        return st;
    if (k < 1) return set_error(GS_ERR_INVALID_ARG, "k must be >= 1 (got %d)", k);
    if (!view_cluster || (proj->n > 0 && !bits_accum))
        return set_error(GS_ERR_INVALID_ARG, "view_cluster or bits_accum is NULL");
    if (!(t_cluster >= 0.f)) return set_error(GS_ERR_INVALID_ARG, "t_cluster must be >= 0");
    if ((st = check_queue(views, bins))) return st;
    const size_t need = sort_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    TileSortArgs ta;
    if ((st = launch_bin_sort(proj, views, bins, ws, (hipStream_t)stream, &ta))) return st;
    return launch_visibility_sorted(proj, views, bins, p, view_cluster, k, t_cluster, bits_accum, ta,
                                    (hipStream_t)stream);
}

gs_status gs_bits_to_list(const uint32_t* bits_row, int64_t n, int32_t* list, int64_t* count, void* ws,
                          size_t ws_bytes, void* stream) {
    if (n < 0 || !count || (n > 0 && (!bits_row || !list)))
        return set_error(GS_ERR_INVALID_ARG, "gs_bits_to_list: bad arguments");
    const size_t need = list_workspace_bytes(n);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    return launch_bits_to_list(bits_row, n, list, count, ws, (hipStream_t)stream);
}

gs_status gs_prune_mask(const float* h, int64_t n, float t_prune, uint8_t* mask, void* stream) {
    if (n < 0 || (n > 0 && (!h || !mask))) return set_error(GS_ERR_INVALID_ARG, "gs_prune_mask: bad arguments");
    if (!(t_prune == t_prune)) return set_error(GS_ERR_INVALID_ARG, "gs_prune_mask: t_prune is NaN");
    return launch_prune_mask(h, n, t_prune, mask, (hipStream_t)stream);
}

gs_status gs_prune(const float* h, int64_t n, float t_prune, const float* const* planes_in, float* const* planes_out,
                   int32_t n_planes, int32_t* kept, int64_t* n_kept, void* ws, size_t ws_bytes, void* stream) {
    if (n < 0 || n_planes < 0 || !n_kept || (n > 0 && (!h || !kept)) || (n_planes > 0 && (!planes_in || !planes_out)))
        return set_error(GS_ERR_INVALID_ARG, "gs_prune: bad arguments");
    if (n >= ((int64_t)1 << 31)) return set_error(GS_ERR_UNSUPPORTED, "gs_prune: at most 2^31-1 Gaussians");
    if (!(t_prune == t_prune)) return set_error(GS_ERR_INVALID_ARG, "gs_prune: t_prune is NaN");
    for (int p = 0; p < n_planes; ++p) {
        if (n > 0 && (!planes_in[p] || !planes_out[p]))
            return set_error(GS_ERR_INVALID_ARG, "gs_prune: plane %d is NULL", p);
        for (int q = 0; q < n_planes; ++q)
            if (n > 0 && planes_out[p] == planes_in[q])
                return set_error(GS_ERR_INVALID_ARG, "gs_prune: output plane %d aliases input plane %d", p, q);
    }
    const size_t need = prune_workspace_bytes(n) + list_workspace_bytes(n);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "workspace too small: %zu bytes, need %zu", ws_bytes, need);
    return launch_prune(h, n, t_prune, planes_in, planes_out, n_planes, kept, n_kept, ws, prune_workspace_bytes(n),
                        (hipStream_t)stream);
}

gs_status gs_gather(const int32_t* index, int64_t n_index, int64_t n_src, const float* const* planes_in,
                    float* const* planes_out, int32_t n_planes, void* stream) {
    if (n_index < 0 || n_src < 0 || n_planes < 0 || (n_index > 0 && !index) ||
        (n_planes > 0 && (!planes_in || !planes_out)))
        return set_error(GS_ERR_INVALID_ARG, "gs_gather: bad arguments");
    if (n_index >= ((int64_t)1 << 31) || n_src >= ((int64_t)1 << 31))
        return set_error(GS_ERR_UNSUPPORTED, "gs_gather: at most 2^31-1 entries");
    for (int p = 0; p < n_planes; ++p) {
        if (n_index > 0 && (!planes_in[p] || !planes_out[p]))
            return set_error(GS_ERR_INVALID_ARG, "gs_gather: plane %d is NULL", p);
        for (int q = 0; q < n_planes; ++q)
            if (n_index > 0 && planes_out[p] == planes_in[q])
                return set_error(GS_ERR_INVALID_ARG, "gs_gather: output plane %d aliases input plane %d", p, q);
    }
    return launch_gather(index, n_index, n_src, planes_in, planes_out, n_planes, (hipStream_t)stream);
}

size_t gs_nn_workspace_bytes(int64_t n) { return nn_workspace_bytes(n); }

static gs_status check_nn(const float* points, int64_t n, size_t ws_bytes, const void* ws, const char* who) {
    if (n < 0 || (n > 0 && !points)) return set_error(GS_ERR_INVALID_ARG, "%s: bad arguments", who);
    if (n >= ((int64_t)1 << 31)) return set_error(GS_ERR_UNSUPPORTED, "%s: at most 2^31-1 points", who);
    const size_t need = nn_workspace_bytes(n);
    if (ws_bytes < need || (need > 0 && !ws))
        return set_error(GS_ERR_INVALID_ARG, "%s: workspace too small: %zu bytes, need %zu", who, ws_bytes, need);
    return GS_OK;
}

gs_status gs_nn_distance(const float* points, int64_t n, float* dist, void* ws, size_t ws_bytes, void* stream) {
    gs_status st = check_nn(points, n, ws_bytes, ws, "gs_nn_distance");
    if (st) return st;
    if (n > 0 && !dist) return set_error(GS_ERR_INVALID_ARG, "gs_nn_distance: dist is NULL");
    return launch_nn_distance(points, n, dist, ws, (hipStream_t)stream);
}

gs_status gs_init_gaussians(const float* points, const float* colours, int64_t n, int32_t sh_degree, float* mean,
                            float* scale, float* quat, float* opacity, float* sh, void* ws, size_t ws_bytes,
                            void* stream) {
    gs_status st = check_nn(points, n, ws_bytes, ws, "gs_init_gaussians");
    if (st) return st;
    if (sh_degree < 0 || sh_degree > 3)
        return set_error(GS_ERR_UNSUPPORTED, "gs_init_gaussians: sh_degree must be 0..3");
    if (n > 0 && (!mean || !scale || !quat || !opacity || !sh))
        return set_error(GS_ERR_INVALID_ARG, "gs_init_gaussians: NULL output plane");
    if (n > 0 && (mean == points || (colours && (sh == colours || mean == colours))))
        return set_error(GS_ERR_INVALID_ARG, "gs_init_gaussians: an output aliases an input");
    return launch_init_gaussians(points, colours, n, sh_degree, mean, scale, quat, opacity, sh, ws,
                                 (hipStream_t)stream);
}

size_t gs_kmeans_workspace_bytes(int64_t m, int32_t k, int32_t max_iter) {
    return kmeans_workspace_bytes(m, k, max_iter);
}

gs_status gs_kmeans_lloyd(const double* pos, int64_t m, int32_t k, int32_t max_iter, double* centres,
                          int32_t* assign, int32_t* iterations, void* ws, size_t ws_bytes, void* stream) {
    if (!pos || !centres || !assign || m < 1 || k < 1 || k > m || max_iter < 1)
        return set_error(GS_ERR_INVALID_ARG, "gs_kmeans_lloyd: need 1 <= k <= m, max_iter >= 1 and non-NULL buffers");
    if (m >= ((int64_t)1 << 31)) return set_error(GS_ERR_UNSUPPORTED, "gs_kmeans_lloyd: at most 2^31-1 points");
    if (k > kmeans_max_centres())
        return set_error(GS_ERR_UNSUPPORTED, "gs_kmeans_lloyd: at most %d centres (got %d)", kmeans_max_centres(), k);
    if (max_iter > 1000000) return set_error(GS_ERR_UNSUPPORTED, "gs_kmeans_lloyd: at most 10^6 iterations");
    const size_t need = kmeans_workspace_bytes(m, k, max_iter);
    if (ws_bytes < need || !ws)
        return set_error(GS_ERR_INVALID_ARG, "gs_kmeans_lloyd: workspace too small: %zu bytes, need %zu", ws_bytes,
                         need);
    const char *p0 = (const char*)pos, *p1 = p0 + 24 * m, *c0 = (const char*)centres, *c1 = c0 + 24 * (int64_t)k,
               *a0 = (const char*)assign, *a1 = a0 + 4 * m;
    auto overlap = [](const char* b0, const char* e0, const char* b1, const char* e1) { return b0 < e1 && b1 < e0; };
    if (overlap(p0, p1, c0, c1) || overlap(p0, p1, a0, a1) || overlap(c0, c1, a0, a1))
        return set_error(GS_ERR_INVALID_ARG, "gs_kmeans_lloyd: pos, centres and assign must not overlap");
    return launch_kmeans_lloyd(pos, m, k, max_iter, centres, assign, iterations, ws, (hipStream_t)stream);
}

gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, double beta1, double beta2, double eps,
                       int64_t step, int32_t zero_grad, void* stream) {
    if (n_groups < 0 || (n_groups > 0 && !groups) || step < 1)
        return set_error(GS_ERR_INVALID_ARG, "gs_adam_step: bad arguments");
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0))
        return set_error(GS_ERR_INVALID_ARG, "gs_adam_step: betas must be in [0, 1), eps >= 0");
    for (int k = 0; k < n_groups; ++k) {
        const gs_adam_group& g = groups[k];
        if (g.count < 0 || (g.count > 0 && (!g.param || !g.grad || !g.m || !g.v)))
            return set_error(GS_ERR_INVALID_ARG, "gs_adam_step: group %d has a NULL buffer or negative count", k);
        if (g.mode != GS_ADAM_LINEAR && g.mode != GS_ADAM_LOG && g.mode != GS_ADAM_LOGIT)
            return set_error(GS_ERR_INVALID_ARG, "gs_adam_step: group %d has unknown mode %d", k, g.mode);
        if (g.count > 0 && (g.param == g.grad || g.param == g.m || g.param == g.v || g.grad == g.m ||
                            g.grad == g.v || g.m == g.v))
            return set_error(GS_ERR_INVALID_ARG, "gs_adam_step: group %d buffers alias", k);
    }
    return launch_adam(groups, n_groups, beta1, beta2, eps, step, zero_grad, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------------------
// camera clustering on the host (a few hundred points; no device work)
// ---------------------------------------------------------------------------------------
static uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

static double d2(const double* a, const double* b) {
#pragma clang fp contract(off)
    const double x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
    return x * x + y * y + z * z;
}

int32_t gs_nearest_centre(const double* centres, int32_t k, const double* x) {
    if (!centres || !x || k < 1) return -1;
    int32_t best = 0;
    double bd = d2(centres, x);
    for (int32_t c = 1; c < k; ++c) {
        const double d = d2(centres + 3 * c, x);
        if (d < bd) {
            bd = d;
            best = c;
        }
    }
    return best;
}

static void kmeans_seed(const double* pos, int32_t m, int32_t k, uint64_t seed, double* centres) {
    uint64_t s = seed;
    // k-means++ seeding
    std::vector<double> dist(m);
    int32_t first = (int32_t)(splitmix64(s) % (uint64_t)m);
    for (int e = 0; e < 3; ++e) centres[e] = pos[3 * first + e];
    for (int32_t i = 0; i < m; ++i) dist[i] = d2(pos + 3 * i, centres);
    for (int32_t c = 1; c < k; ++c) {
        double tot = 0;
        for (int32_t i = 0; i < m; ++i) tot += dist[i];
        int32_t pick = m - 1;
        if (tot > 0) {
            const double r = uniform01(s) * tot;
            double acc = 0;
            for (int32_t i = 0; i < m; ++i) {
                acc += dist[i];
                if (acc > r) {
                    pick = i;
                    break;
                }
            }
        } else {
            pick = (int32_t)(splitmix64(s) % (uint64_t)m);
        }
        for (int e = 0; e < 3; ++e) centres[3 * c + e] = pos[3 * pick + e];
        for (int32_t i = 0; i < m; ++i) dist[i] = std::min(dist[i], d2(pos + 3 * i, centres + 3 * c));
    }
}

gs_status gs_kmeans_seed(const double* pos, int32_t m, int32_t k, uint64_t seed, double* centres) {
    if (!pos || !centres || m < 1 || k < 1 || k > m)
        return set_error(GS_ERR_INVALID_ARG, "gs_kmeans_seed: need 1 <= k <= m and non-NULL buffers");
    kmeans_seed(pos, m, k, seed, centres);
    return GS_OK;
}

gs_status gs_kmeans(const double* pos, int32_t m, int32_t k, uint64_t seed, int32_t max_iter, double* centres,
                    int32_t* assign) {
    if (!pos || !centres || !assign || m < 1 || k < 1 || k > m || max_iter < 0)
        return set_error(GS_ERR_INVALID_ARG, "gs_kmeans: need 1 <= k <= m and non-NULL buffers");
    kmeans_seed(pos, m, k, seed, centres);
    // Lloyd iterations
    for (int32_t i = 0; i < m; ++i) assign[i] = -1;
    std::vector<double> sum(3 * (size_t)k);
    std::vector<int32_t> cnt(k);
    for (int32_t it = 0; it < std::max(1, max_iter); ++it) {
        bool changed = false;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t c = gs_nearest_centre(centres, k, pos + 3 * i);
            if (c != assign[i]) {
                assign[i] = c;
                changed = true;
            }
        }
        if (!changed && it > 0) break;
        std::fill(sum.begin(), sum.end(), 0.0);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int32_t i = 0; i < m; ++i) {
            const int32_t c = assign[i];
            for (int e = 0; e < 3; ++e) sum[3 * c + e] += pos[3 * i + e];
            cnt[c]++;
        }
        // an empty cluster is re-seeded at the point farthest from its assigned centre (the
        // centres of this assignment, before any of them moves; ties to the lowest index)
        int32_t far = -1;
        for (int32_t c = 0; c < k && far < 0; ++c)
            if (cnt[c] == 0) {
                double fd = -1;
                for (int32_t i = 0; i < m; ++i) {
                    const double d = d2(pos + 3 * i, centres + 3 * assign[i]);
                    if (d > fd) {
                        fd = d;
                        far = i;
                    }
                }
            }
        for (int32_t c = 0; c < k; ++c) {
            if (cnt[c] > 0) {
                for (int e = 0; e < 3; ++e) centres[3 * c + e] = sum[3 * c + e] / cnt[c];
            } else {
                for (int e = 0; e < 3; ++e) centres[3 * c + e] = pos[3 * far + e];
            }
        }
        if (it + 1 >= max_iter) {
            for (int32_t i = 0; i < m; ++i) assign[i] = gs_nearest_centre(centres, k, pos + 3 * i);
            break;
        }
    }
    return GS_OK;
}

}  // extern "C"
