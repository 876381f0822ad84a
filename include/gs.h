/*
 * gs.h -- C ABI of the MI355X (gfx950) Gaussian-splatting hot path of RadSplat
 * (arXiv 2403.13806).
 *
 * The library renders a set of 3D Gaussians phi = {(p, k, s, o, q)} (Sec. 3.2)
 * for pinhole cameras with front-to-back alpha compositing (eq. render-gs),
 * computes the max-over-rays importance score used for pruning
 * (eq. importance-score, Sec. 3.3), the per-camera-cluster visibility indicator
 * lists used for test-time filtering (eq. importance-score-vis, Sec. 3.4), and the
 * gradient of a rendered image with respect to every Gaussian parameter (the
 * optimisation of phi in Sec. 3.2). Around that path: the training loss of Sec. 3.2
 * ((1 - lambda) L2 + lambda D-SSIM) and its gradient, pruning (stream compaction of
 * every per-Gaussian array, Sec. 3.3), gathering a Gaussian subset into compact planes
 * (materialised visibility lists), the initialisation of Sec. 3.2 (nearest-neighbour
 * scales), and the Adam step that optimises phi.
 *
 * Model (the paper inherits it from 3D Gaussian splatting and leaves these
 * constants open; the values are the defaults of gs_params):
 *   camera space      p_c = R p + t (x right, y down, z forward)
 *   covariance        Sigma = R(q/|q|) diag(s)^2 R(q/|q|)^T
 *   2D covariance     Sigma' = J R Sigma R^T J^T + lowpass * I, J the Jacobian
 *                     of (fx x/z + cx, fy y/z + cy) at the mean
 *   culling           z > znear, o >= alpha_min, |q| > 0, all finite, projected
 *                     mean inside guard * (image half-size) of the image centre
 *   support           pixel (px, py) is sampled at (px + 0.5, py + 0.5); with
 *                     d = centre - mean2d, it is covered iff d^T Sigma'^-1 d <= q_max,
 *                     q_max = min(kappa^2, 2 ln(o / alpha_min))
 *   opacity           alpha = min(alpha_max, o exp(-d^T Sigma'^-1 d / 2))
 *   colour            c = max(0, sum_{l<=deg,|m|<=l} k_lm Y_lm(dir) + 1/2), Y the
 *                     real orthonormal SH basis (Condon-Shortley phase), dir the
 *                     unit vector from the camera centre to the mean
 *   order             covered Gaussians sorted by (FP32 camera z, index)
 *   compositing       w_j = alpha_j T_j, T_j = prod_{k<j} (1 - alpha_k); the ray
 *                     ends after the first entry that takes T below t_min (that
 *                     entry is composited); C = sum_j w_j c_j + T_final * bg
 * Tiles: a Gaussian is binned into every tile (tile_w x tile_h pixels) of the
 * inclusive rectangle floor((u -/+ hx -/+ 2^-16) / tile_w) x floor((v -/+ hy -/+
 * 2^-16) / tile_h) clamped to the grid, hx = sqrt(q_max Sigma'_xx),
 * hy = sqrt(q_max Sigma'_yy): the exact bounding box of the support, so the image
 * does not depend on the tile size.
 *
 * Conventions for every call:
 *   - Pointers named in the argument structs are DEVICE pointers owned by the
 *     caller; the library never allocates device memory. Scratch memory is a
 *     caller-provided device workspace (gs_workspace_bytes).
 *   - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued
 *     asynchronously; no call synchronises the device.
 *   - Argument errors are detected on the host before anything is enqueued and
 *     returned as GS_ERR_INVALID_ARG / GS_ERR_UNSUPPORTED; a failed launch returns
 *     GS_ERR_HIP. gs_last_error() gives a message for the calling thread.
 *   - Pair-buffer overflow is detected on the device: gs_bin_sort writes the
 *     number of pairs required to *bins->n_pairs and sets bit 0 of *bins->overflow
 *     when it exceeds bins->capacity. No write goes out of bounds; the tile ranges
 *     are then left empty and the caller must retry with a larger capacity. Bit 1
 *     is set if a cross-block wait inside the sort ran out of its spin budget
 *     (results invalid, nothing written out of bounds); the kernels never hang.
 *     Bit 2 is set when a view has more tiles than views->max_view_tiles declares
 *     (results invalid, nothing written out of bounds).
 *   - Accumulating outputs (importance h, visibility bits, gradients) are
 *     combined into what the buffer holds (max, OR, +=), so results over view
 *     chunks compose; the caller initialises them.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
#define GS_OK 0
#define GS_ERR_INVALID_ARG (-1)
#define GS_ERR_CAPACITY (-2)
#define GS_ERR_HIP (-3)
#define GS_ERR_UNSUPPORTED (-4)

/* Pinhole camera, world -> camera p_c = R p + t. 80 bytes. */
typedef struct gs_camera {
    float R[9]; /* row-major */
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height; /* pixels, >= 1 */
    float znear;           /* near plane (camera z), > 0 */
    int32_t reserved;      /* set to 0 */
} gs_camera;

/* Model constants (see the model above). Defaults: 0.3, 3, 1/255, 0.99, 1e-4, 1.3, {0,0,0}. */
typedef struct gs_params {
    float lowpass, kappa, alpha_min, alpha_max, t_min, guard;
    float bg[3];
} gs_params;

/* Gaussian parameters, structure of arrays over n Gaussians (Sec. 3.2):
 *   mean    [3][n]  position p
 *   scale   [3][n]  linear scales s (> 0)
 *   quat    [4][n]  rotation quaternion (w, x, y, z), any non-zero norm
 *   opacity [n]     o in [0, 1]
 *   sh      [(sh_degree+1)^2 * 3][n]; row (k*3 + c) = SH coefficient k (k = l*l+l+m)
 *                   of colour channel c */
typedef struct gs_gaussians {
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* sh;
    int64_t n;
    int32_t sh_degree; /* 0..3 */
} gs_gaussians;

/* Gradient buffers, same layout as gs_gaussians.
 *   overwrite  0: gs_render_bwd adds into the buffers (+=), touching only the Gaussians a
 *              pair contributes to; 1: it writes every entry of every buffer (=), zeros where
 *              nothing contributes, so the buffers need no clearing and are not read. */
typedef struct gs_gaussians_grad {
    float* mean;
    float* scale;
    float* quat;
    float* opacity;
    float* sh;
    int64_t n;
    int32_t sh_degree;
    int32_t overwrite;
} gs_gaussians_grad;

/* Projected Gaussian, 64 bytes, one per (view, Gaussian): everything a compositing
 * pass needs. Conic (ca, cb, cc) = inverse of Sigma' as [[ca, cb], [cb, cc]]. rgb is
 * max(0, sum k Y + 1/2) in FP32, saturated at the largest finite FP32 value. */
typedef struct gs_splat {
    double u, v;
    double ca, cb, cc;
    double qmax;
    float opacity;
    float rgb[3];
} gs_splat;

/* A batch of views rendered together: views are laid out one after another in a
 * global tile space and a global pixel space.
 *   tile_offset[v]  first global tile of view v; tile_offset[n_views] = n_tiles.
 *                   View v has ceil(W/tile_w) * ceil(H/tile_h) tiles, row-major.
 *   pixel_offset[v] first global pixel of view v; pixel_offset[n_views] = n_pixels.
 * Image buffers: rgb is [3 * n_pixels] with view v's planar [3][H][W] image at
 * 3 * pixel_offset[v]; per-pixel buffers (t_final, n_last) are [n_pixels] with view
 * v's [H][W] at pixel_offset[v]. gs_view_layout fills both offset tables on the host. */
typedef struct gs_views {
    const gs_camera* cams;       /* device [n_views] */
    const int32_t* tile_offset;  /* device [n_views + 1] */
    const int64_t* pixel_offset; /* device [n_views + 1] */
    int32_t n_views;
    int32_t tile_w, tile_h;      /* 8, 16 or 32 each (one workgroup thread per tile pixel) */
    int32_t n_tiles;
    int64_t n_pixels;
    int32_t batch_depth;         /* list records staged per lane per batch in compositing: 1 or 2
                                    (2 only for tiles of at most 512 pixels) */
    int32_t lpt;                 /* 1: the traversals take tiles longest list first (bins->queue);
                                    0: in tile order */
    int32_t pixels_per_lane;     /* each lane of the traversals handles 1, 2 (2 x 1) or 4 (2 x 2
                                    in the reverse one; 4 x 1 in the forward ones where tile_w >=
                                    32, else 2 x 1) neighbouring pixels; 2 needs tile_w >= 16, 4
                                    also tile_h >= 16; 0 picks the default for the tile size.
                                    Results do not depend on it, except for the order of the
                                    reverse traversal's FP32 sums */
    int32_t max_view_tiles;      /* tiles of the view with the most (gs_view_layout's table gives
                                    them), or 0: taken as n_tiles. gs_bin_sort writes the pairs
                                    straight into their tiles' ranges when it is at most 8192 */
} gs_views;

/* Per-(view, Gaussian) outputs of gs_preprocess, [n_views][n] each:
 *   splat  records (written only where count > 0)
 *   depth  FP32 camera z (the depth key)
 *   rect   tile rectangle packed as tx0 | ty0 << 16 | tx1 << 32 | ty1 << 48 (inclusive)
 *   count  number of tiles in rect; 0 when the Gaussian is culled or off-screen */
typedef struct gs_projected {
    gs_splat* splat;
    float* depth;
    uint64_t* rect;
    uint32_t* count;
    int64_t n; /* entries per view */
} gs_projected;

/* Binned (tile, depth, index) pairs sorted by key then value, and per-tile ranges.
 *   keys    [capacity] key = global tile << 32 | bits(FP32 depth)
 *   vals    [capacity] index of the Gaussian within its view (0 .. n-1)
 *   ranges  [n_tiles][2] [start, end) of each tile in keys/vals
 *   n_pairs device scalar: pairs required
 *   overflow device scalar: 0 when the bins are valid (see the conventions above); cleared
 *           by every gs_bin_sort
 *   queue   [n_tiles] or NULL: when set, gs_bin_sort also writes every tile id ordered by
 *           decreasing list length (by powers of two; order within a power is unspecified),
 *           the work order of the traversals when views->lpt is set
 *   entry_offset  [n_views * n] or NULL: when set, gs_bin_sort writes the emission slot of
 *           each (view, entry): the exclusive prefix sum of the tile counts in (view, entry)
 *           order, so entry o owns the slots [entry_offset[o], entry_offset[o] + count[o]), one
 *           per tile of its rectangle in row-major order. gs_render_bwd needs it.
 *   overflow_sticky  device scalar or NULL: when set, every gs_bin_sort ORs its overflow word
 *           into it; the library never clears it, so it reports an overflow in any frame since
 *           the caller last cleared it */
typedef struct gs_bins {
    uint64_t* keys;
    uint32_t* vals;
    uint32_t* ranges;
    uint64_t capacity; /* < 2^32 */
    uint64_t* n_pairs;
    uint32_t* overflow;
    uint32_t* queue;
    uint32_t* entry_offset;
    uint32_t* overflow_sticky;
} gs_bins;

/* Host helper: fill tile_offset[n_views+1] and pixel_offset[n_views+1] (HOST arrays)
 * for host cameras cams[n_views] and a tile size; returns GS_ERR_INVALID_ARG for bad
 * sizes or a total tile count >= 2^31. */
gs_status gs_view_layout(const gs_camera* cams, int32_t n_views, int32_t tile_w, int32_t tile_h,
                         int32_t* tile_offset, int64_t* pixel_offset);

/* Device workspace bytes needed by gs_bin_sort / gs_render_bwd / gs_bits_to_list / gs_prune for n
 * entries per view, n_views views, a pair capacity and n_tiles tiles (gs_render_bwd keeps nine
 * FP32 partial gradients per pair: 36 bytes x capacity). */
size_t gs_workspace_bytes(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles);

/* Project every Gaussian (or the listed subset) into every view of `views` (Sec. 3.2:
 * Sigma = R S S^T R^T, Sigma' = J M Sigma M^T J^T), evaluate its SH colour for the
 * view direction (skipped when want_color == 0, rgb is then 0), its FP32 depth key and
 * its tile rectangle. subset: device [n_subset] Gaussian indices in increasing order, or
 * NULL for all; out->n must equal n_subset (or g->n). Entry j of each view refers to
 * Gaussian subset[j] (or j). */
gs_status gs_preprocess(const gs_gaussians* g, const gs_views* views, const gs_params* p, const int32_t* subset,
                        int64_t n_subset, int32_t want_color, gs_projected* out, void* stream);

/* Bin projected Gaussians into tiles and sort the pairs by (tile, depth, index) (the
 * "correctly-sorted points" of eq. render-gs, per tile): pair counts per tile, their
 * exclusive scan (tile ranges, pair total, capacity check), a scatter of the pairs into
 * their tiles' ranges, and a sort of each tile's list by (FP32 depth bits, index) in LDS.
 * The result is deterministic. ws: device workspace of at least
 * gs_workspace_bytes(proj->n, views->n_views, bins->capacity, views->n_tiles). */
gs_status gs_bin_sort(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* ws, size_t ws_bytes,
                      void* stream);

/* gs_bin_sort without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments and results as gs_bin_sort; the scratch is a static device array of
 * GS_BIN_SORT_NOALLOC_BYTES (64 MiB) that each GPU the library runs on holds until the
 * process ends (its address is looked up once per device, on the first call). The call
 * allocates nothing. A frame whose scratch need (the gs_bin_sort workspace: about 25 bytes per
 * pair of capacity, plus 4 bytes per 4096 entries and tile of the largest view, at most 8192)
 * exceeds it returns GS_ERR_UNSUPPORTED before
 * anything is enqueued. Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents (each call clears what it needs itself): calls that overlap on one GPU
 * (other streams, other threads) race, so serialise them. */
#define GS_BIN_SORT_NOALLOC_BYTES (64u << 20)
gs_status gs_bin_sort_noalloc(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* stream);

/* Front-to-back compositing of every pixel of every view (eq. render-gs). Writes rgb
 * [3 * n_pixels], t_final [n_pixels] (transmittance after the last composited entry)
 * and n_last [n_pixels] (1 + position in keys/vals of the pixel's last composited
 * entry, or its tile's range start when none); t_final and n_last are what
 * gs_render_bwd needs. n_contrib (device [n_pixels], or NULL) receives the number of
 * Gaussians composited into each pixel. */
gs_status gs_render_fwd(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                        float* rgb, float* t_final, uint32_t* n_last, uint32_t* n_contrib, void* stream);

/* gs_bin_sort followed by gs_render_fwd, in fewer launches: each tile's sort by (depth, index)
 * (eq. render-gs) is done by the compositing workgroup of that tile right before it composites
 * the tile, so the tiles sorted first start compositing while others are still being sorted.
 * Arguments as in the two calls (ws as for gs_bin_sort); the same results: keys, vals, ranges,
 * counts and flags of bins as gs_bin_sort leaves them, and the same image, t_final, n_last and
 * n_contrib, bit for bit. Tile shapes whose compositing workgroup does not have 256 threads
 * (the sort's) run the two steps as two launches. */
gs_status gs_bin_sort_render_fwd(const gs_projected* proj, const gs_views* views, gs_bins* bins, const gs_params* p,
                                 float* rgb, float* t_final, uint32_t* n_last, uint32_t* n_contrib, void* ws,
                                 size_t ws_bytes, void* stream);

/* L1 photometric loss of a rendered batch against a target (the per-view training loss
 * whose gradient drives gs_render_bwd): dl_drgb[i] = sign(rgb[i] - target[i]) * scale
 * (sign(0) = 0) for i < n, and *loss_accum += scale * sum |rgb - target| (device scalar).
 * scale is usually 1 / n (mean reduction). */
gs_status gs_l1_loss_grad(const float* rgb, const float* target, int64_t n, float scale, float* dl_drgb,
                          float* loss_accum, void* stream);

/* Training loss of the point representation (Sec. 3.2): a weighted sum of the squared error
 * and the structural dissimilarity of the render x against the target y,
 *   L = (1 - lambda) sum (x - y)^2 / n_norm + lambda sum (1 - SSIM(x, y)) / n_norm
 * (the paper weighs the two terms with lambda = 0.2). SSIM is the per-pixel structural
 * similarity of Wang et al.: local means, variances and covariance from an 11 x 11 Gaussian
 * window of standard deviation 1.5 with zero padding outside the plane, C1 = 0.01^2,
 * C2 = 0.03^2 (intensities in [0, 1]). Each sum runs over the n_planes planes [height][width]
 * of img and target (contiguous, plane after plane; a view's planar [3][H][W] image is three
 * planes). n_norm is the element count the mean runs over: pass the batch total to each
 * call of a batch of views of different sizes, so the calls compose.
 *   dl_dimg     device [n_planes][height][width], written: dL/dx (must not alias img/target)
 *   loss_accum  device scalar or NULL: *loss_accum += this call's part of L
 *   ws          device workspace of at least gs_ssim_workspace_bytes(n_planes, height, width)
 * Errors: n_planes outside [0, 65535], a non-positive size or n_norm, a plane of 2^31 pixels
 * or more, lambda outside [0, 1], NULL pointers, dl_dimg aliasing an input or a short workspace
 * return GS_ERR_INVALID_ARG before anything is enqueued. */
size_t gs_ssim_workspace_bytes(int32_t n_planes, int32_t height, int32_t width);
gs_status gs_ssim_loss_grad(const float* img, const float* target, int32_t n_planes, int32_t height, int32_t width,
                            int64_t n_norm, float lambda, float* dl_dimg, float* loss_accum, void* ws,
                            size_t ws_bytes, void* stream);

/* Reverse mode of the render (the optimisation of the point representation phi, Sec. 3.2:
 * the Gaussians' positions, scales, rotations, opacities and SH coefficients are fitted by
 * gradient descent through the compositing of eq. render-gs). Given dL/d(rgb) (layout of rgb)
 * it adds dL/d(parameters) into grad, or writes them (grad->overwrite). Reverse traversal per
 * pixel from n_last, the transmittance before each entry recovered from t_final by division;
 * every pair's nine 2D partial sums (u, v, conic, opacity, colour) go to the pair's own slot
 * (no atomics), and each Gaussian's slots are summed in a fixed order, so the gradients
 * repeat bit for bit from run to run. proj must come from gs_preprocess with want_color = 1
 * and no subset; bins from gs_bin_sort with entry_offset set; ws as for gs_bin_sort
 * (gs_workspace_bytes with the bins' capacity). With grad->overwrite = 0 it adds (+=) and
 * nothing is added after a pair overflow (bins->overflow != 0); with grad->overwrite = 1 it
 * writes (=) every gradient, all zeros after a pair overflow. */
gs_status gs_render_bwd(const gs_gaussians* g, const gs_views* views, const gs_projected* proj,
                        const gs_bins* bins, const gs_params* p, const float* t_final, const uint32_t* n_last,
                        const float* dl_drgb, gs_gaussians_grad* grad, void* ws, size_t ws_bytes, void* stream);

/* Importance score (eq. importance-score): h[i] = max(h[i], max over the batch's pixels
 * of the weight alpha*T with which Gaussian i is composited). h_accum: device [n]
 * (n = proj->n; indices are view-entry indices, i.e. Gaussian indices without a
 * subset). The prune mask of Sec. 3.3 is h < t_prune. */
gs_status gs_importance(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                        float* h_accum, void* stream);

/* Cluster visibility (eq. importance-score-vis): for each view v with cluster
 * c = view_cluster[v] (device [n_views], 0 <= c < k), set bit i of row c of bits_accum
 * (device [k][ceil(n/32)] uint32, bit i%32 of word i/32) when Gaussian i is composited
 * with weight alpha*T > t_cluster in some pixel of v (that is, the per-cluster max
 * exceeds t_cluster). Bits are OR-ed into the buffer. A view whose cluster id lies outside
 * [0, k) sets no bit (the ids are device data, so the library cannot check them on the host). */
gs_status gs_cluster_visibility(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                                const gs_params* p, const int32_t* view_cluster, int32_t k, float t_cluster,
                                uint32_t* bits_accum, void* stream);

/* gs_bin_sort followed by gs_importance, and gs_bin_sort followed by gs_cluster_visibility,
 * with each tile's (depth, index) sort done by the traversal workgroup of that tile right
 * before it walks the tile (as gs_bin_sort_render_fwd does for compositing). Arguments as in
 * the two calls (ws as for gs_bin_sort); the same results bit for bit: the bins as gs_bin_sort
 * leaves them, and the same h_accum or bits_accum. */
gs_status gs_bin_sort_importance(const gs_projected* proj, const gs_views* views, gs_bins* bins, const gs_params* p,
                                 float* h_accum, void* ws, size_t ws_bytes, void* stream);
gs_status gs_bin_sort_cluster_visibility(const gs_projected* proj, const gs_views* views, gs_bins* bins,
                                         const gs_params* p, const int32_t* view_cluster, int32_t k, float t_cluster,
                                         uint32_t* bits_accum, void* ws, size_t ws_bytes, void* stream);

/* Visibility-list compaction (Sec. 3.4, list-based rendering): write the indices of the
 * set bits of bits_row (device [ceil(n/32)]) in increasing order to list (device [n]) and
 * their number to *count (device int64). ws: at least gs_workspace_bytes(n, 1, 0, 0). */
gs_status gs_bits_to_list(const uint32_t* bits_row, int64_t n, int32_t* list, int64_t* count, void* ws,
                          size_t ws_bytes, void* stream);

/* Prune mask (Sec. 3.3): mask[i] = 1 when h[i] < t_prune (Gaussian i is removed), else 0;
 * h: device [n] FP32 (a NaN counts as pruned), mask: device [n] bytes. */
gs_status gs_prune_mask(const float* h, int64_t n, float t_prune, uint8_t* mask, void* stream);

/* Pruning (Sec. 3.3, eq. importance-score and the mask h < t_prune): keep Gaussian i when
 * h[i] >= t_prune (device [n] FP32; a NaN is not kept) and compact n_planes FP32 planes of
 * length n in index order, planes_out[p][k] = planes_in[p][kept[k]]: the parameters and any
 * per-Gaussian state that must follow them (optimizer moments, ...). planes_in, planes_out:
 * HOST arrays of n_planes DEVICE pointers, caller-owned, each output at least [n] and none
 * aliasing an input plane. kept: device [n] int32, the kept indices in increasing order;
 * *n_kept: device int64, their number. ws: device workspace of at least
 * gs_workspace_bytes(n, 1, 0, 0). Asynchronous on the stream; argument errors are reported
 * before anything is enqueued. */
gs_status gs_prune(const float* h, int64_t n, float t_prune, const float* const* planes_in, float* const* planes_out,
                   int32_t n_planes, int32_t* kept, int64_t* n_kept, void* ws, size_t ws_bytes, void* stream);

/* Gather of per-Gaussian planes by an index list: planes_out[p][k] = planes_in[p][index[k]]
 * for k < n_index (host arrays of n_planes device pointers; index is a device int32 list).
 * It materialises a Gaussian subset, for example a camera cluster's visibility list
 * (Sec. 3.4), as compact planes: a render of the compact copy reads coalesced rows instead of
 * gathering, and when the list is increasing it keeps the subset's order, so the render is the
 * same as that of the subset. Indices outside [0, n_src) read nothing and give 0. Output
 * planes must hold n_index floats and must not alias an input plane. Errors: negative counts,
 * NULL pointers, aliasing (GS_ERR_INVALID_ARG), n_index or n_src >= 2^31 (GS_ERR_UNSUPPORTED). */
gs_status gs_gather(const int32_t* index, int64_t n_index, int64_t n_src, const float* const* planes_in,
                    float* const* planes_out, int32_t n_planes, void* stream);

/* Initialisation of the point representation from a point set P (Sec. 3.2), whose points
 * the caller provides (the paper draws them from a radiance field's median depths).
 * gs_nn_distance: dist[i] = min over p in P, p != p_i of ||p_i - p||_2, the isotropic scale
 * the paper gives each initial Gaussian. points is device [3][n] (the layout of
 * gs_gaussians.mean). Coincident copies of p_i are not neighbours; with no point at another
 * position dist[i] = +inf; a point with a non-finite coordinate gets NaN and is no one's
 * neighbour. Exact: squared distances in FP64 from the FP32 coordinates, (dx^2 + dy^2) + dz^2
 * without fused multiply-add, the square root rounded to FP32 once. Uniform cell grid
 * (about one cell per point over the bounding box) searched in rings of cells around each
 * point; the work grows with the distance to the nearest point in cells, so isolated points
 * far from all others are slow.
 *   ws  device workspace of at least gs_nn_workspace_bytes(n)
 * gs_init_gaussians: the same distances as scale (s, s, s), mean = points, quat = (1, 0, 0, 0),
 * opacity = 0.1, SH DC coefficient of channel c = (colour_c - 1/2) / Y_00 (so the colour
 * model returns the given colour; colours device [3][n] or NULL for 1/2), all other SH 0.
 * Outputs in the layout of gs_gaussians for sh_degree 0..3, written; they must not alias
 * points or colours.
 * Errors: n < 0, NULL pointers, aliasing, a short workspace (GS_ERR_INVALID_ARG),
 * n >= 2^31 or sh_degree outside 0..3 (GS_ERR_UNSUPPORTED). */
size_t gs_nn_workspace_bytes(int64_t n);
gs_status gs_nn_distance(const float* points, int64_t n, float* dist, void* ws, size_t ws_bytes, void* stream);
gs_status gs_init_gaussians(const float* points, const float* colours, int64_t n, int32_t sh_degree, float* mean,
                            float* scale, float* quat, float* opacity, float* sh, void* ws, size_t ws_bytes,
                            void* stream);

/* One Adam step over parameter groups (the optimisation of phi in Sec. 3.2; the paper takes
 * its optimiser from 3D Gaussian splatting without restating it). Per element of each group,
 * in the group's parametrisation u of the stored value x:
 *   GS_ADAM_LINEAR  u = x
 *   GS_ADAM_LOG     u = log x (x > 0), du = dx * x
 *   GS_ADAM_LOGIT   u = log(x / (1 - x)), x first clamped to [1e-6, 1 - 1e-6], du = dx x (1 - x)
 *   m = b1 m + (1 - b1) du,  v = b2 v + (1 - b2) du^2,
 *   u -= lr (m / (1 - b1^step)) / (sqrt(v) / sqrt(1 - b2^step) + eps),  x = u mapped back;
 * then grad = 0 when zero_grad is set. The moments and the step are FP32; 1 - b1, 1 - b2 and the
 * bias corrections are formed in FP64 from the FP64 arguments and rounded once (so b2 = 0.999
 * does not turn into 1 - fl32(0.999)). param, grad, m and v are device arrays of count floats
 * each (distinct buffers); step counts from 1. Groups with count 0 are skipped.
 * Errors: NULL pointers, step < 1, a negative count or an unknown mode (GS_ERR_INVALID_ARG). */
#define GS_ADAM_LINEAR 0
#define GS_ADAM_LOG 1
#define GS_ADAM_LOGIT 2
typedef struct gs_adam_group {
    float* param;
    float* grad;
    float* m;
    float* v;
    int64_t count;
    float lr;
    int32_t mode;
} gs_adam_group;
gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, double beta1, double beta2, double eps,
                       int64_t step, int32_t zero_grad, void* stream);

/* Host: k-means on camera positions (Sec. 3.4, input camera clustering), FP64 Lloyd
 * iterations from a k-means++ seeding with the given seed, at most max_iter iterations
 * or until assignments stop changing; ties go to the lowest centre; an empty cluster is
 * re-seeded at the point farthest from its centre in that iteration's assignment (ties to
 * the lowest index); sums run in index order. pos: host [m][3]; centres: host
 * [k][3]; assign: host [m]. */
gs_status gs_kmeans(const double* pos, int32_t m, int32_t k, uint64_t seed, int32_t max_iter, double* centres,
                    int32_t* assign);

/* Host: the k-means++ seeding of gs_kmeans alone (Sec. 3.4, input camera clustering): the
 * same splitmix64 stream from the seed, so gs_kmeans_lloyd from these centres follows
 * gs_kmeans. pos: host [m][3]; centres: host [k][3], written. Needs 1 <= k <= m. */
gs_status gs_kmeans_seed(const double* pos, int32_t m, int32_t k, uint64_t seed, double* centres);

/* Workspace of gs_kmeans_lloyd in bytes (0 for invalid sizes). */
size_t gs_kmeans_workspace_bytes(int64_t m, int32_t k, int32_t max_iter);

/* Device: FP64 Lloyd iterations of k-means on camera positions (Sec. 3.4, input camera
 * clustering), for camera sets too large for the host loop. From the centres given, each
 * iteration assigns every point to its nearest centre (squared distance formed as
 * (dx dx + dy dy) + dz dz without fused multiply-add; ties to the lowest centre) and stops
 * if, after the first iteration, no assignment changed; otherwise each centre moves to the
 * mean of its points and a centre without points moves to the point farthest from its
 * centre in that assignment (ties to the lowest index). After max_iter updates the points
 * are assigned once more. Sums run in a fixed order, so results repeat from run to run and
 * differ from a sequential sum in the last bits only.
 * pos: device [m][3] FP64, finite; centres: device [k][3], initial centres in, final out;
 * assign: device [m] int32 out; iterations: device int32 out (centre updates made), or NULL;
 * ws: device workspace of gs_kmeans_workspace_bytes(m, k, max_iter). Needs 1 <= k <= m,
 * k <= 2048, 1 <= max_iter <= 10^6, m < 2^31; pos, centres and assign must not overlap.
 * Asynchronous on the stream: 2 max_iter + 2 launches, those after convergence return at
 * once. Cost per iteration O(m k). */
gs_status gs_kmeans_lloyd(const double* pos, int64_t m, int32_t k, int32_t max_iter, double* centres,
                          int32_t* assign, int32_t* iterations, void* ws, size_t ws_bytes, void* stream);

/* Host: index of the centre nearest to x (squared distance, ties to the lowest index),
 * the cluster whose list renders a test view (Sec. 3.4). */
int32_t gs_nearest_centre(const double* centres, int32_t k, const double* x);

/* Message for the last error on the calling thread ("" if none). */
const char* gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
