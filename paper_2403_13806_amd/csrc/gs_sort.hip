// Tile binning and the (tile, depth, index) sort that gives every tile its
// front-to-back list ("correctly-sorted points", eq. render-gs):
//   scan     exclusive prefix sum of per-(view, Gaussian) tile counts (wave DPP scan ->
//            block scan -> reduce-then-scan across blocks), total pair count and
//            capacity check on the device
//   emit     one thread per visible (view, Gaussian) writes its tiles' keys
//            (global tile << 32 | FP32 depth bits) and values (entry index), in index
//            order, so a stable sort breaks depth ties by index
//   sort     LSD radix sort, 8-bit digits over the significant key bits only: per-block
//            digit histograms, a device scan of the digit-major histogram table, and a
//            stable scatter that ranks equal digits inside each wave with 8 ballots
//   ranges   [start, end) of every tile in the sorted list
#include "gs_device.hpp"

namespace gs {

constexpr int SCAN_T = 256;                // threads per scan block
constexpr int SCAN_ROUNDS = 16;            // items per thread
constexpr int SCAN_ITEMS = SCAN_T * SCAN_ROUNDS;
constexpr int SORT_T = 256;
constexpr int SORT_ROUNDS = 16;
constexpr int SORT_ITEMS = SORT_T * SORT_ROUNDS;

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------------------
// Device-wide exclusive scan of u32 values with a u64 running total.
// ---------------------------------------------------------------------------------------

// block-wide exclusive scan of one value per thread (256 threads), returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, uint32_t* wsum) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t incl = wave_incl_scan(x);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_T / 64; ++k) {
        const uint32_t s = wsum[k];
        pre += (k < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + incl - x;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                        uint64_t* __restrict__ block_sum) {
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
    uint64_t acc = 0;
    for (int r = 0; r < SCAN_ROUNDS; ++r) {
        const int64_t i = base + r * SCAN_T + threadIdx.x;
        acc += (i < n) ? in[i] : 0u;
    }
    // partial sums per thread are < 2^32 (16 counts of at most 2^27 each)
    uint32_t tot;
    block_excl_scan((uint32_t)acc, tot, wsum);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// single block: exclusive scan of nb u64 block sums; writes the grand total (and the
// capacity check) when requested
__global__ __launch_bounds__(1024) void k_scan_top(const uint64_t* __restrict__ block_sum, int64_t nb,
                                                   uint64_t* __restrict__ block_off, uint64_t* total_out,
                                                   uint32_t* overflow_out, uint64_t capacity) {
    __shared__ uint64_t buf[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(nb, b0 + per);
    uint64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += block_sum[b];
    buf[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t add = (t >= off) ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    uint64_t run = buf[t] - s;
    for (int64_t b = b0; b < b1; ++b) {
        block_off[b] = run;
        run += block_sum[b];
    }
    if (t == 1023) {
        if (total_out) *total_out = buf[1023];
        if (overflow_out) *overflow_out = buf[1023] > capacity ? 1u : 0u;
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_down(const uint32_t* __restrict__ in, int64_t n,
                                                      const uint64_t* __restrict__ block_off,
                                                      uint32_t* __restrict__ out) {
    __shared__ uint32_t wsum[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
    uint32_t carry = (uint32_t)block_off[blockIdx.x];  // offsets past 2^32 only occur on overflow
    for (int r = 0; r < SCAN_ROUNDS; ++r) {
        const int64_t i = base + r * SCAN_T + threadIdx.x;
        const uint32_t x = (i < n) ? in[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(x, tot, wsum);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
}

int64_t scan_blocks(int64_t n) { return (n + SCAN_ITEMS - 1) / SCAN_ITEMS; }

// exclusive scan in -> out (n items); scratch: 2 * scan_blocks(n) u64
gs_status launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint64_t* scratch, uint64_t* total,
                      uint32_t* overflow, uint64_t capacity, hipStream_t stream) {
    if (n <= 0) return GS_OK;
    const int64_t nb = scan_blocks(n);
    if (nb > 1024 * 256) return set_error(GS_ERR_UNSUPPORTED, "scan of %lld items exceeds the supported size", (long long)n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, stream, in, n, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, scratch, nb, scratch + nb, total, overflow,
                       capacity);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_T), 0, stream, in, n, scratch + nb, out);
    return check_launch("scan");
}

// ---------------------------------------------------------------------------------------
// Key emission
// ---------------------------------------------------------------------------------------
struct EmitArgs {
    const uint32_t* count;
    const uint32_t* offs;
    const uint64_t* rect;
    const float* depth;
    const gs_camera* cams;
    const int32_t* tile_offset;
    int64_t n;
    int tile_w;
    const uint32_t* overflow;
    uint64_t capacity;
    uint64_t* keys;
    uint32_t* vals;
};

__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    const int v = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n) return;
    if (*a.overflow) return;
    const int64_t o = (int64_t)v * a.n + j;
    const uint32_t c = a.count[o];
    if (c == 0) return;
    uint64_t off = a.offs[o];
    if (off + c > a.capacity) return;
    const uint64_t r = a.rect[o];
    const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff, y1 = (r >> 48) & 0xffff;
    const uint32_t tiles_x = (uint32_t)div_up(a.cams[v].width, a.tile_w);
    const uint32_t base = (uint32_t)a.tile_offset[v];
    const uint64_t dbits = __float_as_uint(a.depth[o]);
    for (uint32_t ty = y0; ty <= y1; ++ty)
        for (uint32_t tx = x0; tx <= x1; ++tx) {
            a.keys[off] = ((uint64_t)(base + ty * tiles_x + tx) << 32) | dbits;
            a.vals[off] = (uint32_t)j;
            ++off;
        }
}

// ---------------------------------------------------------------------------------------
// LSD radix sort passes
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(SORT_T) void k_radix_hist(const uint64_t* __restrict__ keys, const uint64_t* n_pairs,
                                                       uint64_t capacity, int shift, uint32_t* __restrict__ hist,
                                                       int64_t nblocks) {
    __shared__ uint32_t lh[256];
    const int t = threadIdx.x;
    lh[t] = 0;
    __syncthreads();
    const uint64_t count = min(*n_pairs, capacity);
    const int64_t base = (int64_t)blockIdx.x * SORT_ITEMS;
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t i = base + r * SORT_T + t;
        if ((uint64_t)i < count) atomicAdd(&lh[(keys[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = lh[t];
}

__global__ __launch_bounds__(SORT_T) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const uint64_t* n_pairs, uint64_t capacity, int shift,
                                                          const uint32_t* __restrict__ hist_off, int64_t nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[SORT_T / 64][256];
    const int t = threadIdx.x, w = t >> 6;
    const uint64_t count = min(*n_pairs, capacity);
    const int64_t base = (int64_t)blockIdx.x * SORT_ITEMS;
    if ((uint64_t)base >= count) return;  // uniform across the block
    run[t] = hist_off[(int64_t)t * nblocks + blockIdx.x];
    for (int r = 0; r < SORT_ROUNDS; ++r) {
        const int64_t i = base + r * SORT_T + t;
        const bool valid = (uint64_t)i < count;
        uint64_t k = 0;
        uint32_t val = 0, d = 0;
        if (valid) {
            k = kin[i];
            val = vin[i];
            d = (uint32_t)(k >> shift) & 255u;
        }
        // lanes of this wave holding the same digit
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = mask_rank(m);
        const uint32_t cnt = (uint32_t)__popcll(m);
#pragma unroll
        for (int k2 = 0; k2 < SORT_T / 64; ++k2) wc[k2][t] = 0;
        __syncthreads();
        if (valid && rank == 0) wc[w][d] = cnt;
        __syncthreads();
        {
            uint32_t acc = run[t];
#pragma unroll
            for (int k2 = 0; k2 < SORT_T / 64; ++k2) {
                const uint32_t c = wc[k2][t];
                wc[k2][t] = acc;
                acc += c;
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wc[w][d] + rank;
            kout[pos] = k;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

__global__ void k_ranges(const uint64_t* __restrict__ keys, const uint64_t* n_pairs, uint64_t capacity,
                         const uint32_t* overflow, uint32_t* __restrict__ ranges, int n_tiles) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*overflow) return;
    const uint64_t count = min(*n_pairs, capacity);
    if (k >= count) return;
    const uint32_t tile = (uint32_t)(keys[k] >> 32);
    if (tile >= (uint32_t)n_tiles) return;
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != tile) ranges[2 * tile] = (uint32_t)k;
    if (k + 1 == count || (uint32_t)(keys[k + 1] >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(k + 1);
}

// ---------------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SortLayout {
    size_t offs, scan1, keys_alt, vals_alt, hist, hist_off, scan2, total;
    int64_t nb_sort;
};

SortLayout sort_layout(int64_t n, int32_t n_views, uint64_t capacity) {
    SortLayout L;
    const int64_t vn = n * (int64_t)n_views;
    L.nb_sort = (int64_t)((capacity + SORT_ITEMS - 1) / SORT_ITEMS);
    size_t p = 0;
    L.offs = p;
    p = align256(p + sizeof(uint32_t) * (size_t)vn);
    L.scan1 = p;
    p = align256(p + sizeof(uint64_t) * 2 * (size_t)scan_blocks(vn));
    L.keys_alt = p;
    p = align256(p + sizeof(uint64_t) * (size_t)capacity);
    L.vals_alt = p;
    p = align256(p + sizeof(uint32_t) * (size_t)capacity);
    L.hist = p;
    p = align256(p + sizeof(uint32_t) * 256 * (size_t)L.nb_sort);
    L.hist_off = p;
    p = align256(p + sizeof(uint32_t) * 256 * (size_t)L.nb_sort);
    L.scan2 = p;
    p = align256(p + sizeof(uint64_t) * 2 * (size_t)scan_blocks(256 * L.nb_sort));
    L.total = p;
    return L;
}

size_t sort_workspace_bytes(int64_t n, int32_t n_views, uint64_t capacity) {
    return sort_layout(n, n_views, capacity).total;
}

int key_bits(int n_tiles) {
    int b = 0;
    while (b < 31 && (1u << b) < (uint32_t)n_tiles) ++b;
    return 32 + b;
}

gs_status launch_bin_sort(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* ws,
                          hipStream_t stream) {
    const int64_t n = proj->n;
    const int64_t vn = n * (int64_t)views->n_views;
    SortLayout L = sort_layout(n, views->n_views, bins->capacity);
    char* w = (char*)ws;
    uint32_t* offs = (uint32_t*)(w + L.offs);
    uint64_t* scan1 = (uint64_t*)(w + L.scan1);
    uint64_t* kalt = (uint64_t*)(w + L.keys_alt);
    uint32_t* valt = (uint32_t*)(w + L.vals_alt);
    uint32_t* hist = (uint32_t*)(w + L.hist);
    uint32_t* hist_off = (uint32_t*)(w + L.hist_off);
    uint64_t* scan2 = (uint64_t*)(w + L.scan2);

    // ranges start empty: [0, 0) for every tile
    hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, stream, bins->ranges, 2 * (int64_t)views->n_tiles, 0u);
    if (vn == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, bins->overflow, (int64_t)1, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)bins->n_pairs, (int64_t)2, 0u);
        return check_launch("bin_sort(empty)");
    }
    gs_status st = launch_scan(proj->count, offs, vn, scan1, bins->n_pairs, bins->overflow, bins->capacity, stream);
    if (st != GS_OK) return st;
    const int bits = key_bits(views->n_tiles);
    const int passes = (bits + 7) / 8;
    // with an even number of passes the result lands where the keys were emitted
    uint64_t* k0 = (passes % 2 == 0) ? bins->keys : kalt;
    uint32_t* v0 = (passes % 2 == 0) ? bins->vals : valt;
    uint64_t* k1 = (passes % 2 == 0) ? kalt : bins->keys;
    uint32_t* v1 = (passes % 2 == 0) ? valt : bins->vals;
    EmitArgs e;
    e.count = proj->count;
    e.offs = offs;
    e.rect = proj->rect;
    e.depth = proj->depth;
    e.cams = views->cams;
    e.tile_offset = views->tile_offset;
    e.n = n;
    e.tile_w = views->tile_w;
    e.overflow = bins->overflow;
    e.capacity = bins->capacity;
    e.keys = k0;
    e.vals = v0;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((n + 255) / 256), (unsigned)views->n_views), dim3(256), 0, stream, e);
    if (L.nb_sort > 0) {
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = pass * 8;
            hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)L.nb_sort), dim3(SORT_T), 0, stream, k0, bins->n_pairs,
                               bins->capacity, shift, hist, L.nb_sort);
            st = launch_scan(hist, hist_off, 256 * L.nb_sort, scan2, nullptr, nullptr, 0, stream);
            if (st != GS_OK) return st;
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)L.nb_sort), dim3(SORT_T), 0, stream, k0, v0, k1, v1,
                               bins->n_pairs, bins->capacity, shift, hist_off, L.nb_sort);
            uint64_t* tk = k0;
            k0 = k1;
            k1 = tk;
            uint32_t* tv = v0;
            v0 = v1;
            v1 = tv;
        }
        const unsigned g = (unsigned)((bins->capacity + 255) / 256);
        hipLaunchKernelGGL(k_ranges, dim3(g), dim3(256), 0, stream, bins->keys, bins->n_pairs, bins->capacity,
                           bins->overflow, bins->ranges, views->n_tiles);
    }
    return check_launch("bin_sort");
}

// ---------------------------------------------------------------------------------------
// Bitset -> sorted index list
// ---------------------------------------------------------------------------------------
__global__ void k_popc(const uint32_t* __restrict__ bits, int64_t n, uint32_t* __restrict__ cnt) {
    const int64_t wd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words = (n + 31) / 32;
    if (wd >= words) return;
    uint32_t b = bits[wd];
    const int64_t rem = n - wd * 32;
    if (rem < 32) b &= (1u << rem) - 1u;
    cnt[wd] = __popc(b);
}

__global__ void k_list(const uint32_t* __restrict__ bits, int64_t n, const uint32_t* __restrict__ offs,
                       int32_t* __restrict__ list) {
    const int64_t wd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words = (n + 31) / 32;
    if (wd >= words) return;
    uint32_t b = bits[wd];
    const int64_t rem = n - wd * 32;
    if (rem < 32) b &= (1u << rem) - 1u;
    uint32_t o = offs[wd];
    while (b) {
        const int k = __ffs(b) - 1;
        list[o++] = (int32_t)(wd * 32 + k);
        b &= b - 1u;
    }
}

size_t list_workspace_bytes(int64_t n) {
    const int64_t words = (n + 31) / 32;
    return align256(sizeof(uint32_t) * 2 * (size_t)words) + align256(sizeof(uint64_t) * 2 * (size_t)scan_blocks(words));
}

gs_status launch_bits_to_list(const uint32_t* bits, int64_t n, int32_t* list, int64_t* count, void* ws,
                              hipStream_t stream) {
    const int64_t words = (n + 31) / 32;
    char* w = (char*)ws;
    uint32_t* cnt = (uint32_t*)w;
    uint32_t* offs = cnt + words;
    uint64_t* scan = (uint64_t*)(w + align256(sizeof(uint32_t) * 2 * (size_t)words));
    if (words == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, (uint32_t*)count, (int64_t)2, 0u);
        return check_launch("bits_to_list(empty)");
    }
    const unsigned g = (unsigned)((words + 255) / 256);
    hipLaunchKernelGGL(k_popc, dim3(g), dim3(256), 0, stream, bits, n, cnt);
    gs_status st = launch_scan(cnt, offs, words, scan, (uint64_t*)count, nullptr, 0, stream);
    if (st != GS_OK) return st;
    hipLaunchKernelGGL(k_list, dim3(g), dim3(256), 0, stream, bits, n, offs, list);
    return check_launch("bits_to_list");
}

gs_status launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t stream) {
    if (n <= 0) return GS_OK;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, stream, p, n, value);
    return check_launch("fill");
}

gs_status launch_fill_f32(float* p, int64_t n, float value, hipStream_t stream) {
    if (n <= 0) return GS_OK;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)g), dim3(256), 0, stream, p, n, value);
    return check_launch("fill");
}

}  // namespace gs
