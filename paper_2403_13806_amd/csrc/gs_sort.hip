// Tile binning and the (tile, depth, index) sort that gives every tile its
// front-to-back list ("correctly-sorted points", eq. render-gs):
//   scan     exclusive prefix sum of the per-(view, Gaussian) tile counts in one pass:
//            4096 items per block, wave DPP scan -> block scan -> decoupled look-back
//            across blocks in launch-ticket order; the last block writes the pair total
//            and the capacity check
//   emit     load-balanced: the pairs of a wave's 64 Gaussians are contiguous in the
//            output, so lanes walk that range 64 pairs at a time and find their
//            Gaussian by a 6-step binary search over the wave's offsets in LDS; keys
//            (global tile << 32 | FP32 depth bits) are written coalesced, in index order,
//            so a stable sort breaks depth ties by index
//   sort     onesweep LSD radix sort, 8-bit digits over the significant key bits: one
//            kernel builds the global digit histograms of all passes, then one kernel per
//            pass ranks its 4096 items stably (8 ballots per wave), resolves the digit
//            offsets of earlier blocks by decoupled look-back, and scatters through LDS
//            so that global writes are coalesced runs
//   ranges   [start, end) of every tile in the sorted list
// Every wait on another block is bounded: a wait that exceeds its spin budget sets bit 1
// of the overflow word (results invalid) instead of hanging.
#include <algorithm>

#include "gs_device.hpp"

namespace gs {

constexpr int BLK = 256;                 // threads per scan / sort block
constexpr int IPT = 16;                  // items per thread
constexpr int TILE_ITEMS = BLK * IPT;    // items per block
constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr int MAX_PASSES = 8;

// chained-scan status word: flag in the two top bits, value below
constexpr uint64_t ST_AGG = 1ull << 62;
constexpr uint64_t ST_PRE = 2ull << 62;
constexpr uint64_t ST_VAL = (1ull << 62) - 1;

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// zero up to four buffers in one launch
struct Fill4 {
    uint32_t* p[4];
    int64_t n[4];
};

__global__ void k_zero4(Fill4 f) {
    const int s = blockIdx.y;
    uint32_t* p = f.p[s];
    const int64_t n = f.n[s];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

gs_status launch_zero4(const Fill4& f, hipStream_t stream) {
    int64_t mx = 1;
    for (int k = 0; k < 4; ++k) mx = std::max(mx, f.n[k]);
    const int64_t g = std::min<int64_t>((mx + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero4, dim3((unsigned)g, 4), dim3(256), 0, stream, f);
    return check_launch("zero");
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

__device__ __forceinline__ uint64_t ld_status(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the values published by blocks 0..bid-1 of one chain (entries `stride` apart),
// walking back until an inclusive prefix is found. WIN predecessors are loaded at once so
// the walk pays one memory latency per WIN blocks. Bounded: on timeout it sets bit 1 of
// *err and returns what it has.
template <int WIN>
__device__ uint64_t lookback(const uint64_t* chain, int64_t stride, uint32_t bid, uint32_t* err) {
    uint64_t excl = 0;
    int64_t j = (int64_t)bid - 1;
    uint32_t spins = 0;
    while (j >= 0) {
        uint64_t s[WIN];
#pragma unroll
        for (int k = 0; k < WIN; ++k) s[k] = (j - k >= 0) ? ld_status(chain + (j - k) * stride) : ST_PRE;
        int used = 0;
        bool found = false, stalled = false;
#pragma unroll
        for (int k = 0; k < WIN; ++k) {
            if (found || stalled) continue;
            const uint64_t f = s[k] & ~ST_VAL;
            if (f == 0) {
                stalled = true;
                continue;
            }
            if (j - k >= 0) excl += s[k] & ST_VAL;
            ++used;
            if (f == ST_PRE) found = true;
        }
        if (found) break;
        j -= used;
        if (stalled) {
            if (++spins > SPIN_LIMIT) {
                if (err) atomicOr(err, 2u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
}

// block-wide exclusive scan of one u32 per thread (256 threads); returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, uint32_t* wsum) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t incl = wave_incl_scan(x);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLK / 64; ++k) {
        const uint32_t s = wsum[k];
        pre += (k < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + incl - x;
}

// ---------------------------------------------------------------------------------------
// Single-pass exclusive scan of u32 values (decoupled look-back).
// status[nblocks] and *ticket must be zero on entry; *flags must be zero when used.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(BLK) void k_chained_scan(const uint32_t* __restrict__ in, int64_t n,
                                                      uint32_t* __restrict__ out, uint64_t* status, uint32_t* ticket,
                                                      int64_t nblocks, uint64_t* total_out, uint32_t* flags,
                                                      uint64_t capacity) {
    __shared__ uint32_t wsum[BLK / 64];
    __shared__ uint32_t bid_s;
    __shared__ uint64_t pre_s;
    const int t = threadIdx.x;
    if (t == 0) bid_s = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t bid = bid_s;
    const int64_t base = (int64_t)bid * TILE_ITEMS + (int64_t)t * IPT;
    uint32_t x[IPT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        x[k] = (base + k < n) ? in[base + k] : 0u;
        s += x[k];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(s, tot, wsum);
    if (t == 0) {
        uint64_t pre = 0;
        if (bid == 0) {
            st_status(status, ST_PRE | tot);
        } else {
            st_status(status + bid, ST_AGG | tot);
            pre = lookback<8>(status, 1, bid, flags);
            st_status(status + bid, ST_PRE | (pre + tot));
        }
        pre_s = pre;
        if ((int64_t)bid == nblocks - 1) {
            const uint64_t total = pre + tot;
            if (total_out) *total_out = total;
            if (flags && total > capacity) atomicOr(flags, 1u);
        }
    }
    __syncthreads();
    // offsets past 2^32 only occur when the capacity check has already failed
    uint32_t run = (uint32_t)pre_s + ex;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        if (base + k < n) out[base + k] = run;
        run += x[k];
    }
}

int64_t scan_blocks(int64_t n) { return (n + TILE_ITEMS - 1) / TILE_ITEMS; }

// exclusive scan; ctrl = (zeroed) status[scan_blocks(n)] followed by a ticket word
gs_status launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint64_t* ctrl, uint64_t* total,
                      uint32_t* flags, uint64_t capacity, hipStream_t stream) {
    if (n <= 0) return GS_OK;
    const int64_t nb = scan_blocks(n);
    uint32_t* ticket = (uint32_t*)(ctrl + nb);
    hipLaunchKernelGGL(k_chained_scan, dim3((unsigned)nb), dim3(BLK), 0, stream, in, n, out, ctrl, ticket, nb, total,
                       flags, capacity);
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
    __shared__ uint32_t s_off[256], s_db[256];
    __shared__ uint64_t s_rect[256];
    const int v = blockIdx.y, t = threadIdx.x, w = t >> 6, l = t & 63;
    if (*a.overflow) return;  // the same for every thread
    const int64_t j0 = (int64_t)blockIdx.x * 256 + w * 64;  // first Gaussian of this wave
    const int64_t j = j0 + l;
    const int64_t o = (int64_t)v * a.n + j;
    uint32_t c = 0, off = 0xffffffffu, db = 0;
    uint64_t r = 0;
    if (j < a.n) {
        off = a.offs[o];
        c = a.count[o];
        if (c) {
            r = a.rect[o];
            db = __float_as_uint(a.depth[o]);
        }
    }
    s_off[t] = off;
    s_db[t] = db;
    s_rect[t] = r;
    __syncthreads();
    if (j0 >= a.n) return;
    // the wave's pairs occupy [first offset, last offset + last count)
    const int last = (int)min((int64_t)63, a.n - 1 - j0);
    const uint32_t* wo = s_off + w * 64;
    const uint32_t g0 = wo[0];
    const uint32_t ge = wave_read(off + c, last);
    const uint32_t tiles_x = (uint32_t)div_up(a.cams[v].width, a.tile_w);
    const uint32_t tbase = (uint32_t)a.tile_offset[v];
    for (uint32_t g = g0 + l; g < ge; g += 64) {
        // largest lane L with wo[L] <= g (lanes with no pairs share the next lane's offset)
        int L = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (L + step <= last && wo[L + step] <= g) L += step;
        const uint64_t rr = s_rect[w * 64 + L];
        const uint32_t x0 = rr & 0xffff, y0 = (rr >> 16) & 0xffff, x1 = (rr >> 32) & 0xffff;
        const uint32_t wd = x1 - x0 + 1;
        const uint32_t k = g - wo[L];
        const uint32_t ty = y0 + k / wd, tx = x0 + k % wd;
        a.keys[g] = ((uint64_t)(tbase + ty * tiles_x + tx) << 32) | s_db[w * 64 + L];
        a.vals[g] = (uint32_t)(j0 + L);
    }
}

// ---------------------------------------------------------------------------------------
// Onesweep radix sort
// ---------------------------------------------------------------------------------------
// global digit histograms of every pass (ghist [passes][256], zero on entry). Each thread
// reads a contiguous run of keys; consecutive keys mostly come from one Gaussian (same
// depth digits) or neighbouring tiles (same high tile digits), so equal digits are merged
// in registers and one LDS atomic is issued per run.
constexpr int HIST_RUN = 16;

__global__ __launch_bounds__(256) void k_os_hist(const uint64_t* __restrict__ keys, const uint64_t* n_pairs,
                                                 uint64_t capacity, int passes, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[MAX_PASSES][256];
    const int t = threadIdx.x;
    for (int p = 0; p < MAX_PASSES; ++p) h[p][t] = 0;
    __syncthreads();
    const uint64_t count = min(*n_pairs, capacity);
    const uint64_t stride = (uint64_t)gridDim.x * BLK * HIST_RUN;
    for (uint64_t b0 = ((uint64_t)blockIdx.x * BLK + t) * HIST_RUN; b0 < count; b0 += stride) {
        const uint64_t b1 = min(b0 + HIST_RUN, count);
        uint64_t prev = keys[b0];
        uint32_t cnt[MAX_PASSES];
#pragma unroll
        for (int p = 0; p < MAX_PASSES; ++p) cnt[p] = 1;
        for (uint64_t i = b0 + 1; i < b1; ++i) {
            const uint64_t k = keys[i];
#pragma unroll
            for (int p = 0; p < MAX_PASSES; ++p) {
                if (p >= passes) continue;
                const uint32_t dp = (uint32_t)(prev >> (8 * p)) & 255u, dk = (uint32_t)(k >> (8 * p)) & 255u;
                if (dp == dk) {
                    ++cnt[p];
                } else {
                    atomicAdd(&h[p][dp], cnt[p]);
                    cnt[p] = 1;
                }
            }
            prev = k;
        }
#pragma unroll
        for (int p = 0; p < MAX_PASSES; ++p)
            if (p < passes) atomicAdd(&h[p][(uint32_t)(prev >> (8 * p)) & 255u], cnt[p]);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (h[p][t]) atomicAdd(&ghist[p * 256 + t], h[p][t]);
}

struct PassArgs {
    const uint64_t* kin;
    const uint32_t* vin;
    uint64_t* kout;
    uint32_t* vout;
    const uint64_t* n_pairs;
    uint64_t capacity;
    int shift;
    const uint32_t* ghist;  // this pass's 256 digit counts
    uint64_t* status;       // [nblocks][256], zero on entry
    uint32_t* ticket;       // zero on entry
    uint32_t* err;
};

// Each wave ranks its own contiguous 64*IPT items with wave-private digit counters (no
// block barrier inside the ranking loop); wave offsets per digit are combined once.
__global__ __launch_bounds__(BLK) void k_os_pass(PassArgs a) {
    __shared__ uint32_t bid_s;
    __shared__ uint32_t wcnt[BLK / 64][256];
    __shared__ uint32_t ds[256];
    __shared__ int64_t dbase[256];
    __shared__ uint32_t wsum[BLK / 64];
    __shared__ uint64_t lk[TILE_ITEMS];
    __shared__ uint32_t lv[TILE_ITEMS];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (t == 0) bid_s = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const uint32_t bid = bid_s;
    const uint64_t count = min(*a.n_pairs, a.capacity);
    const uint64_t base = (uint64_t)bid * TILE_ITEMS;
    if (base >= count) return;  // blocks past the data; no block waits on them
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[w][l + 64 * k] = 0;
    const uint64_t wbase = base + (uint64_t)w * (64 * IPT);
    uint64_t key[IPT];
    uint32_t val[IPT], lr[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t i = wbase + r * 64 + l;
        const bool valid = i < count;
        key[r] = valid ? a.kin[i] : 0ull;
        val[r] = valid ? a.vin[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = wbase + r * 64 + l < count;
        const uint32_t d = (uint32_t)(key[r] >> a.shift) & 255u;
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = mask_rank(m);
        const uint32_t old = valid ? wcnt[w][d] : 0u;
        lr[r] = old + rank;
        if (valid && rank == 0) wcnt[w][d] = old + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // digit t: exclusive offsets of the waves (in place) and the block total
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < BLK / 64; ++k) {
        const uint32_t c = wcnt[k][t];
        wcnt[k][t] = mine;
        mine += c;
    }
    uint32_t tot;
    const uint32_t dstart = block_excl_scan(mine, tot, wsum);
    uint32_t gtot;
    const uint32_t gstart = block_excl_scan(a.ghist[t], gtot, wsum);
    ds[t] = dstart;
    // digits of earlier blocks: decoupled look-back, one chain per digit. The status table is
    // [block][digit] so that a wave's publish and each look-back load are 512-byte runs.
    uint64_t* st = a.status + (uint64_t)bid * 256 + t;
    uint64_t excl = 0;
    if (bid == 0) {
        st_status(st, ST_PRE | mine);
    } else {
        st_status(st, ST_AGG | mine);
        excl = lookback<4>(a.status + t, 256, bid, a.err);
        st_status(st, ST_PRE | (excl + mine));
    }
    dbase[t] = (int64_t)gstart + (int64_t)excl - (int64_t)dstart;
    __syncthreads();
    // block-local sort through LDS
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wbase + r * 64 + l < count) {
            const uint32_t d = (uint32_t)(key[r] >> a.shift) & 255u;
            const uint32_t q = ds[d] + wcnt[w][d] + lr[r];
            lk[q] = key[r];
            lv[q] = val[r];
        }
    }
    __syncthreads();
    const uint32_t nitems = (uint32_t)min((uint64_t)TILE_ITEMS, count - base);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t q = r * BLK + t;
        if (q < nitems) {
            const uint64_t k = lk[q];
            const uint32_t d = (uint32_t)(k >> a.shift) & 255u;
            const int64_t pos = dbase[d] + (int64_t)q;
            if (pos >= 0 && (uint64_t)pos < count) {  // always true unless a look-back timed out
                a.kout[pos] = k;
                a.vout[pos] = lv[q];
            }
        }
    }
}

__global__ void k_iota(uint32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
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
// Longest-first tile order for the persistent compositing launch: tiles are bucketed by
// bit length of their list size (33 buckets) and laid out from the longest bucket down.
// ---------------------------------------------------------------------------------------
constexpr int LPT_B = 33;

__device__ __forceinline__ int lpt_bucket(const uint32_t* ranges, int tile) {
    const uint32_t c = ranges[2 * tile + 1] - ranges[2 * tile];
    return c ? 32 - __clz(c) : 0;
}

__global__ __launch_bounds__(256) void k_lpt_hist(const uint32_t* __restrict__ ranges, int n_tiles,
                                                  uint32_t* __restrict__ bh) {
    __shared__ uint32_t lh[LPT_B];
    const int t = threadIdx.x;
    if (t < LPT_B) lh[t] = 0;
    __syncthreads();
    for (int i = blockIdx.x * 256 + t; i < n_tiles; i += gridDim.x * 256) atomicAdd(&lh[lpt_bucket(ranges, i)], 1u);
    __syncthreads();
    if (t < LPT_B && lh[t]) atomicAdd(&bh[t], lh[t]);
}

__global__ __launch_bounds__(256) void k_lpt_scatter(const uint32_t* __restrict__ ranges, int n_tiles,
                                                     const uint32_t* __restrict__ bh, uint32_t* __restrict__ fill,
                                                     uint32_t* __restrict__ queue) {
    __shared__ uint32_t lh[LPT_B], lbase[LPT_B], goff[LPT_B];
    const int t = threadIdx.x;
    if (t == 0) {
        uint32_t acc = 0;
        for (int b = LPT_B - 1; b >= 0; --b) {
            goff[b] = acc;
            acc += bh[b];
        }
    }
    if (t < LPT_B) lh[t] = 0;
    __syncthreads();
    const int i = blockIdx.x * 256 + t;
    int b = 0;
    uint32_t lr = 0;
    if (i < n_tiles) {
        b = lpt_bucket(ranges, i);
        lr = atomicAdd(&lh[b], 1u);
    }
    __syncthreads();
    if (t < LPT_B) lbase[t] = lh[t] ? atomicAdd(&fill[t], lh[t]) : 0u;
    __syncthreads();
    if (i < n_tiles) {
        const uint32_t pos = goff[b] + lbase[b] + lr;
        if (pos < (uint32_t)n_tiles) queue[pos] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int key_bits(int n_tiles) {
    int b = 0;
    while (b < 31 && (1u << b) < (uint32_t)n_tiles) ++b;
    return 32 + b;
}

struct SortLayout {
    size_t offs, ctrl, scan_ctrl, tickets, ghist, lpt, status, ctrl_end, keys_alt, vals_alt, total;
    int64_t nb_sort, nb_scan;
    int passes;
};

SortLayout sort_layout(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles) {
    SortLayout L;
    const int64_t vn = n * (int64_t)n_views;
    L.nb_sort = (int64_t)((capacity + TILE_ITEMS - 1) / TILE_ITEMS);
    L.nb_scan = scan_blocks(vn);
    L.passes = (key_bits(std::max(n_tiles, 1)) + 7) / 8;
    size_t p = 0;
    L.offs = p;
    p = align256(p + sizeof(uint32_t) * (size_t)vn);
    // control block, cleared at the start of every gs_bin_sort
    L.ctrl = p;
    L.scan_ctrl = p;
    p = align256(p + sizeof(uint64_t) * ((size_t)L.nb_scan + 1));
    L.tickets = p;
    p = align256(p + sizeof(uint32_t) * MAX_PASSES);
    L.ghist = p;
    p = align256(p + sizeof(uint32_t) * 256 * MAX_PASSES);
    L.lpt = p;
    p = align256(p + sizeof(uint32_t) * 2 * LPT_B);
    L.status = p;
    p = align256(p + sizeof(uint64_t) * 256 * (size_t)L.nb_sort * (size_t)L.passes);
    L.ctrl_end = p;
    L.keys_alt = p;
    p = align256(p + sizeof(uint64_t) * (size_t)capacity);
    L.vals_alt = p;
    p = align256(p + sizeof(uint32_t) * (size_t)capacity);
    L.total = p;
    return L;
}

size_t sort_workspace_bytes(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles) {
    return sort_layout(n, n_views, capacity, n_tiles).total;
}

// tile work order (only when the caller asked for one); lpt = zeroed [2][LPT_B] counters,
// or NULL when there are no pairs at all (then the identity order is as good as any)
static gs_status launch_lpt(const gs_views* views, gs_bins* bins, uint32_t* lpt, hipStream_t stream) {
    if (!bins->queue || views->n_tiles == 0) return check_launch("bin_sort");
    const unsigned g = (unsigned)((views->n_tiles + 255) / 256);
    if (!lpt) {
        hipLaunchKernelGGL(k_iota, dim3(g), dim3(256), 0, stream, bins->queue, views->n_tiles);
        return check_launch("bin_sort");
    }
    hipLaunchKernelGGL(k_lpt_hist, dim3(std::min(g, 1024u)), dim3(256), 0, stream, bins->ranges, views->n_tiles, lpt);
    hipLaunchKernelGGL(k_lpt_scatter, dim3(g), dim3(256), 0, stream, bins->ranges, views->n_tiles, lpt, lpt + LPT_B,
                       bins->queue);
    return check_launch("bin_sort");
}

gs_status launch_bin_sort(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* ws,
                          hipStream_t stream) {
    const int64_t n = proj->n;
    const int64_t vn = n * (int64_t)views->n_views;
    SortLayout L = sort_layout(n, views->n_views, bins->capacity, views->n_tiles);
    char* w = (char*)ws;
    uint32_t* offs = (uint32_t*)(w + L.offs);
    uint64_t* scan_ctrl = (uint64_t*)(w + L.scan_ctrl);
    uint32_t* tickets = (uint32_t*)(w + L.tickets);
    uint32_t* ghist = (uint32_t*)(w + L.ghist);
    uint64_t* status = (uint64_t*)(w + L.status);
    uint64_t* kalt = (uint64_t*)(w + L.keys_alt);
    uint32_t* valt = (uint32_t*)(w + L.vals_alt);

    // ranges start empty; flags, pair count and the control block start at zero
    gs_status st;
    Fill4 f;
    f.p[0] = bins->ranges;
    f.n[0] = 2 * (int64_t)views->n_tiles;
    f.p[1] = bins->overflow;
    f.n[1] = 1;
    f.p[2] = (uint32_t*)bins->n_pairs;
    f.n[2] = 2;
    f.p[3] = (uint32_t*)(w + L.ctrl);
    f.n[3] = vn == 0 ? 0 : (int64_t)((L.ctrl_end - L.ctrl) / 4);
    if ((st = launch_zero4(f, stream))) return st;
    if (vn == 0) return launch_lpt(views, bins, nullptr, stream);
    if ((st = launch_scan(proj->count, offs, vn, scan_ctrl, bins->n_pairs, bins->overflow, bins->capacity, stream)))
        return st;
    const int passes = L.passes;
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
    if (L.nb_sort == 0) return launch_lpt(views, bins, (uint32_t*)(w + L.lpt), stream);
    const unsigned hist_blocks = (unsigned)std::min<int64_t>(L.nb_sort * 4, 1024);
    hipLaunchKernelGGL(k_os_hist, dim3(hist_blocks), dim3(BLK), 0, stream, k0, bins->n_pairs, bins->capacity, passes,
                       ghist);
    for (int pass = 0; pass < passes; ++pass) {
        PassArgs pa;
        pa.kin = k0;
        pa.vin = v0;
        pa.kout = k1;
        pa.vout = v1;
        pa.n_pairs = bins->n_pairs;
        pa.capacity = bins->capacity;
        pa.shift = 8 * pass;
        pa.ghist = ghist + 256 * pass;
        pa.status = status + (size_t)256 * L.nb_sort * pass;
        pa.ticket = tickets + pass;
        pa.err = bins->overflow;
        hipLaunchKernelGGL(k_os_pass, dim3((unsigned)L.nb_sort), dim3(BLK), 0, stream, pa);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    const unsigned g = (unsigned)((bins->capacity + 255) / 256);
    hipLaunchKernelGGL(k_ranges, dim3(g), dim3(256), 0, stream, bins->keys, bins->n_pairs, bins->capacity,
                       bins->overflow, bins->ranges, views->n_tiles);
    return launch_lpt(views, bins, (uint32_t*)(w + L.lpt), stream);
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
    return align256(sizeof(uint32_t) * 2 * (size_t)words) + align256(sizeof(uint64_t) * ((size_t)scan_blocks(words) + 1));
}

gs_status launch_bits_to_list(const uint32_t* bits, int64_t n, int32_t* list, int64_t* count, void* ws,
                              hipStream_t stream) {
    const int64_t words = (n + 31) / 32;
    char* w = (char*)ws;
    uint32_t* cnt = (uint32_t*)w;
    uint32_t* offs = cnt + words;
    uint64_t* ctrl = (uint64_t*)(w + align256(sizeof(uint32_t) * 2 * (size_t)words));
    gs_status st;
    if ((st = launch_fill_u32((uint32_t*)count, 2, 0u, stream))) return st;
    if (words == 0) return GS_OK;
    if ((st = launch_fill_u32((uint32_t*)ctrl, 2 * (scan_blocks(words) + 1), 0u, stream))) return st;
    const unsigned g = (unsigned)((words + 255) / 256);
    hipLaunchKernelGGL(k_popc, dim3(g), dim3(256), 0, stream, bits, n, cnt);
    if ((st = launch_scan(cnt, offs, words, ctrl, (uint64_t*)count, nullptr, 0, stream))) return st;
    hipLaunchKernelGGL(k_list, dim3(g), dim3(256), 0, stream, bits, n, offs, list);
    return check_launch("bits_to_list");
}

}  // namespace gs
