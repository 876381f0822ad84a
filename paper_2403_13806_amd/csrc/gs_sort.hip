// Tile binning and the (tile, depth, index) order that gives every tile its front-to-back
// list ("correctly-sorted points", eq. render-gs):
//   offsets  exclusive prefix sum of the per-(view, Gaussian) tile counts in two levels:
//            sums of 256-entry blocks, one workgroup scanning those (it writes the pair
//            total and the capacity check), and the scan inside each block during emission
//   walk     load-balanced: the pairs of a wave's 64 Gaussians are numbered in entry order,
//            lanes take them 64 at a time and find their Gaussian by a 6-step binary search
//            over the wave's offsets in LDS; each pair is a global tile id and FP32 depth
//            bits << 32 | Gaussian index
//   group    at most 4096 tiles: every row of 4096 entries counts its pairs per tile in LDS,
//            column scans give each row's start inside every tile's range, and a second walk
//            writes each pair straight into its tile's range (slots from LDS counters).
//            Beyond: the pairs are written in entry order and grouped by onesweep LSD radix
//            passes on the tile id (ceil(tile bits / 8) passes of 8 bits: one kernel builds the
//            digit histograms of all passes, then one kernel per pass ranks its 4096 items
//            with 8 ballots per wave, resolves the digit offsets of earlier blocks by
//            decoupled look-back, and scatters through LDS into coalesced runs)
//   ranges   [start, end) of every tile in the grouped list
//   sort     one workgroup per tile orders the tile's list by its unique 64-bit (depth bits,
//            index) values in LDS (radix passes on the depth bits, or a bitonic network when
//            depths repeat, so the result does not depend on the order the grouping left) and
//            writes the keys (tile << 32 | depth bits) and the Gaussian indices; a list longer
//            than the LDS buffer is sorted by the same workgroup in chunks of that size, merged
//            (merge path) back and forth through a scratch buffer
// Every wait on another block is bounded: a wait that exceeds its spin budget sets bit 1
// of the overflow word (results invalid) instead of hanging.
#include <algorithm>

#include "gs_device.hpp"
#include "gs_tile_sort.hpp"

namespace gs {

constexpr int BLK = 256;                 // threads per scan / sort block
constexpr int IPT = 16;                  // items per thread
constexpr int TILE_ITEMS = BLK * IPT;    // items per block
constexpr uint32_t SPIN_LIMIT = 1u << 22;

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
// Pair emission
// ---------------------------------------------------------------------------------------
// Pair offsets in entry order (view-major, then Gaussian) come in two levels: the tile counts
// of every 256-entry emission block are summed (k_count_bsums), one workgroup scans those block
// sums (k_scan_bsums: the block prefixes, the pair total and the capacity check), and each
// emission block scans its own 256 counts. No chain of waits between blocks.
constexpr int SB_T = 1024;  // threads of the block-sum scan

// It also clears the frame's state first (the job of k_zero4 when there is no pair to bin):
// no later kernel of the frame runs before it ends.
__global__ __launch_bounds__(256) void k_count_bsums(const uint32_t* __restrict__ count, int64_t n, int64_t nbv,
                                                     uint32_t* __restrict__ bsum, Fill4 clear) {
    {
        const int64_t tid = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        const int64_t nth = (int64_t)gridDim.x * gridDim.y * blockDim.x;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            for (int64_t i = tid; i < clear.n[b]; i += nth) clear.p[b][i] = 0u;
    }
    const int v = blockIdx.y, w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint32_t* cv = count + (int64_t)v * n;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t bx = (int64_t)blockIdx.x * 16 + w * 4 + q;  // emission block of this wave
        if (bx >= nbv) break;                                     // the same for the whole wave
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j = bx * 256 + k * 64 + l;
            sum += j < n ? cv[j] : 0u;
        }
        sum = wave_read(wave_incl_scan(sum), 63);
        if (l == 0) bsum[(int64_t)v * nbv + bx] = sum;
    }
}

// one workgroup scans the block sums in chunks of SB_T * 4 (coalesced loads, the next chunk
// requested before the current one is scanned) with a running carry
__global__ __launch_bounds__(SB_T) void k_scan_bsums(uint32_t* __restrict__ bsum, int64_t m, uint64_t* total_out,
                                                     uint32_t* flags, uint64_t capacity, uint32_t* sticky) {
    constexpr int CH = SB_T * 4;
    __shared__ uint64_t part[SB_T / 64 + 1];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint64_t carry = 0;
    uint32_t nx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nx[k] = (int64_t)4 * t + k < m ? bsum[4 * t + k] : 0u;
    for (int64_t base = 0; base < m; base += CH) {
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = nx[k];
        const int64_t nb = base + CH;
#pragma unroll
        for (int k = 0; k < 4; ++k) nx[k] = nb + 4 * t + k < m ? bsum[nb + 4 * t + k] : 0u;
        const uint64_t s = (uint64_t)x[0] + x[1] + x[2] + x[3];
        // inclusive scan of the per-thread sums over the wave, then over the waves
        uint64_t incl = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = (uint64_t)__shfl_up((long long)incl, d);
            if (l >= d) incl += y;
        }
        if (l == 63) part[w] = incl;
        __syncthreads();
        if (t == 0) {
            uint64_t run = 0;
            for (int k = 0; k < SB_T / 64; ++k) {
                const uint64_t v = part[k];
                part[k] = run;
                run += v;
            }
            part[SB_T / 64] = run;
        }
        __syncthreads();
        // offsets past 2^32 only occur when the capacity check below has failed
        uint64_t pre = carry + part[w] + incl - s;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (base + 4 * t + k < m) bsum[base + 4 * t + k] = (uint32_t)pre;
            pre += x[k];
        }
        carry += part[SB_T / 64];
        __syncthreads();  // part is rewritten by the next chunk
    }
    if (t == 0) {
        if (total_out) *total_out = carry;
        if (flags && carry > capacity) {
            atomicOr(flags, 1u);
            if (sticky) atomicOr(sticky, 1u);
        }
    }
}

struct EmitArgs {
    const uint32_t* count;
    const uint32_t* bpre;  // exclusive pair offset of each 256-entry emission block
    const uint64_t* rect;
    const float* depth;
    const gs_camera* cams;
    const int32_t* tile_offset;
    int64_t n;             // Gaussians per view
    int tile_w;
    const uint32_t* overflow;
    uint32_t* tkey;        // global tile of each pair
    uint64_t* tval;        // FP32 depth bits << 32 | Gaussian index
    uint32_t* eoff;        // [n_views * n] first pair of each entry, or NULL
};

__global__ __launch_bounds__(256) void k_emit(EmitArgs a) {
    __shared__ uint32_t s_off[256], s_db[256], s_wsum[4];
    __shared__ uint64_t s_rect[256];
    __shared__ double s_inv[256];  // 1 / rectangle width
    const int v = blockIdx.y, t = threadIdx.x, w = t >> 6, l = t & 63;
    if (*a.overflow) return;  // the same for every thread
    const int64_t j0 = (int64_t)blockIdx.x * 256 + w * 64;  // first Gaussian of this wave
    const int64_t j = j0 + l;
    const int64_t o = (int64_t)v * a.n + j;
    uint32_t c = 0, off = 0xffffffffu, db = 0;
    uint64_t r = 0;
    if (j < a.n) {
        c = a.count[o];
        if (c) {
            r = a.rect[o];
            db = __float_as_uint(a.depth[o]);
        }
    }
    uint32_t btot;
    const uint32_t ex = block_excl_scan(c, btot, s_wsum);
    if (j < a.n) {
        off = a.bpre[(int64_t)v * gridDim.x + blockIdx.x] + ex;
        if (a.eoff) a.eoff[o] = off;
    }
    s_off[t] = off;
    s_db[t] = db;
    s_rect[t] = r;
    s_inv[t] = 1.0 / (double)((uint32_t)(r >> 32 & 0xffff) - (uint32_t)(r & 0xffff) + 1u);
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
        const int q = w * 64 + L;
        const uint64_t rr = s_rect[q];
        const uint32_t x0 = rr & 0xffff, y0 = (rr >> 16) & 0xffff, x1 = (rr >> 32) & 0xffff;
        const uint32_t wd = x1 - x0 + 1;
        const uint32_t k = g - wo[L];
        // k / wd through FP64 (exact to within one for k < 2^32), then corrected
        uint32_t ky = (uint32_t)((double)k * s_inv[q]);
        uint32_t kx = k - ky * wd;
        if ((int32_t)kx < 0) {
            --ky;
            kx += wd;
        } else if (kx >= wd) {
            ++ky;
            kx -= wd;
        }
        a.tkey[g] = tbase + (y0 + ky) * tiles_x + x0 + kx;
        a.tval[g] = ((uint64_t)s_db[q] << 32) | (uint32_t)(j0 + L);
    }
}

// ---------------------------------------------------------------------------------------
// Onesweep LSD radix sort of u32 tile keys carrying u64 values
// ---------------------------------------------------------------------------------------
// global digit histograms of every pass (ghist [passes][256], zero on entry). Each thread
// reads a contiguous run of keys; consecutive keys often share digits (pairs of one
// Gaussian lie in neighbouring tiles), so equal digits are merged in registers and one LDS
// atomic is issued per run.
constexpr int HIST_RUN = 16;
constexpr int KEY_PASSES = 4;

__global__ __launch_bounds__(256) void k_os_hist(const uint32_t* __restrict__ keys, const uint64_t* n_items,
                                                 uint64_t bound, int passes, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[KEY_PASSES][256];
    const int t = threadIdx.x;
    for (int p = 0; p < KEY_PASSES; ++p) h[p][t] = 0;
    __syncthreads();
    const uint64_t count = min(*n_items, bound);
    const uint64_t stride = (uint64_t)gridDim.x * BLK * HIST_RUN;
    for (uint64_t b0 = ((uint64_t)blockIdx.x * BLK + t) * HIST_RUN; b0 < count; b0 += stride) {
        const uint64_t b1 = min(b0 + HIST_RUN, count);
        uint32_t prev = keys[b0];
        uint32_t cnt[KEY_PASSES];
#pragma unroll
        for (int p = 0; p < KEY_PASSES; ++p) cnt[p] = 1;
        for (uint64_t i = b0 + 1; i < b1; ++i) {
            const uint32_t k = keys[i];
#pragma unroll
            for (int p = 0; p < KEY_PASSES; ++p) {
                if (p >= passes) continue;
                const uint32_t dp = (prev >> (8 * p)) & 255u, dk = (k >> (8 * p)) & 255u;
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
        for (int p = 0; p < KEY_PASSES; ++p)
            if (p < passes) atomicAdd(&h[p][(prev >> (8 * p)) & 255u], cnt[p]);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p)
        if (h[p][t]) atomicAdd(&ghist[p * 256 + t], h[p][t]);
}

struct PassArgs {
    const uint32_t* kin;
    const void* vin;  // V[]
    uint32_t* kout;
    void* vout;       // V[] (u32 in the last tile pass)
    const uint64_t* n_items;
    uint64_t bound;
    int shift;
    const uint32_t* ghist;  // this pass's 256 digit counts
    uint64_t* status;       // [nblocks][256], zero on entry
    uint32_t* ticket;       // zero on entry
    uint32_t* err;
};

// One stable counting pass on an 8-bit digit of u32 keys carrying values of type V. Each
// wave ranks its own contiguous 64*IPT items with wave-private digit counters (no block
// barrier inside the ranking loop); wave offsets per digit are combined once.
template <typename V>
__global__ __launch_bounds__(BLK) void k_os_pass(PassArgs a) {
    __shared__ uint32_t bid_s;
    __shared__ uint32_t wcnt[BLK / 64][256];
    __shared__ uint32_t ds[256];
    __shared__ int64_t dbase[256];
    __shared__ uint32_t wsum[BLK / 64];
    __shared__ uint32_t lk[TILE_ITEMS];
    __shared__ V lv[TILE_ITEMS];
    const V* vin = (const V*)a.vin;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (t == 0) bid_s = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const uint32_t bid = bid_s;
    const uint64_t count = min(*a.n_items, a.bound);
    const uint64_t base = (uint64_t)bid * TILE_ITEMS;
    if (base >= count) return;  // blocks past the data; no block waits on them
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[w][l + 64 * k] = 0;
    const uint64_t wbase = base + (uint64_t)w * (64 * IPT);
    uint32_t key[IPT], lr[IPT];
    V val[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint64_t i = wbase + r * 64 + l;
        const bool valid = i < count;
        key[r] = valid ? a.kin[i] : 0u;
        val[r] = valid ? vin[i] : (V)0;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = wbase + r * 64 + l < count;
        const uint32_t d = (key[r] >> a.shift) & 255u;
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
            const uint32_t d = (key[r] >> a.shift) & 255u;
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
            const uint32_t k = lk[q];
            const uint32_t d = (k >> a.shift) & 255u;
            const int64_t pos = dbase[d] + (int64_t)q;
            if (pos >= 0 && (uint64_t)pos < count) {  // always true unless a look-back timed out
                a.kout[pos] = k;
                ((V*)a.vout)[pos] = lv[q];
            }
        }
    }
}

__global__ void k_ranges(const uint32_t* __restrict__ tkeys, const uint64_t* n_pairs, uint64_t capacity,
                         const uint32_t* overflow, uint32_t* __restrict__ ranges, int n_tiles) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*overflow) return;
    const uint64_t count = min(*n_pairs, capacity);
    if (k >= count) return;
    const uint32_t tile = tkeys[k];
    if (tile >= (uint32_t)n_tiles) return;
    if (k == 0 || tkeys[k - 1] != tile) ranges[2 * tile] = (uint32_t)k;
    if (k + 1 == count || tkeys[k + 1] != tile) ranges[2 * tile + 1] = (uint32_t)(k + 1);
}

// ---------------------------------------------------------------------------------------
// Emission straight into tile buckets, for batches whose views have at most 8192 tiles each:
// the pairs are never written in entry order. Each row of 4096 entries (16 emission blocks of
// one view) builds its view's tile histogram in LDS by walking its entries' pairs
// (k_bucket_count, which also writes the emission blocks' pair sums); column scans over each
// view's rows give, per tile, the pairs of earlier rows, the tile's total, and each view's
// total (k_bucket_colscan); then each row walks its pairs again and writes each one at tile
// start + earlier rows' pairs + a slot taken from an LDS counter of the tile (k_bucket_emit).
// The order inside a tile's list is then whatever the LDS counters gave; the tile sort orders
// it by the unique (depth bits, index) values, so the result is deterministic.
// ---------------------------------------------------------------------------------------
constexpr int BUCKET_TILES = 8192;     // tiles of one view (LDS counters)
constexpr int BUCKET_MAX_ROWS = 2048;  // rows of one view: the column scan holds 16 columns of each in LDS
constexpr int EB_ROW = 4096;           // entries per bucket row (16 emission blocks of 256)

// The pairs of a wave's 64 consecutive entries [j0, j0 + 64) of one view: lane e holds entry
// e's tile count c and rectangle r. Stages the entries' pair offsets (within the 64), rectangles
// and 1 / width in the wave's LDS slots, then the lanes take the pairs 64 at a time and call
// f(pair offset g, entry lane L, tile of the view) for each. Returns the 64 entries' pair total.
struct WaveStage {
    uint32_t off[64];
    uint64_t rect[64];
    double inv[64];
};

template <class F>
__device__ __forceinline__ uint32_t walk_pairs(WaveStage& st, uint32_t c, uint64_t r, int last, uint32_t tiles_x,
                                               F&& f) {
    const int l = threadIdx.x & 63;
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t total = wave_read(incl, 63);
    st.off[l] = incl - c;
    st.rect[l] = r;
    st.inv[l] = 1.0 / (double)((uint32_t)(r >> 32 & 0xffff) - (uint32_t)(r & 0xffff) + 1u);
    wave_sync();
    for (uint32_t g = l; g < total; g += 64) {
        // largest lane L with off[L] <= g (lanes with no pairs share the next lane's offset)
        int L = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (L + step <= last && st.off[L + step] <= g) L += step;
        const uint64_t rr = st.rect[L];
        const uint32_t x0 = rr & 0xffff, y0 = (rr >> 16) & 0xffff, x1 = (rr >> 32) & 0xffff;
        const uint32_t wd = x1 - x0 + 1;
        const uint32_t k = g - st.off[L];
        // k / wd through FP64 (exact to within one for k < 2^32), then corrected
        uint32_t ky = (uint32_t)((double)k * st.inv[L]);
        uint32_t kx = k - ky * wd;
        if ((int32_t)kx < 0) {
            --ky;
            kx += wd;
        } else if (kx >= wd) {
            ++ky;
            kx -= wd;
        }
        f(g, L, (y0 + ky) * tiles_x + x0 + kx);
    }
    wave_sync();  // the slots are rewritten by the next call
    return total;
}

// Longest-first tile order from one workgroup of NT threads: tiles are bucketed by the bit
// length of their list size len(i) (LPT_B buckets) in LDS, the buckets laid out from the longest
// down, then every tile placed by an LDS counter of its bucket. (The order inside a bucket is
// whatever the counters give: it only decides which tile a workgroup takes, never a result.)
constexpr int LPT_B = 33;

__device__ __forceinline__ int lpt_bits(uint32_t c) { return c ? 32 - __clz(c) : 0; }

template <int NT, class Len>
__device__ void lpt_order_block(Len len, int n_tiles, uint32_t* __restrict__ queue) {
    __shared__ uint32_t lh[LPT_B], base[LPT_B];
    const int t = threadIdx.x;
    if (t < LPT_B) lh[t] = 0;
    __syncthreads();
    for (int i = t; i < n_tiles; i += NT) atomicAdd(&lh[lpt_bits(len(i))], 1u);
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int b = LPT_B - 1; b >= 0; --b) {
            base[b] = acc;
            acc += lh[b];
        }
    }
    __syncthreads();
    for (int i = t; i < n_tiles; i += NT) {
        const uint32_t pos = atomicAdd(&base[lpt_bits(len(i))], 1u);
        if (pos < (uint32_t)n_tiles) queue[pos] = (uint32_t)i;
    }
}

struct BucketArgs {
    const uint32_t* count;
    const uint64_t* rect;
    const float* depth;
    const gs_camera* cams;
    const int32_t* tile_offset;
    int64_t n;           // entries per view
    int64_t nbv;         // emission blocks (256 entries) per view
    int64_t nbr;         // bucket rows (4096 entries) per view
    int tile_w;
    int n_views;
    int stride;          // columns per row: the largest view's tile count (declared), rounded up to 16
    uint32_t* bsum;      // [n_views][nbv] pair sums, then (scanned) exclusive pair offsets
    uint32_t* bh;        // [n_views][nbr][stride] tile histograms, then exclusive prefixes over rows
    uint32_t* tot;       // [n_tiles] pairs per tile
    uint64_t* view_tot;  // [n_views] pairs per view (zero on entry)
    uint32_t* overflow;  // bit 0: the pairs exceed the capacity; bit 2: a view exceeds stride
    uint32_t* sticky;    // or NULL
    uint64_t* n_pairs;   // pair total (zero on entry; the column scans add it up)
    uint64_t* vout;      // FP32 depth bits << 32 | Gaussian index, grouped by tile
    uint64_t capacity;
    uint32_t* ranges;    // [n_tiles][2], written by each view's first row
    uint32_t* eoff;      // [n_views * n] first pair of each entry, or NULL
    uint32_t* queue;     // longest-first tile order, built by an extra workgroup of the emission, or NULL
    int n_tiles;         // all views' tiles
};

constexpr int BK_T = EB_ROW / 4;  // threads of the bucket kernels: one wave per emission block of the row

// tiles of view v, and whether they fit the rows' columns (a view larger than declared is
// reported by the column scans and nothing is binned)
__device__ __forceinline__ int view_tiles(const BucketArgs& a, int v) {
    return a.tile_offset[v + 1] - a.tile_offset[v];
}

// It also clears the frame's state first (the job of k_zero4 when there is no pair to bin):
// no later kernel of the frame runs before it ends.
__global__ __launch_bounds__(BK_T) void k_bucket_count(BucketArgs a, Fill4 clear) {
    __shared__ uint32_t hist[BUCKET_TILES];
    __shared__ WaveStage st[BK_T / 64];
    const int v = blockIdx.y, t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t* cv = a.count + (int64_t)v * a.n;
    const uint64_t* rv = a.rect + (int64_t)v * a.n;
    // wave w takes the row's emission block w, 64 entries at a time; the block's counts and
    // rectangles are requested first, together (rectangles of culled entries too: in random
    // storage order their cache lines are read for the visible ones anyway)
    const int64_t eb = (int64_t)blockIdx.x * (BK_T / 64) + w;
    uint32_t c4[4];
    uint64_t r4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = eb * 256 + k * 64 + l;
        c4[k] = j < a.n ? cv[j] : 0u;
        r4[k] = j < a.n ? rv[j] : 0ull;
    }
    {
        const int64_t tid = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        const int64_t nth = (int64_t)gridDim.x * gridDim.y * blockDim.x;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            for (int64_t i = tid; i < clear.n[b]; i += nth) clear.p[b][i] = 0u;
    }
    const int nt = view_tiles(a, v);
    const bool fits = nt <= a.stride;  // the same for the whole workgroup
    const int ncols = (nt + 15) & ~15;
    for (int i = t; i < ncols && fits; i += BK_T) hist[i] = 0u;
    __syncthreads();
    const uint32_t tiles_x = (uint32_t)div_up(a.cams[v].width, a.tile_w);
    {
        uint32_t bsum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j0 = eb * 256 + k * 64;
            if (j0 >= a.n) break;  // the same for the whole wave
            const int last = (int)min((int64_t)63, a.n - 1 - j0);
            bsum += walk_pairs(st[w], c4[k], c4[k] ? r4[k] : 0ull, last, tiles_x, [&](uint32_t, int, uint32_t tile) {
                if (fits && tile < (uint32_t)nt) atomicAdd(&hist[tile], 1u);
            });
        }
        if (l == 0 && eb * 256 < a.n) a.bsum[(int64_t)v * a.nbv + eb] = bsum;
    }
    __syncthreads();
    uint32_t* row = a.bh + ((int64_t)v * a.nbr + blockIdx.x) * a.stride;
    for (int i = t; i < ncols && fits; i += BK_T) row[i] = hist[i];
}

// Exclusive prefix over a view's rows of every tile's count (in place) and the tile totals.
// Workgroup (g, v) takes tiles [CS g, CS g + CS) of view v: their counts of every row are read
// into LDS, each of BLK / CS chunks of rows summed, the chunk sums scanned, then the prefixes
// written. Each workgroup also adds its totals to the view's and to the pair total. The first
// workgroup of a view too large for the rows' columns sets bit 2 of the overflow word. (Narrow
// column groups give more workgroups than CUs for a view of a few thousand tiles.)
constexpr int COLSCAN_CS = 8;

template <int CS>
__global__ __launch_bounds__(BLK) void k_bucket_colscan(BucketArgs a) {
    constexpr int NCH = BLK / CS;
    __shared__ uint32_t sub[BUCKET_MAX_ROWS * CS];
    __shared__ uint32_t csum[CS][NCH + 1];
    const int t = threadIdx.x, v = blockIdx.y;
    const int nt = view_tiles(a, v);
    if (nt > a.stride) {
        if (blockIdx.x == 0 && t == 0) {
            atomicOr(a.overflow, 4u);
            if (a.sticky) atomicOr(a.sticky, 4u);
        }
        return;
    }
    const int c0 = blockIdx.x * CS;
    if (c0 >= nt) return;  // the whole workgroup
    const int nrows = (int)a.nbr;
    uint32_t* bh = a.bh + (int64_t)v * a.nbr * a.stride;
    for (int i = t; i < nrows * CS; i += BLK) sub[i] = bh[(uint64_t)(i / CS) * a.stride + c0 + (i % CS)];
    __syncthreads();
    const int col = t % CS, chunk = t / CS;
    const int per = (nrows + NCH - 1) / NCH, r0 = min(nrows, chunk * per), r1 = min(nrows, r0 + per);
    uint32_t s = 0;
    for (int r = r0; r < r1; ++r) s += sub[r * CS + col];
    csum[col][chunk] = s;
    __syncthreads();
    if (t < CS) {
        uint32_t run = 0;
        for (int k = 0; k < NCH; ++k) {
            const uint32_t x = csum[t][k];
            csum[t][k] = run;
            run += x;
        }
        if (c0 + t < nt) a.tot[a.tile_offset[v] + c0 + t] = run;
        csum[t][NCH] = run;  // (zero for the padding columns)
    }
    __syncthreads();
    if (t == 0) {
        uint64_t all = 0;
        for (int k = 0; k < CS; ++k) all += csum[k][NCH];
        if (all) {
            atomicAdd((unsigned long long*)a.n_pairs, (unsigned long long)all);
            atomicAdd((unsigned long long*)(a.view_tot + v), (unsigned long long)all);
        }
    }
    uint32_t run = csum[col][chunk];
    for (int r = r0; r < r1; ++r) {
        const uint32_t x = sub[r * CS + col];
        sub[r * CS + col] = run;
        run += x;
    }
    __syncthreads();
    for (int i = t; i < nrows * CS; i += BLK) bh[(uint64_t)(i / CS) * a.stride + c0 + (i % CS)] = sub[i];
}

// block-wide exclusive scan of the N counts c[] in place (N / NT consecutive per thread)
template <int NT, int N>
__device__ __forceinline__ void block_excl_scan_lds(uint32_t* c, uint32_t* wsum) {
    constexpr int PER = N / NT;
    const int t = threadIdx.x;
    uint32_t x[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        x[k] = c[t * PER + k];
        s += x[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<NT>(s, tot, wsum);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        c[t * PER + k] = run;
        run += x[k];
    }
    __syncthreads();
}

__global__ __launch_bounds__(BK_T) void k_bucket_emit(BucketArgs a) {
    __shared__ uint32_t cur[BUCKET_TILES];  // next slot of every tile in this row's part of the bucket
    __shared__ uint32_t wsum[BK_T / 64];
    __shared__ WaveStage st[BK_T / 64];
    __shared__ uint32_t s_db[BK_T / 64][64];
    __shared__ uint64_t s_vstart;
    const int v = blockIdx.y, t = threadIdx.x, w = t >> 6, l = t & 63;
    if (blockIdx.x == a.nbr) {  // the extra column: view 0's builds the longest-first order
        if (v == 0) lpt_order_block<BK_T>([&](int i) { return a.tot[i]; }, a.n_tiles, a.queue);
        return;
    }
    const bool first = blockIdx.x == 0 && blockIdx.y == 0;
    const uint32_t* cv = a.count + (int64_t)v * a.n;
    const uint64_t* rv = a.rect + (int64_t)v * a.n;
    const float* dv = a.depth + (int64_t)v * a.n;
    // the wave's emission block: its counts, rectangles and depths and its first pair are
    // requested first, together, so they arrive while the tile starts are scanned
    const int64_t eb = (int64_t)blockIdx.x * (BK_T / 64) + w;
    uint32_t c4[4], d4[4];
    uint64_t r4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = eb * 256 + k * 64 + l;
        c4[k] = j < a.n ? cv[j] : 0u;
        r4[k] = j < a.n ? rv[j] : 0ull;
        d4[k] = j < a.n ? __float_as_uint(dv[j]) : 0u;
    }
    const uint32_t run0 = eb * 256 < a.n ? a.bsum[(int64_t)v * a.nbv + eb] : 0u;
    // the capacity check (every workgroup reads the complete total; the first sets the flags)
    if (*a.n_pairs > a.capacity) {
        if (first && t == 0) {
            atomicOr(a.overflow, 1u);
            if (a.sticky) atomicOr(a.sticky, 1u);
        }
        return;
    }
    if (*a.overflow) return;  // a view too large for the rows (set by the column scans)
    const int nt = view_tiles(a, v);
    const int tbase = a.tile_offset[v];
    // the view's first pair: the totals of the earlier views
    if (t < 64) {
        uint64_t s = 0;
        for (int k = t; k < v; k += 64) s += a.view_tot[k];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (t == 0) s_vstart = s;
    }
    // tile starts within the view: exclusive scan of its totals (each view's first row writes
    // the ranges)
    for (int i = t; i < BUCKET_TILES; i += BK_T) cur[i] = i < nt ? a.tot[tbase + i] : 0u;
    __syncthreads();
    block_excl_scan_lds<BK_T, BUCKET_TILES>(cur, wsum);
    const uint32_t vstart = (uint32_t)s_vstart;  // (below 2^32 when the capacity check passed)
    const uint32_t* row = a.bh + ((int64_t)v * a.nbr + blockIdx.x) * a.stride;
    for (int i = t; i < nt; i += BK_T) {
        const uint32_t s0 = vstart + cur[i];
        if (blockIdx.x == 0) {
            a.ranges[2 * (tbase + i)] = s0;
            a.ranges[2 * (tbase + i) + 1] = s0 + a.tot[tbase + i];
        }
        cur[i] = s0 + row[i];
    }
    __syncthreads();
    const uint32_t tiles_x = (uint32_t)div_up(a.cams[v].width, a.tile_w);
    {
        if (eb * 256 >= a.n) return;  // the whole wave (no workgroup barrier below)
        uint32_t run = run0;  // first pair of the emission block
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t j0 = eb * 256 + k * 64;
            if (j0 >= a.n) break;
            const int64_t j = j0 + l;
            const uint32_t c = c4[k];
            const uint64_t r = c ? r4[k] : 0ull;
            const uint32_t db = c ? d4[k] : 0u;
            if (a.eoff && j < a.n) a.eoff[(int64_t)v * a.n + j] = run + wave_incl_scan(c) - c;
            s_db[w][l] = db;
            const int last = (int)min((int64_t)63, a.n - 1 - j0);
            run += walk_pairs(st[w], c, r, last, tiles_x, [&](uint32_t, int L, uint32_t tile) {
                if (tile >= (uint32_t)nt) return;
                const uint32_t pos = atomicAdd(&cur[tile], 1u);
                if (pos < a.capacity) a.vout[pos] = ((uint64_t)s_db[w][L] << 32) | (uint32_t)(j0 + L);
            });
        }
    }
}

// ---------------------------------------------------------------------------------------
// Per-tile sort (gs_tile_sort.hpp): one workgroup per tile, longest lists first when ordered
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(TS_T) void k_tile_sort_small(TileSortArgs a) {
    __shared__ TileSortLds sm;
    const int tile = a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
    // the last launch of the binning: every flag of this frame is set by now
    if (a.sticky && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t o = *a.overflow;
        if (o) atomicOr(a.sticky, o);
    }
    sort_tile(sm, a, tile);
}

void launch_tile_sort(const TileSortArgs& ta, hipStream_t stream) {
    if (ta.n_tiles > 0) hipLaunchKernelGGL(k_tile_sort_small, dim3((unsigned)ta.n_tiles), dim3(TS_T), 0, stream, ta);
}

__global__ void k_iota(uint32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------------------
// Longest-first tile order of the traversals (views->lpt): tiles are bucketed by
// bit length of their list size (33 buckets) and laid out from the longest bucket down.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int lpt_bucket(const uint32_t* ranges, int tile) {
    return lpt_bits(ranges[2 * tile + 1] - ranges[2 * tile]);
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

// The same order from one workgroup, for at most LPT_ONE_TILES tiles: bucket counts in LDS,
// their descending scan, then every tile placed by an LDS counter of its bucket (one launch).
constexpr int LPT_ONE_T = 1024, LPT_ONE_TILES = 65536;

__global__ __launch_bounds__(LPT_ONE_T) void k_lpt_one(const uint32_t* __restrict__ ranges, int n_tiles,
                                                       uint32_t* __restrict__ queue) {
    lpt_order_block<LPT_ONE_T>([&](int i) { return ranges[2 * i + 1] - ranges[2 * i]; }, n_tiles, queue);
}

// ---------------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int tile_bits(int n_tiles) {
    int b = 0;
    while (b < 31 && (1u << b) < (uint32_t)n_tiles) ++b;
    return b;
}

struct SortLayout {
    // control block, cleared at the start of every gs_bin_sort: scan chain, pass tickets,
    // digit histograms, LPT counters, pass status tables
    size_t ctrl, scan, tickets, ghist, lpt, view_tot, status, ctrl_end;
    size_t offs, tk0, tk1, tv0, tv1, bk_bh, bk_tot, total;
    int64_t nb_scan, nb_sort, nbr;
    int passes;
    // emission into tile buckets is possible: rows of a view and the histogram space (sized for
    // views of up to min(n_tiles, BUCKET_TILES) tiles) within bounds; it is used when the
    // largest view also has at most BUCKET_TILES tiles
    bool bucket;
};

SortLayout sort_layout(int64_t n, int32_t n_views, uint64_t capacity, int32_t n_tiles) {
    SortLayout L;
    const int64_t vn = n * (int64_t)n_views;
    const size_t nt = (size_t)std::max(n_tiles, 1);
    L.nb_scan = scan_blocks(vn);
    L.nb_sort = (int64_t)((capacity + TILE_ITEMS - 1) / TILE_ITEMS);
    L.passes = std::max(1, (tile_bits(std::max(n_tiles, 1)) + 7) / 8);
    L.nbr = (n + EB_ROW - 1) / EB_ROW;
    // histogram rows of the widest view the bucket emission takes (sized for min(n_tiles, 8192)
    // columns, which bounds any view's); kept within one value buffer's bytes (8 per pair of
    // capacity), or 256 MB: a batch of eight 1M-entry views takes 64 MB, against a grouping
    // that costs hundreds of microseconds more per batch
    const size_t bk_stride = (size_t)((std::min(std::max(n_tiles, 1), BUCKET_TILES) + 15) / 16 * 16);
    const size_t bk_bytes = sizeof(uint32_t) * bk_stride * (size_t)L.nbr * (size_t)std::max(n_views, 1);
    L.bucket = L.nbr <= BUCKET_MAX_ROWS && bk_bytes <= std::max<size_t>(8 * (size_t)capacity, (size_t)256 << 20);
    size_t p = 0;
    L.ctrl = p;
    L.scan = p;
    p = align256(p + sizeof(uint64_t) * ((size_t)L.nb_scan + 1));
    L.tickets = p;
    p = align256(p + sizeof(uint32_t) * KEY_PASSES);
    L.ghist = p;
    p = align256(p + sizeof(uint32_t) * 256 * KEY_PASSES);
    L.lpt = p;
    p = align256(p + sizeof(uint32_t) * 2 * LPT_B);
    L.view_tot = p;
    p = align256(p + sizeof(uint64_t) * (size_t)std::max(n_views, 1));
    L.status = p;
    p = align256(p + sizeof(uint64_t) * 256 * (size_t)L.nb_sort * (size_t)L.passes);
    L.ctrl_end = p;
    L.offs = p;  // pair offsets of the 256-entry emission blocks of every view
    p = align256(p + sizeof(uint32_t) * (size_t)((n + 255) / 256) * (size_t)std::max(n_views, 0));
    const size_t k4 = sizeof(uint32_t) * (size_t)capacity, v8 = sizeof(uint64_t) * (size_t)capacity;
    L.tk0 = p;
    p = align256(p + k4);
    L.tk1 = p;
    p = align256(p + k4);
    L.tv0 = p;
    p = align256(p + v8);
    L.tv1 = p;
    p = align256(p + v8);
    L.bk_bh = p;
    if (L.bucket) p = align256(p + bk_bytes);
    L.bk_tot = p;
    if (L.bucket) p = align256(p + sizeof(uint32_t) * nt);
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
    if (views->n_tiles <= LPT_ONE_TILES) {
        hipLaunchKernelGGL(k_lpt_one, dim3(1), dim3(LPT_ONE_T), 0, stream, bins->ranges, views->n_tiles, bins->queue);
        return check_launch("bin_sort");
    }
    hipLaunchKernelGGL(k_lpt_hist, dim3(std::min(g, 1024u)), dim3(256), 0, stream, bins->ranges, views->n_tiles, lpt);
    hipLaunchKernelGGL(k_lpt_scatter, dim3(g), dim3(256), 0, stream, bins->ranges, views->n_tiles, lpt, lpt + LPT_B,
                       bins->queue);
    return check_launch("bin_sort");
}

// Beyond 4096 tiles: the pairs are written in entry order (tile; depth bits, index), grouped by
// the onesweep passes on the tile id, and the tile ranges read off the grouped keys. Sets vin
// to the grouped values and valt to the other value buffer.
static void launch_entry_order_grouping(const gs_projected* proj, const gs_views* views, gs_bins* bins,
                                        const SortLayout& L, char* w, hipStream_t stream, uint64_t*& vin,
                                        uint64_t*& valt) {
    auto U32 = [&](size_t off) { return (uint32_t*)(w + off); };
    auto U64 = [&](size_t off) { return (uint64_t*)(w + off); };
    const int64_t n = proj->n;
    EmitArgs e;
    e.count = proj->count;
    e.bpre = U32(L.offs);
    e.rect = proj->rect;
    e.depth = proj->depth;
    e.cams = views->cams;
    e.tile_offset = views->tile_offset;
    e.n = n;
    e.tile_w = views->tile_w;
    e.overflow = bins->overflow;
    e.tkey = U32(L.tk0);
    e.tval = U64(L.tv0);
    e.eoff = bins->entry_offset;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((n + 255) / 256), (unsigned)views->n_views), dim3(256), 0, stream, e);
    uint32_t* kin = U32(L.tk0);
    uint32_t* kalt = U32(L.tk1);
    vin = U64(L.tv0);
    valt = U64(L.tv1);
    const int np = L.passes;
    uint32_t* ghist = U32(L.ghist);
    const unsigned hb = (unsigned)std::min<int64_t>(L.nb_sort, 1024);
    hipLaunchKernelGGL(k_os_hist, dim3(hb), dim3(BLK), 0, stream, U32(L.tk0), bins->n_pairs, bins->capacity, np,
                       ghist);
    for (int pass = 0; pass < np; ++pass) {
        PassArgs pa;
        pa.kin = kin;
        pa.vin = vin;
        pa.kout = kalt;
        pa.vout = valt;
        pa.n_items = bins->n_pairs;
        pa.bound = bins->capacity;
        pa.shift = 8 * pass;
        pa.ghist = ghist + 256 * pass;
        pa.status = U64(L.status) + (size_t)256 * L.nb_sort * pass;
        pa.ticket = U32(L.tickets) + pass;
        pa.err = bins->overflow;
        hipLaunchKernelGGL(k_os_pass<uint64_t>, dim3((unsigned)L.nb_sort), dim3(BLK), 0, stream, pa);
        std::swap(kin, kalt);
        std::swap(vin, valt);
    }
    const unsigned rg = (unsigned)((bins->capacity + 255) / 256);
    hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(256), 0, stream, kin, bins->n_pairs, bins->capacity, bins->overflow,
                       bins->ranges, views->n_tiles);
}

// defer: when not NULL the per-tile sort is not launched; its arguments are returned there for a
// compositing launch that sorts each tile itself (n_tiles = 0 there when nothing is to be sorted)
gs_status launch_bin_sort(const gs_projected* proj, const gs_views* views, gs_bins* bins, void* ws,
                          hipStream_t stream, TileSortArgs* defer) {
    if (defer) {
        *defer = TileSortArgs{};
        defer->overflow = bins->overflow;
        defer->n_tiles = 0;
    }
    const int64_t n = proj->n;
    const int64_t vn = n * (int64_t)views->n_views;
    SortLayout L = sort_layout(n, views->n_views, bins->capacity, views->n_tiles);
    char* w = (char*)ws;
    auto U32 = [&](size_t off) { return (uint32_t*)(w + off); };
    auto U64 = [&](size_t off) { return (uint64_t*)(w + off); };

    // ranges start empty; flags, pair count and the control block start at zero
    gs_status st;
    Fill4 f;
    f.p[0] = bins->ranges;
    f.n[0] = 2 * (int64_t)views->n_tiles;
    f.p[1] = bins->overflow;
    f.n[1] = 1;
    f.p[2] = (uint32_t*)bins->n_pairs;
    f.n[2] = 2;
    f.p[3] = U32(L.ctrl);
    f.n[3] = vn == 0 ? 0 : (int64_t)((L.ctrl_end - L.ctrl) / 4);
    if (vn == 0 || views->n_tiles == 0) {
        if ((st = launch_zero4(f, stream))) return st;
        return launch_lpt(views, bins, nullptr, stream);
    }

    // the largest view's tiles decide between the bucket emission and the entry-order grouping
    const int mvt = views->max_view_tiles > 0 ? views->max_view_tiles : views->n_tiles;
    const bool bucket = L.bucket && mvt <= BUCKET_TILES;
    if (bucket) f.n[3] = (int64_t)((L.status - L.ctrl) / 4);  // (no onesweep status tables)

    // 1. pair sums of the emission blocks (clearing the state above first); with tile buckets
    // also every row's tile histogram
    const int64_t nbv = (n + 255) / 256;
    BucketArgs ba;
    ba.count = proj->count;
    ba.rect = proj->rect;
    ba.depth = proj->depth;
    ba.cams = views->cams;
    ba.tile_offset = views->tile_offset;
    ba.n = n;
    ba.nbv = nbv;
    ba.nbr = L.nbr;
    ba.tile_w = views->tile_w;
    ba.n_views = views->n_views;
    ba.stride = (std::min(mvt, views->n_tiles) + 15) / 16 * 16;
    ba.bsum = U32(L.offs);
    ba.bh = U32(L.bk_bh);
    ba.tot = U32(L.bk_tot);
    ba.view_tot = U64(L.view_tot);
    ba.overflow = bins->overflow;
    ba.sticky = bins->overflow_sticky;
    ba.n_pairs = bins->n_pairs;
    ba.vout = U64(L.tv1);
    ba.capacity = bins->capacity;
    ba.ranges = bins->ranges;
    ba.eoff = bins->entry_offset;
    ba.n_tiles = views->n_tiles;
    // with the tile buckets the longest-first order comes from an extra workgroup of the
    // emission (from the tile totals), beside the emission instead of a launch after it
    ba.queue = bucket && bins->queue && views->n_tiles <= LPT_ONE_TILES ? bins->queue : nullptr;
    uint64_t* vin;
    uint64_t* valt;
    if (bucket) {
        // (the emission blocks' pair offsets are only scanned when the entries' first pairs
        // are asked for; the column scans give the pair total and the emission its check)
        hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)L.nbr, (unsigned)views->n_views), dim3(BK_T), 0, stream, ba, f);
        if (bins->entry_offset)
            hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(SB_T), 0, stream, U32(L.offs), nbv * views->n_views,
                               (uint64_t*)nullptr, (uint32_t*)nullptr, bins->capacity, (uint32_t*)nullptr);
        // 2. per-tile prefixes over the rows, tile totals and the pair total, 3. pairs written
        // into their tiles
        hipLaunchKernelGGL(k_bucket_colscan<COLSCAN_CS>, dim3((unsigned)(ba.stride / COLSCAN_CS), (unsigned)views->n_views),
                           dim3(BLK), 0, stream, ba);
        hipLaunchKernelGGL(k_bucket_emit, dim3((unsigned)L.nbr + (ba.queue ? 1u : 0u), (unsigned)views->n_views),
                           dim3(BK_T), 0, stream, ba);
        vin = U64(L.tv1);
        valt = U64(L.tv0);
    } else {
        hipLaunchKernelGGL(k_count_bsums, dim3((unsigned)((nbv + 15) / 16), (unsigned)views->n_views), dim3(256), 0,
                           stream, proj->count, n, nbv, U32(L.offs), f);
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(SB_T), 0, stream, U32(L.offs), nbv * views->n_views,
                           bins->n_pairs, bins->overflow, bins->capacity, bins->overflow_sticky);
        if (L.nb_sort == 0) return launch_lpt(views, bins, U32(L.lpt), stream);
        launch_entry_order_grouping(proj, views, bins, L, w, stream, vin, valt);
    }
    // 5. the longest-first order when asked for (from the ranges, unless the emission built it;
    // the tile sort takes the longest lists first too), 6. each tile's list by (depth, index);
    // keys and values
    if (!ba.queue && (st = launch_lpt(views, bins, U32(L.lpt), stream))) return st;
    TileSortArgs ta;
    ta.pairs = vin;
    ta.scratch = valt;
    ta.ranges = bins->ranges;
    ta.n_tiles = views->n_tiles;
    ta.capacity = bins->capacity;
    ta.overflow = bins->overflow;
    ta.keys = bins->keys;
    ta.vals = bins->vals;
    ta.sticky = bins->overflow_sticky;
    ta.order = bins->queue;
    if (defer) {
        *defer = ta;
        return check_launch("bin_sort");
    }
    launch_tile_sort(ta, stream);
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
