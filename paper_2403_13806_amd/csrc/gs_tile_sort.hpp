// Per-tile sort by (depth bits, index), shared by the binning's sort launch and the
// compositing launch that sorts each tile just before compositing it. A workgroup of TS_T
// threads sorts one tile's list in LDS.
#pragma once
#include "gs_device.hpp"

namespace gs {

constexpr int TS_T = 256;  // threads of a tile-sort workgroup

// block-wide exclusive scan of one u32 per thread (NT threads); returns the block total
template <int NT = TS_T>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, uint32_t* wsum) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t incl = wave_incl_scan(x);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        const uint32_t s = wsum[k];
        pre += (k < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + incl - x;
}

constexpr int SMALL_LIST = 2048;  // 16 KB of LDS per workgroup

struct TileSortArgs {
    uint64_t* pairs;    // values grouped by tile; also the merge buffer of very long lists
    uint64_t* scratch;  // [capacity]
    const uint32_t* ranges;
    int n_tiles;
    uint64_t capacity;
    const uint32_t* overflow;
    uint64_t* keys;
    uint32_t* vals;
    uint32_t* sticky;      // OR-ed with the overflow word, or NULL
    const uint32_t* order; // tiles longest list first (workgroup b sorts order[b]), or NULL
};

// Ascending bitonic sort of s[0, N) by a 256-thread workgroup (N a power of two >= 2).
// Pair i of a stage goes to thread i mod 256, so in a stage of stride j <= 64 the pairs of
// one wave (i = 64 c + lane, c = wave mod 4) stay inside the 128-element chunks c of that
// wave: those stages need no workgroup barrier, only the wider ones do.
static __device__ void bitonic_lds(uint64_t* s, int N) {
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const bool wide = j > 64;
            if (wide) __syncthreads();
            for (int i = threadIdx.x; i < (N >> 1); i += TS_T) {
                const int lo = 2 * i - (i & (j - 1)), hi = lo + j;
                const uint64_t x = s[lo], y = s[hi];
                if ((x > y) == ((lo & k) == 0)) {
                    s[lo] = y;
                    s[hi] = x;
                }
            }
            if (wide)
                __syncthreads();
            else
                wave_sync();
        }
    }
    __syncthreads();
}

static __device__ __forceinline__ int pow2_at_least(int x) {
    int p = 2;
    while (p < x) p <<= 1;
    return p;
}

// sort src[0, len) (len <= cap) through the LDS buffer s into s[0, len)
static __device__ void sort_in_lds(uint64_t* s, const uint64_t* src, int len) {
    const int N = pow2_at_least(len);
    for (int i = threadIdx.x; i < N; i += TS_T) s[i] = i < len ? src[i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, N);
}

static __device__ void write_tile(const TileSortArgs& a, int tile, uint32_t start, const uint64_t* s, int len) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        const uint64_t x = s[i];
        a.keys[start + i] = ((uint64_t)tile << 32) | (x >> 32);
        a.vals[start + i] = (uint32_t)x;
    }
}

// number of elements taken from A among the first d of the merge of sorted A and B
// (keys are unique)
static __device__ __forceinline__ int merge_split(const uint64_t* A, int na, const uint64_t* B, int nb, int d) {
    int lo = max(0, d - nb), hi = min(d, na);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] < B[d - 1 - mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// A list longer than SMALL_LIST, sorted by the workgroup that owns its tile: chunks of
// SMALL_LIST by the bitonic sort in LDS into the scratch area of the list, then pairwise merges
// (merge path: thread i takes the i-th 1/256 of the merged output) back and forth between the
// scratch and the list's own area, then the keys and values written.
static __device__ void sort_long(const TileSortArgs& a, int tile, uint32_t start, int len, uint64_t* s) {
    uint64_t* src = a.scratch + start;
    uint64_t* dst = a.pairs + start;
    for (int c0 = 0; c0 < len; c0 += SMALL_LIST) {
        const int cl = min(SMALL_LIST, len - c0);
        sort_in_lds(s, a.pairs + start + c0, cl);
        for (int i = threadIdx.x; i < cl; i += blockDim.x) src[c0 + i] = s[i];
        __syncthreads();
    }
    for (int wd = SMALL_LIST; wd < len; wd <<= 1) {
        for (int m0 = 0; m0 < len; m0 += 2 * wd) {
            const int na = min(wd, len - m0), nb = max(0, min(wd, len - m0 - wd));
            const uint64_t* A = src + m0;
            const uint64_t* B = A + na;
            const int M = na + nb;
            const int d0 = (int)((int64_t)M * threadIdx.x / blockDim.x);
            const int d1 = (int)((int64_t)M * (threadIdx.x + 1) / blockDim.x);
            int i = merge_split(A, na, B, nb, d0), j = d0 - i;
            for (int d = d0; d < d1; ++d) {
                const bool takeA = j >= nb || (i < na && A[i] < B[j]);
                dst[m0 + d] = takeA ? A[i++] : B[j++];
            }
        }
        __syncthreads();
        uint64_t* tmp = src;
        src = dst;
        dst = tmp;
    }
    write_tile(a, tile, start, src, len);
}

// Stable LSD radix sort of one tile's list (len <= SMALL_LIST) by its FP32 depth bits,
// 8-bit digits, in LDS. Wave w owns the contiguous items [w C, (w + 1) C) (C a multiple of 64)
// and ranks them with wave-private digit counters; passes whose digit is the same for every
// item of the tile are skipped. Equal depths keep the order the grouping left, which is not
// index order (the bucket emission takes slots from LDS counters): runs of equal depth bits in
// the sorted list (rare, and short) are then put in index order, or, for a run longer than 64,
// the whole list is sorted again by its unique 64-bit (depth bits, index) values with a
// bitonic network, so the result is the (depth, index) order whatever order the list came in.
constexpr int RS_ROUNDS = SMALL_LIST / TS_T;  // items per thread

struct TileSortLds {
    union {
        struct {
            uint32_t k[SMALL_LIST], v[SMALL_LIST];
        } kv;
        uint64_t kv64[SMALL_LIST];
    } lds;
    uint32_t wcnt[TS_T / 64][256];
    uint32_t ds[256];
    uint32_t wsum[TS_T / 64];
    uint32_t diff, ties;
};

// Sorts tile `tile` (called by all TS_T threads of a workgroup; every return is taken by the
// whole workgroup). The sticky overflow flag is the caller's.
static __device__ void sort_tile(TileSortLds& sm, const TileSortArgs& a, int tile) {
    uint32_t* sk = sm.lds.kv.k;
    uint32_t* sv = sm.lds.kv.v;
    auto& wcnt = sm.wcnt;
    auto& ds = sm.ds;
    auto& wsum = sm.wsum;
    uint32_t& diff = sm.diff;
    uint32_t& ties = sm.ties;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (*a.overflow || tile >= a.n_tiles) return;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    if (end <= start || (uint64_t)end > a.capacity) return;
    const int len = (int)(end - start);
    if (len > SMALL_LIST) {  // (the same for the whole workgroup)
        sort_long(a, tile, start, len, sm.lds.kv64);
        return;
    }
    const uint64_t* src = a.pairs + start;
    const int C = (((len + 3) >> 2) + 63) & ~63;
    const int R = C >> 6;
    const int wb = w * C;
    if (t == 0) diff = 0, ties = 0;
    const uint32_t k0 = (uint32_t)(src[0] >> 32);
    uint32_t key[RS_ROUNDS], val[RS_ROUNDS], lr[RS_ROUNDS];
    uint32_t dx = 0;
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int i = wb + 64 * r + l;
        const bool valid = r < R && i < len;
        const uint64_t x = valid ? src[i] : 0ull;
        key[r] = (uint32_t)(x >> 32);
        val[r] = (uint32_t)x;
        if (valid) dx |= key[r] ^ k0;
    }
    __syncthreads();
    if (dx) atomicOr(&diff, dx);
    __syncthreads();
    const uint32_t dmask = diff;
    for (int shift = 0; shift < 32; shift += 8) {
        if (((dmask >> shift) & 255u) == 0) continue;  // the same for the whole workgroup
#pragma unroll
        for (int k = 0; k < 4; ++k) wcnt[w][l + 64 * k] = 0;
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            const bool valid = wb + 64 * r + l < len;
            const uint32_t d = (key[r] >> shift) & 255u;
            uint64_t m = ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool on = (d >> bit) & 1u;
                const uint64_t bb = ballot(on);
                m &= on ? bb : ~bb;
            }
            const uint32_t rank = mask_rank(m);
            const uint32_t old = valid ? wcnt[w][d] : 0u;
            lr[r] = old + rank;
            if (valid && rank == 0) wcnt[w][d] = old + (uint32_t)__popcll(m);
        }
        __syncthreads();
        uint32_t mine = 0;
#pragma unroll
        for (int k = 0; k < TS_T / 64; ++k) {
            const uint32_t c = wcnt[k][t];
            wcnt[k][t] = mine;
            mine += c;
        }
        uint32_t tot;
        ds[t] = block_excl_scan(mine, tot, wsum);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            if (wb + 64 * r + l < len) {
                const uint32_t d = (key[r] >> shift) & 255u;
                const uint32_t q = ds[d] + wcnt[w][d] + lr[r];
                sk[q] = key[r];
                sv[q] = val[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            const int i = wb + 64 * r + l;
            if (i < len) {
                key[r] = sk[i];
                val[r] = sv[i];
            }
        }
    }
    // equal depth bits next to each other in the sorted list? (sk holds the last pass's
    // order; with no pass at all every depth is the same)
    bool tie = dmask == 0u && len > 1;
    if (dmask != 0u) {
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            const int i = wb + 64 * r + l;
            tie |= i + 1 < len && key[r] == sk[i + 1];
        }
    }
    if (tie) atomicOr(&ties, 1u);
    __syncthreads();
    if (ties) {  // the same for the whole workgroup
        if (dmask == 0u) {  // no pass ran: the list is not in LDS yet
#pragma unroll
            for (int r = 0; r < RS_ROUNDS; ++r) {
                if (r >= R) break;
                const int i = wb + 64 * r + l;
                if (i < len) sk[i] = key[r], sv[i] = val[r];
            }
            __syncthreads();
        }
        // the thread holding the first item of a run of equal depths puts the run's indices in
        // increasing order (runs are short: two items, as a rule); a run longer than 64 sends
        // the whole list to the bitonic sort of its (depth bits, index) values
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            const int i = wb + 64 * r + l;
            if (i >= len) continue;
            const uint32_t kk = sk[i];
            if ((i > 0 && sk[i - 1] == kk) || i + 1 >= len || sk[i + 1] != kk) continue;
            int j = i + 1;
            while (j < len && j - i <= 64 && sk[j] == kk) ++j;
            if (j - i > 64) {
                atomicOr(&ties, 2u);
                continue;
            }
            for (int x = i + 1; x < j; ++x) {  // insertion sort of sv[i, j)
                const uint32_t y = sv[x];
                int z = x - 1;
                while (z >= i && sv[z] > y) {
                    sv[z + 1] = sv[z];
                    --z;
                }
                sv[z + 1] = y;
            }
        }
        __syncthreads();
        if (ties & 2u) {
            sort_in_lds(sm.lds.kv64, src, len);
            write_tile(a, tile, start, sm.lds.kv64, len);
            return;
        }
#pragma unroll
        for (int r = 0; r < RS_ROUNDS; ++r) {
            if (r >= R) break;
            const int i = wb + 64 * r + l;
            if (i < len) val[r] = sv[i];
        }
    }
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        if (r >= R) break;
        const int i = wb + 64 * r + l;
        if (i < len) {
            a.keys[start + i] = ((uint64_t)tile << 32) | key[r];
            a.vals[start + i] = val[r];
        }
    }
}

}  // namespace gs
