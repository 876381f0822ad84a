// Device-side helpers shared by the gfx950 kernels: wave64 primitives built on DPP
// and ballots, tile/view lookup, and launch error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

#define GS_WAVE 64

namespace gs {

// ---------------------------------------------------------------------------------------
// Host-side error state (thread-local message) and launch checking.
// ---------------------------------------------------------------------------------------
gs_status set_error(gs_status code, const char* fmt, ...);
gs_status check_launch(const char* what);
// workgroups of a persistent launch of fn: CUs x resident workgroups per CU, at most n_items
int persistent_grid(const void* fn, int threads, int64_t n_items);

// ---------------------------------------------------------------------------------------
// wave64 primitives. Every helper must be called with all 64 lanes active.
// DPP control words (gfx9): quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E,
// row_shr:n = 0x110 + n, row_mirror = 0x140, row_half_mirror = 0x141,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.
// ---------------------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND = true>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, BANK_MASK, BOUND);
}

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of a 64-bit lane mask below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// inclusive prefix sum over the wave (u32)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    int v = (int)x;
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    v += dpp<0x142, 0xa, 0xf, false>(v);
    v += dpp<0x143, 0xc, 0xf, false>(v);
    return (uint32_t)v;
}

__device__ __forceinline__ uint32_t wave_read(uint32_t x, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

// max over the wave of non-negative floats (integer order of their bit patterns)
__device__ __forceinline__ float wave_max_nonneg(float x) {
    int v = __float_as_int(x);
    v = max(v, dpp<0xB1>(v));
    v = max(v, dpp<0x4E>(v));
    v = max(v, dpp<0x141>(v));
    v = max(v, dpp<0x140>(v));
    int a = max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
    int b = max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
    return __int_as_float(max(a, b));
}

// sum over the wave (fixed association order, so results are reproducible)
__device__ __forceinline__ float wave_sum(float x) {
    x += __int_as_float(dpp<0xB1>(__float_as_int(x)));
    x += __int_as_float(dpp<0x4E>(__float_as_int(x)));
    x += __int_as_float(dpp<0x141>(__float_as_int(x)));
    x += __int_as_float(dpp<0x140>(__float_as_int(x)));
    float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0)) +
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32)) +
              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return a + b;
}

// the LDS writes of this wave are visible to its later LDS reads (no other wave involved)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one step of a segmented scan of nine fields keyed by the owner lane L
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_step(int L, float (&x)[9]) {
    const int Ld = __builtin_amdgcn_update_dpp(-1, L, CTRL, ROW_MASK, 0xf, false);
    const bool merge = Ld == L;
#pragma unroll
    for (int f = 0; f < 9; ++f) {
        const float y = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x[f]), CTRL, ROW_MASK, 0xf, true));
        x[f] = merge ? x[f] + y : x[f];
    }
}

// Segmented inclusive scan of nine fields over the wave's lanes, runs keyed by the owner L
// (non-decreasing over the lanes; a lane with a unique key is a run of its own), with the
// steps of a wave scan: shifts by 1, 2, 4, 8 inside each row of 16, then the last lane of a
// row added into the next rows. A lane adds what arrives only from a lane of its own run (a
// source with the same owner means every lane in between has it too); lanes that receive
// nothing get zeros. The last lane of each run ends with the run's sum, formed in the same
// order on every call. Must be called with all 64 lanes active.
__device__ __forceinline__ void seg_scan9(int L, float (&x)[9]) {
    seg_step<0x111, 0xf>(L, x);
    seg_step<0x112, 0xf>(L, x);
    seg_step<0x114, 0xf>(L, x);
    seg_step<0x118, 0xf>(L, x);
    seg_step<0x142, 0xa>(L, x);
    seg_step<0x143, 0xc>(L, x);
}

// ---------------------------------------------------------------------------------------
// View lookup for a global tile id: largest v with tile_offset[v] <= tile.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int view_of_tile(const int32_t* __restrict__ tile_offset, int n_views, int tile) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_offset[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__host__ __device__ __forceinline__ int div_up(int a, int b) { return (a + b - 1) / b; }

// position of workgroup b in an order where each of the 8 XCDs (workgroups are dispatched to
// them round-robin, each XCD has its own L2) takes one contiguous range of [0, n): work on
// neighbouring tiles then shares an L2. Worth it where neighbours share data and costs are even
// (the loss windows); the compositing tiles keep the plain order, which spreads the expensive
// centre of a view over all XCDs.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t n) {
    const int64_t q = n / 8, rem = n % 8, x = b % 8, s = b / 8;
    return x * q + (x < rem ? x : rem) + s;
}

}  // namespace gs
