// Pruning (Sec. 3.3): the Gaussians whose importance h_i = max over all training rays of
// their composited weight stays below t_prune are removed, and every per-Gaussian array that
// must follow the parameters (the parameters themselves, optimizer moments, ...) is
// compacted in index order. HBM-bound stream compaction:
//   keep     one wave per 64 Gaussians: ballot of [h_i >= t_prune] into two bitset words
//   list     the bitset to the increasing list of kept indices (popcount, single-pass scan,
//            per-word expansion), shared with the visibility-list compaction
//   gather   one lane per kept Gaussian loads its index once and copies that Gaussian's value
//            of up to 32 planes per launch; writes are coalesced, reads follow the increasing
//            kept indices
// The gather alone (gs_gather) also materialises a Gaussian subset, such as a camera cluster's
// visibility list (Sec. 3.4), as compact planes, so renders of that subset read coalesced rows.
#include <algorithm>

#include "gs_device.hpp"

namespace gs {

gs_status launch_bits_to_list(const uint32_t*, int64_t, int32_t*, int64_t*, void*, hipStream_t);

__global__ __launch_bounds__(256) void k_keep_bits(const float* __restrict__ h, int64_t n, float t,
                                                   uint32_t* __restrict__ bits) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool keep = i < n && h[i] >= t;  // a NaN importance is not kept
    const uint64_t m = ballot(keep);
    const int l = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * 256 + (threadIdx.x & ~63)) >> 5;  // first word of the wave
    const int64_t words = (n + 31) >> 5;
    if (l == 0 && w0 < words) bits[w0] = (uint32_t)m;
    if (l == 32 && w0 + 1 < words) bits[w0 + 1] = (uint32_t)(m >> 32);
}

constexpr int PLANES_PER_LAUNCH = 32;

struct PlaneTable {
    const float* in[PLANES_PER_LAUNCH];
    float* out[PLANES_PER_LAUNCH];
    int count;
};

// out[p][k] = in[p][index[k]] for k < min(*n_index, bound) (n_index NULL: k < bound); an index
// outside [0, n_src) reads nothing and writes 0
__global__ __launch_bounds__(256) void k_gather_planes(PlaneTable tab, const int32_t* __restrict__ index,
                                                       const int64_t* n_index, int64_t bound, int64_t n_src) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nk = n_index ? min(*n_index, bound) : bound;
    if (k >= nk) return;
    const int64_t i = index[k];
    const bool ok = i >= 0 && i < n_src;
#pragma unroll 4
    for (int p = 0; p < tab.count; ++p) tab.out[p][k] = ok ? tab.in[p][i] : 0.f;
}

static gs_status gather_launches(const float* const* planes_in, float* const* planes_out, int32_t n_planes,
                                 const int32_t* index, const int64_t* n_index, int64_t bound, int64_t n_src,
                                 hipStream_t stream) {
    for (int p0 = 0; p0 < n_planes; p0 += PLANES_PER_LAUNCH) {
        PlaneTable tab;
        tab.count = std::min(PLANES_PER_LAUNCH, n_planes - p0);
        for (int p = 0; p < PLANES_PER_LAUNCH; ++p) {
            tab.in[p] = p < tab.count ? planes_in[p0 + p] : nullptr;
            tab.out[p] = p < tab.count ? planes_out[p0 + p] : nullptr;
        }
        hipLaunchKernelGGL(k_gather_planes, dim3((unsigned)((bound + 255) / 256)), dim3(256), 0, stream, tab, index,
                           n_index, bound, n_src);
    }
    return check_launch("gather");
}

gs_status launch_gather(const int32_t* index, int64_t n_index, int64_t n_src, const float* const* planes_in,
                        float* const* planes_out, int32_t n_planes, hipStream_t stream) {
    if (n_index == 0 || n_planes == 0) return GS_OK;
    return gather_launches(planes_in, planes_out, n_planes, index, nullptr, n_index, n_src, stream);
}

size_t prune_workspace_bytes(int64_t n) {
    const size_t words = (size_t)((n + 31) / 32);
    return ((sizeof(uint32_t) * words + 255) & ~(size_t)255);
}

// ws: the keep bitset followed by the list workspace
gs_status launch_prune(const float* h, int64_t n, float t, const float* const* planes_in, float* const* planes_out,
                       int32_t n_planes, int32_t* kept, int64_t* n_kept, void* ws, size_t list_ws_offset,
                       hipStream_t stream) {
    uint32_t* bits = (uint32_t*)ws;
    if (n > 0)
        hipLaunchKernelGGL(k_keep_bits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, h, n, t, bits);
    gs_status st = launch_bits_to_list(bits, n, kept, n_kept, (char*)ws + list_ws_offset, stream);
    if (st || n == 0) return st;
    return gather_launches(planes_in, planes_out, n_planes, kept, n_kept, n, n, stream);
}

}  // namespace gs

namespace gs {

// m_i = [h_i < t_prune] as bytes (the prune mask itself)
__global__ __launch_bounds__(256) void k_prune_mask(const float* __restrict__ h, int64_t n, float t,
                                                    uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) mask[i] = !(h[i] >= t);  // consistent with the kept set: a NaN importance is pruned
}

gs_status launch_prune_mask(const float* h, int64_t n, float t, uint8_t* mask, hipStream_t stream) {
    if (n == 0) return GS_OK;
    hipLaunchKernelGGL(k_prune_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, h, n, t, mask);
    return check_launch("prune_mask");
}

}  // namespace gs
