// Initialisation of the point representation from a point set (Sec. 3.2): one Gaussian per
// point, its isotropic scale the distance to the nearest point of the set at another position,
// opacity 0.1, identity rotation, DC colour from a given per-point colour, higher SH 0.
//
// Exact nearest-neighbour distances on a uniform cell grid:
//   k_bbox       bounding box of the finite points: per-workgroup partials (ordered-integer
//                min/max), combined by k_bbox_final
//   k_grid       one thread: cell size h with at most `cap` cells (about one point per cell over
//                the box), grid dimensions
//   k_cell_count cell of every point, its rank inside the cell (atomic counter per cell)
//   k_scan_*     exclusive scan of the cell counts (blocks, block totals, offsets)
//   k_scatter    points stored cell by cell (x, y, z, index) for coherent reads
//   k_nn         one lane per stored point, neighbouring lanes in the same or nearby cells:
//                Chebyshev rings of cells around the point's cell, nearest squared distance
//                over points at another position, stopping after ring r once that distance is
//                at most the distance to the nearest face of the searched block of cells (less a
//                rounding margin): every point not yet visited lies beyond one of those faces
// Squared distances are FP64 from the FP32 coordinates, (dx dx + dy dy) + dz dz without fused
// multiply-add, and the distance is rounded to FP32 once, so the minimum does not depend on the
// visiting order.
#include <cmath>

#include "gs_device.hpp"

namespace gs {

namespace {

constexpr int NB = 256;
constexpr int BBOX_BLOCKS = 256;  // workgroups of the bounding-box pass
constexpr int SCAN_T = 1024, SCAN_IPT = 4, SCAN_ITEMS = SCAN_T * SCAN_IPT;
constexpr double kY00 = 0.28209479177387814;  // 1 / (2 sqrt(pi))

struct GridCtrl {
    uint32_t lo[3], hi[3];  // ordered-integer encoding of the FP32 bounds
    uint32_t n_finite;
    int32_t gdim[3];
    int64_t ncell;
    double org[3];
    double h, inv_h, eps;
};

__device__ __forceinline__ uint32_t f2o(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

struct NnLayout {
    GridCtrl* ctrl;
    uint32_t* bbox;    // [BBOX_BLOCKS][7] per-workgroup bounds and counts
    uint32_t* cell;    // [n] cell of each point (0xffffffff: non-finite)
    uint32_t* rank;    // [n]
    uint32_t* start;   // [cap + 1] counts, then exclusive starts
    uint32_t* totals;  // [n scan blocks]
    float4* sorted;    // [n] (x, y, z, index bits) cell by cell
    int64_t cap;
};

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// cells of the grid: about one per point, at most 2^24 - 1 (the scan of the cap + 1 counters
// then has at most SCAN_ITEMS block totals)
static int64_t cell_cap(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(n, ((int64_t)1 << 24) - 1)); }

static int64_t scan_blocks(int64_t items) { return (items + SCAN_ITEMS - 1) / SCAN_ITEMS; }

static NnLayout nn_layout(void* ws, int64_t n) {
    NnLayout L;
    L.cap = cell_cap(n);
    char* p = static_cast<char*>(ws);
    L.ctrl = reinterpret_cast<GridCtrl*>(p);
    p += a256(sizeof(GridCtrl));
    L.bbox = reinterpret_cast<uint32_t*>(p);
    p += a256(sizeof(uint32_t) * 7 * BBOX_BLOCKS);
    L.cell = reinterpret_cast<uint32_t*>(p);
    p += a256(sizeof(uint32_t) * (size_t)n);
    L.rank = reinterpret_cast<uint32_t*>(p);
    p += a256(sizeof(uint32_t) * (size_t)n);
    L.start = reinterpret_cast<uint32_t*>(p);
    p += a256(sizeof(uint32_t) * (size_t)(L.cap + 1));
    L.totals = reinterpret_cast<uint32_t*>(p);
    p += a256(sizeof(uint32_t) * (size_t)scan_blocks(L.cap + 1));
    L.sorted = reinterpret_cast<float4*>(p);
    return L;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// per-workgroup bounds of the finite points and their count: partial[b] = (lo[3], hi[3], count)
__global__ __launch_bounds__(NB) void k_bbox(const float* __restrict__ pts, int64_t n, uint32_t* __restrict__ partial) {
    __shared__ uint32_t red[NB / 64][7];
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u}, cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x; i < n; i += (int64_t)gridDim.x * NB) {
        const float x = pts[i], y = pts[n + i], z = pts[2 * n + i];
        if (!finite3(x, y, z)) continue;
        const uint32_t o[3] = {f2o(x), f2o(y), f2o(z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) lo[a] = min(lo[a], o[a]), hi[a] = max(hi[a], o[a]);
        ++cnt;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int s = 32; s >= 1; s >>= 1) {
            lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], s));
            hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], s));
        }
    }
    for (int s = 32; s >= 1; s >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, s);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) red[w][a] = lo[a], red[w][3 + a] = hi[a];
        red[w][6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int f = threadIdx.x;
        uint32_t v = red[0][f];
        for (int k = 1; k < NB / 64; ++k) v = f < 3 ? min(v, red[k][f]) : (f < 6 ? max(v, red[k][f]) : v + red[k][f]);
        partial[blockIdx.x * 7 + f] = v;
    }
}

// one workgroup: the partial bounds combined into the control block
__global__ __launch_bounds__(NB) void k_bbox_final(const uint32_t* __restrict__ partial, int nb, GridCtrl* c) {
    __shared__ uint32_t red[NB / 64][7];
    const int t = threadIdx.x, w = t >> 6;
    uint32_t v[7] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u, 0u};
    if (t < nb) {
#pragma unroll
        for (int f = 0; f < 7; ++f) v[f] = partial[t * 7 + f];
    }
#pragma unroll
    for (int f = 0; f < 7; ++f)
        for (int s = 32; s >= 1; s >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v[f], s);
            v[f] = f < 3 ? min(v[f], o) : (f < 6 ? max(v[f], o) : v[f] + o);
        }
    if ((t & 63) == 0)
        for (int f = 0; f < 7; ++f) red[w][f] = v[f];
    __syncthreads();
    if (t < 7) {
        uint32_t x = red[0][t];
        for (int k = 1; k < NB / 64; ++k) x = t < 3 ? min(x, red[k][t]) : (t < 6 ? max(x, red[k][t]) : x + red[k][t]);
        if (t < 3) c->lo[t] = x;
        else if (t < 6) c->hi[t - 3] = x;
        else c->n_finite = x;
    }
}

__global__ void k_grid(GridCtrl* c, int64_t cap) {
    if (c->n_finite == 0) {
        for (int a = 0; a < 3; ++a) c->gdim[a] = 1, c->org[a] = 0.0;
        c->ncell = 1, c->h = 1.0, c->inv_h = 1.0, c->eps = 0.0;
        return;
    }
    double ext[3], emax = 0.0, amax = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double lo = (double)o2f(c->lo[a]), hi = (double)o2f(c->hi[a]);
        c->org[a] = lo;
        ext[a] = hi - lo;
        emax = fmax(emax, ext[a]);
        amax = fmax(amax, fmax(fabs(lo), fabs(hi)));
    }
    auto cells = [&](double h) {
        double p = 1.0;
        for (int a = 0; a < 3; ++a) p *= floor(ext[a] / h) + 1.0;
        return p;
    };
    double h = emax > 0.0 ? emax / cbrt((double)cap) * 1.0000001 : 1.0;
    while (cells(h) > (double)cap) h *= 1.25;
    if (emax > 0.0)
        while (cells(h * 0.8) <= (double)cap && h * 0.8 > emax * 1e-9) h *= 0.8;
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) {
        c->gdim[a] = (int32_t)(floor(ext[a] / h) + 1.0);
        nc *= c->gdim[a];
    }
    c->ncell = nc;
    c->h = h;
    c->inv_h = 1.0 / h;
    // rounding of the cell boundaries, relative to the coordinates' magnitude
    c->eps = 1e-12 * (amax + emax + h);
}

__device__ __forceinline__ int cell_axis(double x, double org, double inv_h, int g) {
    const double t = floor((x - org) * inv_h);
    return (int)fmin(fmax(t, 0.0), (double)(g - 1));
}

__global__ __launch_bounds__(NB) void k_cell_count(const float* __restrict__ pts, int64_t n, const GridCtrl* c,
                                                   uint32_t* __restrict__ cell, uint32_t* __restrict__ rank,
                                                   uint32_t* __restrict__ count, float* __restrict__ dist) {
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i >= n) return;
    const float x = pts[i], y = pts[n + i], z = pts[2 * n + i];
    if (!finite3(x, y, z)) {
        cell[i] = 0xffffffffu;
        dist[i] = __uint_as_float(0x7fc00000u);  // NaN: a non-finite point has no neighbour
        return;
    }
    const int gx = cell_axis(x, c->org[0], c->inv_h, c->gdim[0]);
    const int gy = cell_axis(y, c->org[1], c->inv_h, c->gdim[1]);
    const int gz = cell_axis(z, c->org[2], c->inv_h, c->gdim[2]);
    const uint32_t id = (uint32_t)(((int64_t)gz * c->gdim[1] + gy) * c->gdim[0] + gx);
    cell[i] = id;
    rank[i] = atomicAdd(&count[id], 1u);
}

__global__ __launch_bounds__(NB) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i < n) p[i] = v;
}

// exclusive scan of x[0 .. m): per block of SCAN_ITEMS, then the block totals, then offsets
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        const uint32_t s = l < SCAN_T / 64 ? wsum[l] : 0u;
        const uint32_t si = wave_incl_scan(s);
        if (l < SCAN_T / 64) wsum[l] = si - s;
        if (l == SCAN_T / 64 - 1) wsum[SCAN_T / 64] = si;
    }
    __syncthreads();
    total = wsum[SCAN_T / 64];
    return wsum[w] + incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(uint32_t* __restrict__ x, int64_t m,
                                                        uint32_t* __restrict__ totals) {
    __shared__ uint32_t wsum[SCAN_T / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS + (int64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT], s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        v[k] = base + k < m ? x[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(s, wsum, total);
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        if (base + k < m) x[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// one workgroup: the block totals (at most SCAN_ITEMS of them) to exclusive offsets
__global__ __launch_bounds__(SCAN_T) void k_scan_totals(uint32_t* __restrict__ totals, int64_t nb) {
    __shared__ uint32_t wsum[SCAN_T / 64 + 1];
    const int64_t base = (int64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT], s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        v[k] = base + k < nb ? totals[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(s, wsum, total);
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        if (base + k < nb) totals[base + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(NB) void k_scan_add(uint32_t* __restrict__ x, int64_t m,
                                                 const uint32_t* __restrict__ totals) {
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i < m) x[i] += totals[i / SCAN_ITEMS];
}

__global__ __launch_bounds__(NB) void k_scatter(const float* __restrict__ pts, int64_t n,
                                                const uint32_t* __restrict__ cell, const uint32_t* __restrict__ rank,
                                                const uint32_t* __restrict__ start, float4* __restrict__ sorted) {
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i >= n || cell[i] == 0xffffffffu) return;
    sorted[start[cell[i]] + rank[i]] = make_float4(pts[i], pts[n + i], pts[2 * n + i], __int_as_float((int)i));
}

__device__ __forceinline__ double dist2(float4 p, double qx, double qy, double qz) {
#pragma clang fp contract(off)
    const double dx = (double)p.x - qx, dy = (double)p.y - qy, dz = (double)p.z - qz;
    return (dx * dx + dy * dy) + dz * dz;
}

// the points of cells [id0, id1] of one grid row: contiguous in the cell-ordered copy
__device__ __forceinline__ void scan_cells(const uint32_t* __restrict__ start, const float4* __restrict__ sorted,
                                           int64_t id0, int64_t id1, double qx, double qy, double qz, double& best) {
    const uint32_t b = start[id0], e = start[id1 + 1];
    for (uint32_t j = b; j < e; ++j) {
        const double d = dist2(sorted[j], qx, qy, qz);
        if (d > 0.0 && d < best) best = d;
    }
}

__global__ __launch_bounds__(NB) void k_nn(const GridCtrl* __restrict__ c, const uint32_t* __restrict__ start,
                                           const float4* __restrict__ sorted, int64_t cap, float* __restrict__ dist) {
    const int64_t pos = (int64_t)blockIdx.x * NB + threadIdx.x;
    const uint32_t total = start[cap];
    if (pos >= total) return;
    const float4 q = sorted[pos];
    const double qx = q.x, qy = q.y, qz = q.z;
    const int G0 = c->gdim[0], G1 = c->gdim[1], G2 = c->gdim[2];
    const double h = c->h, eps = c->eps;
    const int cx = cell_axis(qx, c->org[0], c->inv_h, G0);
    const int cy = cell_axis(qy, c->org[1], c->inv_h, G1);
    const int cz = cell_axis(qz, c->org[2], c->inv_h, G2);
    const int rmax = max(G0, max(G1, G2));
    double best = INFINITY;
    // ring 0 alone can never end the search (its bound is 0), so the first step covers rings
    // 0 and 1 together: every row of the 3 x 3 x 3 block as one contiguous range
    for (int r = 1; r <= max(rmax, 1); ++r) {
        const bool block = r == 1;
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= G2) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= G1) continue;
                const int64_t row = ((int64_t)z * G1 + y) * G0;
                if (block || dz == -r || dz == r || dy == -r || dy == r) {
                    scan_cells(start, sorted, row + max(cx - r, 0), row + min(cx + r, G0 - 1), qx, qy, qz, best);
                } else {
                    if (cx - r >= 0) scan_cells(start, sorted, row + cx - r, row + cx - r, qx, qy, qz, best);
                    if (r > 0 && cx + r < G0) scan_cells(start, sorted, row + cx + r, row + cx + r, qx, qy, qz, best);
                }
            }
        }
        // every unvisited point lies in a cell at least r + 1 rings away, beyond one of the six
        // faces of the searched block (a face on the grid's border has nothing beyond it)
        double reach = INFINITY;
        const int cc[3] = {cx, cy, cz}, gd[3] = {G0, G1, G2};
        const double qq[3] = {qx, qy, qz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (cc[a] - r > 0) reach = fmin(reach, qq[a] - (c->org[a] + (double)(cc[a] - r) * h));
            if (cc[a] + r < gd[a] - 1) reach = fmin(reach, (c->org[a] + (double)(cc[a] + r + 1) * h) - qq[a]);
        }
        reach -= eps;
        if (reach > 0.0 && best <= reach * reach) break;
    }
    const int i = __float_as_int(q.w);
    dist[i] = best < INFINITY ? (float)__dsqrt_rn(best) : INFINITY;
}

// dist may be one of the scale planes (each point's distance is read before it is written)
__global__ __launch_bounds__(NB) void k_init_params(const float* __restrict__ pts, const float* __restrict__ col,
                                                    int64_t n, int n_sh_rows, const float* dist,
                                                    float* __restrict__ mean, float* scale,
                                                    float* __restrict__ quat, float* __restrict__ opacity,
                                                    float* __restrict__ sh) {
    const int64_t i = (int64_t)blockIdx.x * NB + threadIdx.x;
    if (i >= n) return;
    const float s = dist[i];
    for (int a = 0; a < 3; ++a) mean[a * n + i] = pts[a * n + i], scale[a * n + i] = s;
    quat[i] = 1.f, quat[n + i] = 0.f, quat[2 * n + i] = 0.f, quat[3 * n + i] = 0.f;
    opacity[i] = 0.1f;
    for (int r = 0; r < n_sh_rows; ++r) {
        float v = 0.f;
        if (r < 3 && col) v = (float)(((double)col[r * n + i] - 0.5) / kY00);
        sh[r * n + i] = v;
    }
}

}  // namespace

size_t nn_workspace_bytes(int64_t n) {
    if (n <= 0) return 0;
    const int64_t cap = cell_cap(n);
    return a256(sizeof(GridCtrl)) + a256(sizeof(uint32_t) * 7 * BBOX_BLOCKS) + 2 * a256(sizeof(uint32_t) * (size_t)n) +
           a256(sizeof(uint32_t) * (size_t)(cap + 1)) + a256(sizeof(uint32_t) * (size_t)scan_blocks(cap + 1)) +
           sizeof(float4) * (size_t)n;
}

gs_status launch_nn_distance(const float* pts, int64_t n, float* dist, void* ws, hipStream_t s) {
    if (n == 0) return GS_OK;
    const NnLayout L = nn_layout(ws, n);
    const unsigned g = (unsigned)((n + NB - 1) / NB);
    const int64_t m = L.cap + 1, nb = scan_blocks(m);
    const unsigned nbb = std::min<unsigned>(g, BBOX_BLOCKS);
    hipLaunchKernelGGL(k_bbox, dim3(nbb), dim3(NB), 0, s, pts, n, L.bbox);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(NB), 0, s, L.bbox, (int)nbb, L.ctrl);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(1), 0, s, L.ctrl, L.cap);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + NB - 1) / NB)), dim3(NB), 0, s, L.start, m, 0u);
    hipLaunchKernelGGL(k_cell_count, dim3(g), dim3(NB), 0, s, pts, n, L.ctrl, L.cell, L.rank, L.start, dist);
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(SCAN_T), 0, s, L.start, m, L.totals);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(SCAN_T), 0, s, L.totals, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((m + NB - 1) / NB)), dim3(NB), 0, s, L.start, m, L.totals);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(NB), 0, s, pts, n, L.cell, L.rank, L.start, L.sorted);
    hipLaunchKernelGGL(k_nn, dim3(g), dim3(NB), 0, s, L.ctrl, L.start, L.sorted, L.cap, dist);
    return check_launch("nn_distance");
}

gs_status launch_init_gaussians(const float* pts, const float* col, int64_t n, int32_t sh_degree, float* mean,
                                float* scale, float* quat, float* opacity, float* sh, void* ws, hipStream_t s) {
    if (n == 0) return GS_OK;
    // the distances go to the last scale plane first
    float* dist = scale + 2 * n;
    gs_status st = launch_nn_distance(pts, n, dist, ws, s);
    if (st != GS_OK) return st;
    const int rows = (sh_degree + 1) * (sh_degree + 1) * 3;
    hipLaunchKernelGGL(k_init_params, dim3((unsigned)((n + NB - 1) / NB)), dim3(NB), 0, s, pts, col, n, rows, dist,
                       mean, scale, quat, opacity, sh);
    return check_launch("init_gaussians");
}

}  // namespace gs
