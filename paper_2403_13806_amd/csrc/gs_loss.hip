// Training loss of the point representation (Sec. 3.2): L = (1 - lambda) sum (x - y)^2 / n +
// lambda sum (1 - SSIM) / n, lambda = 0.2 in the paper, and its gradient with respect to the
// rendered image x. SSIM is the per-pixel structural similarity of Wang et al.: local means,
// variances and covariance from an 11 x 11 Gaussian window (sigma 1.5) with zero padding,
// C1 = 0.01^2, C2 = 0.03^2.
//
// Two HBM-bound launches over 64 x 16 pixel tiles of every plane, both LDS-tiled separable
// window sums (a horizontal pass into LDS, then a vertical pass in registers):
//   k_ssim_stats  x, y (+5 pixel halo) -> local moments -> SSIM, the loss partial of the
//                 tile, and three FP32 maps: beta = dS/dE[x^2], gamma = dS/dE[xy] and the
//                 mean term alpha_c (below).
//   k_ssim_grad   the three maps (+5 pixel halo) -> their window sums (the adjoint of the
//                 local sums) -> dL/dx; workgroup (0, 0) also adds the tile partials, in a
//                 fixed order, into the loss word.
// FP32 accuracy. Each tile shifts x and y by the mean (cx, cy) of its input window (padding
// counts as 0) before the window sums, so variances come from E[x'^2] - E[x']^2 of small
// numbers: without it, flat or saturated areas, where the variance is 0 but E[x^2] is up to 1,
// leave a rounding residue of order 1e-7 against C2 = 9e-4. The gradient is
//   dS/dx_q = sum_p w(p - q) (alpha_p + 2 x_q beta_p + y_q gamma_p),
// alpha_p = dS/dmu_x at fixed E[x^2], E[xy], a difference of terms up to 2 / C2. It is carried
// centred: alpha_c = alpha + 2 cx beta + cy gamma = delta - 2 (mu_x - cx) beta - (mu_y - cy) gamma
// with delta = dS/dmu_x at fixed variances and covariance, all small in smooth areas; the
// gradient launch moves the halo's alpha_c to its own tile's shift and applies x_q - cx.
// Algorithmic traffic: 8 bytes read and 12 written per pixel by the first launch, 20 read and
// 4 written by the second (plus 8 bytes of shift per tile).
#include <cmath>

#include "gs_device.hpp"

namespace gs {

namespace {

constexpr int SX = 64, SY = 16, SR = 5, ST = 2 * SR + 1;
constexpr int IX = SX + 2 * SR, IY = SY + 2 * SR;  // 74 x 26 input window of a tile
constexpr int NTH = 256;

struct SsimArgs {
    const float* x;
    const float* y;
    float* maps;      // [3][planes][H][W]
    float* partial;   // [planes][tiles]
    float2* shift;    // [planes][tiles] (cx, cy) of each tile
    float* dl;
    float* loss;
    int64_t plane;    // H * W
    int32_t h, w, tiles_x, n_tiles, n_planes;
    int32_t vec;      // rows of 4 pixels are 16-byte aligned in x, y and dl (w % 4 == 0, aligned bases)
    float lam, inv_n;
    float g[ST];      // normalised 1D window
};

constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

__device__ __forceinline__ float2 block_sum2(float u, float v, float* red) {
    const float su = wave_sum(u), sv = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = su, red[4 + (threadIdx.x >> 6)] = sv;
    __syncthreads();
    return make_float2((red[0] + red[1]) + (red[2] + red[3]), (red[4] + red[5]) + (red[6] + red[7]));
}

__device__ __forceinline__ float block_sum(float v, float* red) {
    const float s = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// One job = one tile of one plane; jobs are numbered plane-major.
struct Job {
    int64_t p;
    int tile, x0, y0;
    bool interior;  // the whole input window lies inside the plane
};

__device__ __forceinline__ Job job_of(const SsimArgs& a, int64_t j) {
    Job jb;
    jb.p = j / a.n_tiles;
    jb.tile = (int)(j - jb.p * a.n_tiles);
    jb.x0 = (jb.tile % a.tiles_x) * SX;
    jb.y0 = (jb.tile / a.tiles_x) * SY;
    jb.interior = jb.x0 >= SR && jb.x0 + SX + SR <= a.w && jb.y0 >= SR && jb.y0 + SY + SR <= a.h;
    return jb;
}

constexpr int NLD = (IY * IX + NTH - 1) / NTH;  // window elements per thread
constexpr int NV = 4 * IX;                       // vertical-pass items: 74 columns x 4 row groups
constexpr int VX = 76;                           // row stride of the vertical sums in LDS

// window element k of this thread: row r, column c of the IY x IX window
__device__ __forceinline__ void elem(int k, int& r, int& c) {
    const int i = threadIdx.x + k * NTH;
    r = i / IX;
    c = i - r * IX;
}

// x and y over a job's input window (zero outside the plane), into registers
__device__ __forceinline__ void load_window(const SsimArgs& a, const Job& jb, float2 (&v)[NLD]) {
    const int64_t base = jb.p * a.plane + (int64_t)(jb.y0 - SR) * a.w + (jb.x0 - SR);
    const float* __restrict__ xp = a.x + base;
    const float* __restrict__ yp = a.y + base;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        int r, c;
        elem(k, r, c);
        const int o = r * a.w + c;
        const bool in = (k + 1) * NTH <= IY * IX || r < IY;
        v[k] = make_float2(0.f, 0.f);
        if (jb.interior) {
            if (in) v[k] = make_float2(xp[o], yp[o]);
        } else if (in && (unsigned)(jb.y0 + r - SR) < (unsigned)a.h && (unsigned)(jb.x0 + c - SR) < (unsigned)a.w) {
            v[k] = make_float2(xp[o], yp[o]);
        }
    }
}

// Persistent grid over the jobs (round k of workgroup b takes job k G + xcd_order(b, G), so
// each XCD works on a band of neighbouring tiles); the next job's window is loaded into
// registers while the current one is computed. Vertical sums first (over the window's 74 columns), then
// horizontal sums (over the tile's 16 rows): the halo costs 74/64 of the first pass only.
__global__ __launch_bounds__(NTH) void k_ssim_stats(SsimArgs a) {
    __shared__ __align__(16) float2 s_in[IY][IX];
    __shared__ __align__(16) float s_v[5][SY][VX];
    __shared__ float red[8];
    const int tid = threadIdx.x;
    const int64_t n_jobs = (int64_t)a.n_planes * a.n_tiles;
    const bool vec = a.vec;
    float2 v[NLD];
    int64_t j = xcd_order(blockIdx.x, gridDim.x);  // halos of neighbouring tiles share an L2
    if (j < n_jobs) load_window(a, job_of(a, j), v);
    for (; j < n_jobs; j += gridDim.x) {
        const Job jb = job_of(a, j);
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int k = 0; k < NLD; ++k) sx += v[k].x, sy += v[k].y;
        const float2 cs = block_sum2(sx, sy, red);
        const float cx = cs.x * (1.f / (IY * IX)), cy = cs.y * (1.f / (IY * IX));
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            int r, c;
            elem(k, r, c);
            if ((k + 1) * NTH <= IY * IX || r < IY) s_in[r][c] = make_float2(v[k].x - cx, v[k].y - cy);
        }
        if (tid == 0) a.shift[j] = make_float2(cx, cy);
        __syncthreads();
        if (j + gridDim.x < n_jobs) load_window(a, job_of(a, j + gridDim.x), v);

        // vertical window sums of x, y, x^2, y^2, xy: one column, four output rows per item
        for (int it = tid; it < NV; it += NTH) {
            const int g4 = it / IX, c = it - g4 * IX, r0 = 4 * g4;
            float vx[ST + 3], vy[ST + 3], pxx[ST + 3], pyy[ST + 3], pxy[ST + 3];
#pragma unroll
            for (int q = 0; q < ST + 3; ++q) {
                const float2 e = s_in[r0 + q][c];
                vx[q] = e.x, vy[q] = e.y, pxx[q] = e.x * e.x, pyy[q] = e.y * e.y, pxy[q] = e.x * e.y;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float hx = 0.f, hy = 0.f, hxx = 0.f, hyy = 0.f, hxy = 0.f;
#pragma unroll
                for (int t = 0; t < ST; ++t) {
                    hx = fmaf(a.g[t], vx[k + t], hx);
                    hy = fmaf(a.g[t], vy[k + t], hy);
                    hxx = fmaf(a.g[t], pxx[k + t], hxx);
                    hyy = fmaf(a.g[t], pyy[k + t], hyy);
                    hxy = fmaf(a.g[t], pxy[k + t], hxy);
                }
                s_v[0][r0 + k][c] = hx, s_v[1][r0 + k][c] = hy, s_v[2][r0 + k][c] = hxx;
                s_v[3][r0 + k][c] = hyy, s_v[4][r0 + k][c] = hxy;
            }
        }
        __syncthreads();

        // horizontal window sums: one row, four adjacent output columns per thread
        const int r = tid >> 4, c0 = (tid & 15) * 4;
        float mom[5][4];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            float w[16];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 f4 = *reinterpret_cast<const float4*>(&s_v[m][r][c0 + 4 * u]);
                w[4 * u] = f4.x, w[4 * u + 1] = f4.y, w[4 * u + 2] = f4.z, w[4 * u + 3] = f4.w;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < ST; ++t) acc = fmaf(a.g[t], w[k + t], acc);
                mom[m][k] = acc;
            }
        }

        float part = 0.f;
        float out[3][4];
        const int gy = jb.y0 + r, gx0 = jb.x0 + c0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float ma = mom[0][k], mb = mom[1][k];  // shifted means mu_x - cx, mu_y - cy
            const float vx = mom[2][k] - ma * ma, vy = mom[3][k] - mb * mb, cxy = mom[4][k] - ma * mb;
            const float mx = ma + cx, my = mb + cy;
            const float a1 = 2.f * mx * my + kC1, a2 = 2.f * cxy + kC2;
            const float b1 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
            const float rb = __builtin_amdgcn_rcpf(b1 * b2);
            const float ss = a1 * a2 * rb;
            const float beta = -ss * b1 * rb;  // -S / b2
            const float gamma = 2.f * a1 * rb;
            const float delta = 2.f * a2 * rb * (my - mx * a1 * b2 * rb);
            out[0][k] = delta - 2.f * ma * beta - mb * gamma;  // alpha_c
            out[1][k] = beta;
            out[2][k] = gamma;
            const float2 e = s_in[SR + r][SR + c0 + k];
            const float d = (e.x - e.y) + (cx - cy);
            if (gy < a.h && gx0 + k < a.w) part += (1.f - a.lam) * d * d + a.lam * (1.f - ss);
        }
        if (gy < a.h) {
            const int64_t o = jb.p * a.plane + (int64_t)gy * a.w + gx0;
            const int64_t ms = a.n_planes * a.plane;
            if (vec && gx0 + 4 <= a.w) {
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    *reinterpret_cast<float4*>(a.maps + m * ms + o) = make_float4(out[m][0], out[m][1], out[m][2], out[m][3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (gx0 + k < a.w) {
#pragma unroll
                        for (int m = 0; m < 3; ++m) a.maps[m * ms + o + k] = out[m][k];
                    }
            }
        }
        const float tot = block_sum(part, red);
        if (tid == 0) a.partial[j] = tot;
        __syncthreads();  // s_in, s_v and red are rewritten by the next job
    }
}

// the three maps over a job's input window, and the shift of each element's own tile
struct MapWindow {
    float m[3][NLD];
    float2 ca[NLD];
};

__device__ __forceinline__ void load_maps(const SsimArgs& a, const Job& jb, MapWindow& w) {
    const int64_t stride = a.n_planes * a.plane;
    const float* __restrict__ mp = a.maps + jb.p * a.plane + (int64_t)(jb.y0 - SR) * a.w + (jb.x0 - SR);
    const float2* __restrict__ sh = a.shift + jb.p * a.n_tiles;
    const float2 cb = sh[jb.tile];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        int r, c;
        elem(k, r, c);
        const int o = r * a.w + c;
        const bool in = ((k + 1) * NTH <= IY * IX || r < IY) &&
                        (jb.interior || ((unsigned)(jb.y0 + r - SR) < (unsigned)a.h &&
                                         (unsigned)(jb.x0 + c - SR) < (unsigned)a.w));
        w.m[0][k] = w.m[1][k] = w.m[2][k] = 0.f;
        w.ca[k] = cb;
        if (in) {
            w.m[0][k] = mp[o], w.m[1][k] = mp[o + stride], w.m[2][k] = mp[o + 2 * stride];
            // the tile of a halo element: one row / column of tiles away at most
            const int dty = r < SR ? -1 : (r >= SY + SR ? 1 : 0);
            const int dtx = c < SR ? -1 : (c >= SX + SR ? 1 : 0);
            if (dty | dtx) w.ca[k] = sh[jb.tile + dty * a.tiles_x + dtx];
        }
    }
}

// LDS holds the maps window, then the vertical sums; the horizontal sums stay in registers.
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_ssim_grad(SsimArgs a) {
    __shared__ float s_m[3][IY][IX];
    __shared__ __align__(16) float s_v[3][SY][VX];
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int64_t n_jobs = (int64_t)a.n_planes * a.n_tiles;
    const bool vec = a.vec;
    MapWindow w;
    int64_t j = xcd_order(blockIdx.x, gridDim.x);  // halos of neighbouring tiles share an L2
    if (j < n_jobs) load_maps(a, job_of(a, j), w);
    for (; j < n_jobs; j += gridDim.x) {
        const Job jb = job_of(a, j);
        const float2 cb = a.shift[j];
#pragma unroll
        for (int k = 0; k < NLD; ++k) {
            int r, c;
            elem(k, r, c);
            if ((k + 1) * NTH <= IY * IX || r < IY) {
                // alpha_c of a halo element is centred on its own tile's shift: move it to this tile's
                s_m[0][r][c] = fmaf(2.f * (cb.x - w.ca[k].x), w.m[1][k], fmaf(cb.y - w.ca[k].y, w.m[2][k], w.m[0][k]));
                s_m[1][r][c] = w.m[1][k];
                s_m[2][r][c] = w.m[2][k];
            }
        }
        __syncthreads();
        if (j + gridDim.x < n_jobs) load_maps(a, job_of(a, j + gridDim.x), w);

        for (int it = tid; it < NV; it += NTH) {
            const int g4 = it / IX, c = it - g4 * IX, r0 = 4 * g4;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                float vv[ST + 3];
#pragma unroll
                for (int q = 0; q < ST + 3; ++q) vv[q] = s_m[m][r0 + q][c];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    float acc = 0.f;
#pragma unroll
                    for (int t = 0; t < ST; ++t) acc = fmaf(a.g[t], vv[k + t], acc);
                    s_v[m][r0 + k][c] = acc;
                }
            }
        }
        __syncthreads();

        const int r = tid >> 4, c0 = (tid & 15) * 4;
        float w3[3][4];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float vv[16];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 f4 = *reinterpret_cast<const float4*>(&s_v[m][r][c0 + 4 * u]);
                vv[4 * u] = f4.x, vv[4 * u + 1] = f4.y, vv[4 * u + 2] = f4.z, vv[4 * u + 3] = f4.w;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < ST; ++t) acc = fmaf(a.g[t], vv[k + t], acc);
                w3[m][k] = acc;
            }
        }

        const int gy = jb.y0 + r, gx0 = jb.x0 + c0;
        const float c_l2 = 2.f * (1.f - a.lam) * a.inv_n, c_s = a.lam * a.inv_n;
        if (gy < a.h) {
            const int64_t o = jb.p * a.plane + (int64_t)gy * a.w + gx0;
            if (vec && gx0 + 4 <= a.w) {
                const float4 x4 = *reinterpret_cast<const float4*>(a.x + o);
                const float4 y4 = *reinterpret_cast<const float4*>(a.y + o);
                const float xv[4] = {x4.x, x4.y, x4.z, x4.w}, yv[4] = {y4.x, y4.y, y4.z, y4.w};
                float dv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float ds = fmaf(2.f * (xv[k] - cb.x), w3[1][k], fmaf(yv[k] - cb.y, w3[2][k], w3[0][k]));
                    dv[k] = c_l2 * (xv[k] - yv[k]) - c_s * ds;
                }
                *reinterpret_cast<float4*>(a.dl + o) = make_float4(dv[0], dv[1], dv[2], dv[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (gx0 + k < a.w) {
                        const float xv = a.x[o + k], yv = a.y[o + k];
                        const float ds = fmaf(2.f * (xv - cb.x), w3[1][k], fmaf(yv - cb.y, w3[2][k], w3[0][k]));
                        a.dl[o + k] = c_l2 * (xv - yv) - c_s * ds;
                    }
            }
        }
        __syncthreads();  // s_m and s_v are rewritten by the next job
    }

    // workgroup 0: the loss, from the first launch's tile partials in a fixed order
    if (blockIdx.x == 0 && a.loss) {
        float acc = 0.f;
        for (int64_t i = tid; i < n_jobs; i += NTH) acc += a.partial[i];
        const float tot = block_sum(acc, red);
        if (tid == 0) atomicAdd(a.loss, tot * a.inv_n);
    }
}

}  // namespace

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t ssim_workspace_bytes(int32_t n_planes, int32_t h, int32_t w) {
    if (n_planes <= 0 || h <= 0 || w <= 0) return 0;
    const size_t tiles = (size_t)div_up(w, SX) * (size_t)div_up(h, SY) * (size_t)n_planes;
    const size_t maps = 3 * sizeof(float) * (size_t)n_planes * (size_t)h * (size_t)w;
    return align256(maps) + align256(sizeof(float) * tiles) + sizeof(float2) * tiles;
}

gs_status launch_ssim_loss_grad(const float* img, const float* target, int32_t n_planes, int32_t h, int32_t w,
                                int64_t n_norm, float lam, float* dl, float* loss, void* ws, hipStream_t s) {
    if (n_planes == 0) return GS_OK;
    SsimArgs a{};
    a.x = img, a.y = target, a.dl = dl, a.loss = loss;
    a.plane = (int64_t)h * w;
    a.h = h, a.w = w;
    a.tiles_x = div_up(w, SX);
    a.n_tiles = a.tiles_x * div_up(h, SY);
    a.n_planes = n_planes;
    a.lam = lam;
    a.inv_n = (float)(1.0 / (double)n_norm);
    auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    a.vec = (w % 4 == 0) && al16(img) && al16(target) && al16(dl);
    const size_t maps = 3 * sizeof(float) * (size_t)n_planes * (size_t)a.plane;
    const size_t tiles = (size_t)a.n_tiles * (size_t)n_planes;
    a.maps = static_cast<float*>(ws);
    a.partial = reinterpret_cast<float*>(static_cast<char*>(ws) + align256(maps));
    a.shift = reinterpret_cast<float2*>(static_cast<char*>(ws) + align256(maps) + align256(sizeof(float) * tiles));
    double g[ST], sum = 0.0;
    for (int t = 0; t < ST; ++t) {
        const double d = t - SR;
        g[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[t];
    }
    for (int t = 0; t < ST; ++t) a.g[t] = (float)(g[t] / sum);
    const int64_t n_jobs = (int64_t)a.n_tiles * n_planes;
    const int grid_a = persistent_grid(reinterpret_cast<const void*>(k_ssim_stats), NTH, n_jobs);
    const int grid_b = persistent_grid(reinterpret_cast<const void*>(k_ssim_grad), NTH, n_jobs);
    hipLaunchKernelGGL(k_ssim_stats, dim3(grid_a), dim3(NTH), 0, s, a);
    gs_status st = check_launch("ssim_loss_grad (statistics)");
    if (st != GS_OK) return st;
    hipLaunchKernelGGL(k_ssim_grad, dim3(grid_b), dim3(NTH), 0, s, a);
    return check_launch("ssim_loss_grad (gradient)");
}

}  // namespace gs
