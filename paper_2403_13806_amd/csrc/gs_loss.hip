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
constexpr int MX = 76;                              // map row stride in LDS (16-byte rows)
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

__global__ __launch_bounds__(NTH) void k_ssim_stats(SsimArgs a) {
    __shared__ __align__(16) float2 s_in[IY][IX];
    __shared__ __align__(16) float s_h[5][IY][SX];
    __shared__ float red[8];
    const int tile = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const int x0 = (tile % a.tiles_x) * SX, y0 = (tile / a.tiles_x) * SY;
    const float* __restrict__ xp = a.x + p * a.plane;
    const float* __restrict__ yp = a.y + p * a.plane;

    constexpr int NLD = (IY * IX + NTH - 1) / NTH;
    float2 v[NLD];
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int i = tid + k * NTH;
        const int r = i / IX, c = i - r * IX;
        const int gy = y0 + r - SR, gx = x0 + c - SR;
        v[k] = make_float2(0.f, 0.f);
        if (i < IY * IX && gy >= 0 && gy < a.h && gx >= 0 && gx < a.w) {
            const int64_t o = (int64_t)gy * a.w + gx;
            v[k] = make_float2(xp[o], yp[o]);
        }
        sx += v[k].x, sy += v[k].y;
    }
    const float2 cs = block_sum2(sx, sy, red);
    const float cx = cs.x * (1.f / (IY * IX)), cy = cs.y * (1.f / (IY * IX));
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int i = tid + k * NTH;
        if (i < IY * IX) {
            const int r = i / IX, c = i - r * IX;
            s_in[r][c] = make_float2(v[k].x - cx, v[k].y - cy);
        }
    }
    if (tid == 0) a.shift[(int64_t)p * a.n_tiles + tile] = make_float2(cx, cy);
    __syncthreads();

    // horizontal window sums of x, y, x^2, y^2, xy: four adjacent columns per item
    for (int it = tid; it < IY * (SX / 4); it += NTH) {
        const int r = it >> 4, c0 = (it & 15) * 4;
        float vx[ST + 3], vy[ST + 3];
#pragma unroll
        for (int j = 0; j < (ST + 3) / 2; ++j) {
            const float4 q = *reinterpret_cast<const float4*>(&s_in[r][c0 + 2 * j]);
            vx[2 * j] = q.x, vy[2 * j] = q.y, vx[2 * j + 1] = q.z, vy[2 * j + 1] = q.w;
        }
        float o[5][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float sx = 0.f, sy = 0.f, sxx = 0.f, syy = 0.f, sxy = 0.f;
#pragma unroll
            for (int t = 0; t < ST; ++t) {
                const float gx = a.g[t] * vx[k + t], gy = a.g[t] * vy[k + t];
                sx += gx, sy += gy;
                sxx = fmaf(gx, vx[k + t], sxx);
                syy = fmaf(gy, vy[k + t], syy);
                sxy = fmaf(gx, vy[k + t], sxy);
            }
            o[0][k] = sx, o[1][k] = sy, o[2][k] = sxx, o[3][k] = syy, o[4][k] = sxy;
        }
#pragma unroll
        for (int m = 0; m < 5; ++m)
            *reinterpret_cast<float4*>(&s_h[m][r][c0]) = make_float4(o[m][0], o[m][1], o[m][2], o[m][3]);
    }
    __syncthreads();

    // vertical window sums: one column, four rows per thread
    const int c = tid & 63, r0 = (tid >> 6) * 4;
    float mom[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        float v[ST + 3];
#pragma unroll
        for (int j = 0; j < ST + 3; ++j) v[j] = s_h[m][r0 + j][c];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < ST; ++t) s = fmaf(a.g[t], v[k + t], s);
            mom[m][k] = s;
        }
    }

    float part = 0.f;
    const int gx = x0 + c;
    float* __restrict__ m0 = a.maps + p * a.plane;
    float* __restrict__ m1 = m0 + a.n_planes * a.plane;
    float* __restrict__ m2 = m1 + a.n_planes * a.plane;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int gy = y0 + r0 + k;
        if (gx < a.w && gy < a.h) {
            const float ma = mom[0][k], mb = mom[1][k];  // shifted means mu_x - cx, mu_y - cy
            const float vx = mom[2][k] - ma * ma, vy = mom[3][k] - mb * mb, cxy = mom[4][k] - ma * mb;
            const float mx = ma + cx, my = mb + cy;
            const float a1 = 2.f * mx * my + kC1, a2 = 2.f * cxy + kC2;
            const float b1 = mx * mx + my * my + kC1, b2 = vx + vy + kC2;
            const float rb = 1.f / (b1 * b2);
            const float s = a1 * a2 * rb;
            const float beta = -s * b1 * rb;   // -S / b2
            const float gamma = 2.f * a1 * rb;
            const float delta = 2.f * a2 * rb * (my - mx * a1 * b2 * rb);
            const float alpha_c = delta - 2.f * ma * beta - mb * gamma;
            const float2 xy = s_in[SR + r0 + k][SR + c];
            const float d = (xy.x - xy.y) + (cx - cy);
            part += (1.f - a.lam) * d * d + a.lam * (1.f - s);
            const int64_t o = (int64_t)gy * a.w + gx;
            m0[o] = alpha_c;
            m1[o] = beta;
            m2[o] = gamma;
        }
    }
    const float tot = block_sum(part, red);
    if (tid == 0) a.partial[(int64_t)p * a.n_tiles + tile] = tot;
}

__global__ __launch_bounds__(NTH) void k_ssim_grad(SsimArgs a) {
    __shared__ __align__(16) float s_m[3][IY][MX];
    __shared__ __align__(16) float s_h[3][IY][SX];
    __shared__ float red[4];
    const int tile = blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const int x0 = (tile % a.tiles_x) * SX, y0 = (tile / a.tiles_x) * SY;
    const int64_t maps_stride = a.n_planes * a.plane;
    const float* __restrict__ mp = a.maps + p * a.plane;
    const float2* __restrict__ sh = a.shift + (int64_t)p * a.n_tiles;
    const float2 cb = sh[tile];

    for (int i = tid; i < IY * IX; i += NTH) {
        const int r = i / IX, c = i - r * IX;
        const int gy = y0 + r - SR, gx = x0 + c - SR;
        float v0 = 0.f, v1 = 0.f, v2 = 0.f;
        if (gy >= 0 && gy < a.h && gx >= 0 && gx < a.w) {
            const int64_t o = (int64_t)gy * a.w + gx;
            v0 = mp[o], v1 = mp[o + maps_stride], v2 = mp[o + 2 * maps_stride];
            // alpha_c of a halo pixel is centred on its own tile's shift: move it to this tile's
            const float2 ca = sh[(gy / SY) * a.tiles_x + gx / SX];
            v0 = fmaf(2.f * (cb.x - ca.x), v1, fmaf(cb.y - ca.y, v2, v0));
        }
        s_m[0][r][c] = v0, s_m[1][r][c] = v1, s_m[2][r][c] = v2;
    }
    __syncthreads();

    for (int it = tid; it < IY * (SX / 4); it += NTH) {
        const int r = it >> 4, c0 = (it & 15) * 4;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float v[16];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 q = *reinterpret_cast<const float4*>(&s_m[m][r][c0 + 4 * j]);
                v[4 * j] = q.x, v[4 * j + 1] = q.y, v[4 * j + 2] = q.z, v[4 * j + 3] = q.w;
            }
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < ST; ++t) s = fmaf(a.g[t], v[k + t], s);
                o[k] = s;
            }
            *reinterpret_cast<float4*>(&s_h[m][r][c0]) = make_float4(o[0], o[1], o[2], o[3]);
        }
    }
    __syncthreads();

    const int c = tid & 63, r0 = (tid >> 6) * 4;
    float w3[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        float v[ST + 3];
#pragma unroll
        for (int j = 0; j < ST + 3; ++j) v[j] = s_h[m][r0 + j][c];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < ST; ++t) s = fmaf(a.g[t], v[k + t], s);
            w3[m][k] = s;
        }
    }

    const int gx = x0 + c;
    const float* __restrict__ xp = a.x + p * a.plane;
    const float* __restrict__ yp = a.y + p * a.plane;
    float* __restrict__ dp = a.dl + p * a.plane;
    const float c_l2 = 2.f * (1.f - a.lam) * a.inv_n, c_s = a.lam * a.inv_n;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int gy = y0 + r0 + k;
        if (gx < a.w && gy < a.h) {
            const int64_t o = (int64_t)gy * a.w + gx;
            const float xv = xp[o], yv = yp[o];
            const float ds = fmaf(2.f * (xv - cb.x), w3[1][k], fmaf(yv - cb.y, w3[2][k], w3[0][k]));
            dp[o] = c_l2 * (xv - yv) - c_s * ds;
        }
    }

    // workgroup (0, 0): the loss, from the first launch's tile partials in a fixed order
    if (tile == 0 && p == 0 && a.loss) {
        const int64_t n_part = (int64_t)a.n_planes * a.n_tiles;
        float s = 0.f;
        for (int64_t i = tid; i < n_part; i += NTH) s += a.partial[i];
        __syncthreads();
        const float tot = block_sum(s, red);
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
    const dim3 grid((unsigned)a.n_tiles, (unsigned)n_planes);
    hipLaunchKernelGGL(k_ssim_stats, grid, dim3(NTH), 0, s, a);
    gs_status st = check_launch("ssim_loss_grad (statistics)");
    if (st != GS_OK) return st;
    hipLaunchKernelGGL(k_ssim_grad, grid, dim3(NTH), 0, s, a);
    return check_launch("ssim_loss_grad (gradient)");
}

}  // namespace gs
