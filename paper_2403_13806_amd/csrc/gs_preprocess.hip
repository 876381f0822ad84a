// Projection of 3D Gaussians into pinhole views (Sec. 3.2: Sigma = R S S^T R^T,
// Sigma' = J M Sigma M^T J^T) and its reverse-mode derivative.
//
// One thread per (view, Gaussian). Everything that decides a key or a pixel's support
// (camera-space mean, projected mean, 2D covariance, conic, support radius, tile
// rectangle) is computed in FP64: on CDNA4 an FP64 FMA issues at the same rate as an
// unpacked FP32 one, and FP64 geometry makes the tile keys reproducible bit for bit.
// Contraction into FMAs is switched off for that part so every operation is the
// correctly rounded IEEE operation in the stated order. SH colour is FP32.
#include <math.h>

#include "gs_device.hpp"

namespace gs {

// ---------------------------------------------------------------------------------------
// Real SH basis up to degree 3 (orthonormal, Condon-Shortley phase), index l*l + l + m,
// written as polynomials in the unit direction (x, y, z):
//   C0 = 1/(2 sqrt(pi)), C1 = sqrt(3/(4 pi)), C2a = sqrt(15/(4 pi)), C2b = sqrt(5/(16 pi)),
//   C2c = sqrt(15/(16 pi)), C3a = sqrt(35/(32 pi)), C3b = sqrt(105/(4 pi)),
//   C3c = sqrt(21/(32 pi)), C3d = sqrt(7/(16 pi)), C3e = sqrt(105/(16 pi)).
// ---------------------------------------------------------------------------------------
#define SH_C0 0.28209479177387814f
#define SH_C1 0.4886025119029199f
#define SH_C2A 1.0925484305920792f
#define SH_C2B 0.31539156525252005f
#define SH_C2C 0.5462742152960396f
#define SH_C3A 0.5900435899266435f
#define SH_C3B 2.890611442640554f
#define SH_C3C 0.4570457994644658f
#define SH_C3D 0.3731763325901154f
#define SH_C3E 1.445305721320277f

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float Y[16]) {
    Y[0] = SH_C0;
    if (deg < 1) return;
    Y[1] = -SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = -SH_C1 * x;
    if (deg < 2) return;
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_C2A * x * y;
    Y[5] = -SH_C2A * y * z;
    Y[6] = SH_C2B * (3.f * zz - 1.f);
    Y[7] = -SH_C2A * x * z;
    Y[8] = SH_C2C * (xx - yy);
    if (deg < 3) return;
    Y[9] = -SH_C3A * y * (3.f * xx - yy);
    Y[10] = SH_C3B * x * y * z;
    Y[11] = -SH_C3C * y * (5.f * zz - 1.f);
    Y[12] = SH_C3D * z * (5.f * zz - 3.f);
    Y[13] = -SH_C3C * x * (5.f * zz - 1.f);
    Y[14] = SH_C3E * z * (xx - yy);
    Y[15] = -SH_C3A * x * (xx - 3.f * yy);
}

// sum_k (s k_k) grad Y_k(x, y, z): the gradient of each basis polynomial above with respect
// to (x, y, z), contracted with the weights s k_k as it is formed (no 16 x 3 table is held)
__device__ __forceinline__ void sh_wgrad(int deg, float x, float y, float z, const float* kk, float sc, float gd[3]) {
    float w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = (k < (deg + 1) * (deg + 1)) ? kk[k] * sc : 0.f;
    gd[0] = gd[1] = gd[2] = 0.f;
    if (deg < 1) return;
    gd[1] -= SH_C1 * w[1];
    gd[2] += SH_C1 * w[2];
    gd[0] -= SH_C1 * w[3];
    if (deg < 2) return;
    gd[0] += SH_C2A * y * w[4];
    gd[1] += SH_C2A * x * w[4];
    gd[1] -= SH_C2A * z * w[5];
    gd[2] -= SH_C2A * y * w[5];
    gd[2] += SH_C2B * 6.f * z * w[6];
    gd[0] -= SH_C2A * z * w[7];
    gd[2] -= SH_C2A * x * w[7];
    gd[0] += SH_C2C * 2.f * x * w[8];
    gd[1] -= SH_C2C * 2.f * y * w[8];
    if (deg < 3) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    gd[0] -= SH_C3A * 6.f * x * y * w[9];
    gd[1] -= SH_C3A * (3.f * xx - 3.f * yy) * w[9];
    gd[0] += SH_C3B * y * z * w[10];
    gd[1] += SH_C3B * x * z * w[10];
    gd[2] += SH_C3B * x * y * w[10];
    gd[1] -= SH_C3C * (5.f * zz - 1.f) * w[11];
    gd[2] -= SH_C3C * 10.f * y * z * w[11];
    gd[2] += SH_C3D * (15.f * zz - 3.f) * w[12];
    gd[0] -= SH_C3C * (5.f * zz - 1.f) * w[13];
    gd[2] -= SH_C3C * 10.f * x * z * w[13];
    gd[0] += SH_C3E * 2.f * x * z * w[14];
    gd[1] -= SH_C3E * 2.f * y * z * w[14];
    gd[2] += SH_C3E * (xx - yy) * w[14];
    gd[0] -= SH_C3A * (3.f * xx - 3.f * yy) * w[15];
    gd[1] += SH_C3A * 6.f * x * y * w[15];
}

// ---------------------------------------------------------------------------------------
// FP64 projection of one Gaussian into one camera.
// ---------------------------------------------------------------------------------------
struct Proj {
    double x, y, z;      // camera-space mean
    double u, v;         // projected mean
    double qn;           // |q|
    double qh[4];        // q / |q|
    double Rq[3][3];     // rotation of the Gaussian
    double Sg[3][3];     // 3D covariance
    double T[2][3];      // J R
    double sxx, sxy, syy;
    double det;
    double qmax, hx, hy;
};

// The eleven geometric parameters of one Gaussian (position, scale, quaternion, opacity).
struct Geom {
    float p[3], s[3], q[4], o;
};

__device__ __forceinline__ Geom load_geom(const float* __restrict__ mean, const float* __restrict__ scale,
                                          const float* __restrict__ quat, const float* __restrict__ opac,
                                          int64_t n_all, int64_t i) {
    Geom g;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.p[k] = mean[k * n_all + i];
        g.s[k] = scale[k * n_all + i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) g.q[k] = quat[k * n_all + i];
    g.o = opac[i];
    return g;
}

// Returns false when the Gaussian is culled. The operation order below is part of the
// tile-key definition; do not reassociate.
__device__ bool project_vals(const gs_camera& cam, const gs_params& p, const Geom& gm, Proj& P, double& o) {
#pragma clang fp contract(off)
    const double p0 = gm.p[0], p1 = gm.p[1], p2 = gm.p[2];
    const double s0 = gm.s[0], s1 = gm.s[1], s2 = gm.s[2];
    const double q0 = gm.q[0], q1 = gm.q[1], q2 = gm.q[2], q3 = gm.q[3];
    o = gm.o;
    if (!(isfinite(p0) && isfinite(p1) && isfinite(p2) && isfinite(s0) && isfinite(s1) && isfinite(s2) &&
          isfinite(q0) && isfinite(q1) && isfinite(q2) && isfinite(q3) && isfinite(o)))
        return false;
    const double R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2], R3 = cam.R[3], R4 = cam.R[4], R5 = cam.R[5],
                 R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
    P.x = (((R0 * p0) + (R1 * p1)) + (R2 * p2)) + (double)cam.t[0];
    P.y = (((R3 * p0) + (R4 * p1)) + (R5 * p2)) + (double)cam.t[1];
    P.z = (((R6 * p0) + (R7 * p1)) + (R8 * p2)) + (double)cam.t[2];
    if (!(P.z > (double)cam.znear)) return false;
    if (!(o >= (double)p.alpha_min)) return false;
    const double fx = cam.fx, fy = cam.fy;
    P.u = ((fx * P.x) / P.z) + (double)cam.cx;
    P.v = ((fy * P.y) / P.z) + (double)cam.cy;
    const double hw = 0.5 * (double)cam.width, hh = 0.5 * (double)cam.height;
    const double guard = p.guard;
    if (!(fabs(P.u - hw) <= guard * hw)) return false;
    if (!(fabs(P.v - hh) <= guard * hh)) return false;
    P.qn = sqrt((((q0 * q0) + (q1 * q1)) + (q2 * q2)) + (q3 * q3));
    if (!(P.qn > 0.0)) return false;
    const double w = q0 / P.qn, x = q1 / P.qn, y = q2 / P.qn, z = q3 / P.qn;
    P.qh[0] = w; P.qh[1] = x; P.qh[2] = y; P.qh[3] = z;
    P.Rq[0][0] = 1.0 - 2.0 * ((y * y) + (z * z));
    P.Rq[0][1] = 2.0 * ((x * y) - (w * z));
    P.Rq[0][2] = 2.0 * ((x * z) + (w * y));
    P.Rq[1][0] = 2.0 * ((x * y) + (w * z));
    P.Rq[1][1] = 1.0 - 2.0 * ((x * x) + (z * z));
    P.Rq[1][2] = 2.0 * ((y * z) - (w * x));
    P.Rq[2][0] = 2.0 * ((x * z) - (w * y));
    P.Rq[2][1] = 2.0 * ((y * z) + (w * x));
    P.Rq[2][2] = 1.0 - 2.0 * ((x * x) + (y * y));
    const double ss[3] = {s0 * s0, s1 * s1, s2 * s2};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            P.Sg[a][b] = (((P.Rq[a][0] * ss[0]) * P.Rq[b][0]) + ((P.Rq[a][1] * ss[1]) * P.Rq[b][1])) +
                         ((P.Rq[a][2] * ss[2]) * P.Rq[b][2]);
    const double J00 = fx / P.z, J02 = -((fx * P.x) / (P.z * P.z));
    const double J11 = fy / P.z, J12 = -((fy * P.y) / (P.z * P.z));
    const double Rc[9] = {R0, R1, R2, R3, R4, R5, R6, R7, R8};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.T[0][k] = (J00 * Rc[0 * 3 + k]) + (J02 * Rc[2 * 3 + k]);
        P.T[1][k] = (J11 * Rc[1 * 3 + k]) + (J12 * Rc[2 * 3 + k]);
    }
    double M[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int l = 0; l < 3; ++l)
            M[a][l] = ((P.T[a][0] * P.Sg[0][l]) + (P.T[a][1] * P.Sg[1][l])) + (P.T[a][2] * P.Sg[2][l]);
    const double S00 = ((M[0][0] * P.T[0][0]) + (M[0][1] * P.T[0][1])) + (M[0][2] * P.T[0][2]);
    const double S01 = ((M[0][0] * P.T[1][0]) + (M[0][1] * P.T[1][1])) + (M[0][2] * P.T[1][2]);
    const double S11 = ((M[1][0] * P.T[1][0]) + (M[1][1] * P.T[1][1])) + (M[1][2] * P.T[1][2]);
    const double lp = p.lowpass;
    P.sxx = S00 + lp;
    P.syy = S11 + lp;
    P.sxy = S01;
    P.det = (P.sxx * P.syy) - (P.sxy * P.sxy);
    if (!(P.det > 0.0)) return false;
    const double kappa = p.kappa;
    P.qmax = kappa * kappa;
    const double ql = 2.0 * log(o / (double)p.alpha_min);
    if (ql < P.qmax) P.qmax = ql;
    P.hx = sqrt(P.qmax * P.sxx);
    P.hy = sqrt(P.qmax * P.syy);
    return true;
}

__device__ __forceinline__ bool project_one(const gs_camera& cam, const gs_params& p, const float* __restrict__ mean,
                                            const float* __restrict__ scale, const float* __restrict__ quat,
                                            const float* __restrict__ opac, int64_t n_all, int64_t i, Proj& P,
                                            double& o) {
    return project_vals(cam, p, load_geom(mean, scale, quat, opac, n_all, i), P, o);
}

// unit direction (world) from the camera centre C = -R^T t to the mean, and |mean - C|
__device__ __forceinline__ void view_dir(const gs_camera& cam, double p0, double p1, double p2, float d[3],
                                         double& len) {
    double C[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        C[k] = -((((double)cam.R[0 * 3 + k] * cam.t[0]) + ((double)cam.R[1 * 3 + k] * cam.t[1])) +
                 ((double)cam.R[2 * 3 + k] * cam.t[2]));
    const double a = p0 - C[0], b = p1 - C[1], c = p2 - C[2];
    len = sqrt(a * a + b * b + c * c);
    d[0] = (float)(a / len);
    d[1] = (float)(b / len);
    d[2] = (float)(c / len);
}

struct PreArgs {
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opac;
    const float* sh;
    int64_t n_all;
    int deg;
    const gs_camera* cams;
    gs_params p;
    int tile_w, tile_h;
    const int32_t* subset;
    int64_t n;
    int n_views;
    int want_color;
    gs_splat* splat;
    float* depth;
    uint64_t* rect;
    uint32_t* count;
};

// The geometric part of entry o (view cam): writes its count and, when it meets some tile, its
// depth and tile rectangle; returns the count.
__device__ __forceinline__ uint32_t project_geom(const PreArgs& a, const gs_camera& cam, int64_t o, const Geom& gm,
                                                 Proj& P, double& op) {
    if (!project_vals(cam, a.p, gm, P, op)) {
        a.count[o] = 0u;
        return 0u;
    }
    // tile rectangle of the support's bounding box, widened by 2^-16 px
    double rx0, rx1, ry0, ry1;
    {
#pragma clang fp contract(off)
        const double eps = 1.0 / 65536.0;
        const double tw = a.tile_w, th = a.tile_h;
        rx0 = floor(((P.u - P.hx) - eps) / tw);
        rx1 = floor(((P.u + P.hx) + eps) / tw);
        ry0 = floor(((P.v - P.hy) - eps) / th);
        ry1 = floor(((P.v + P.hy) + eps) / th);
    }
    const int tiles_x = div_up(cam.width, a.tile_w), tiles_y = div_up(cam.height, a.tile_h);
    rx0 = fmax(rx0, 0.0);
    ry0 = fmax(ry0, 0.0);
    rx1 = fmin(rx1, (double)(tiles_x - 1));
    ry1 = fmin(ry1, (double)(tiles_y - 1));
    uint32_t cnt = 0;
    if (rx1 >= rx0 && ry1 >= ry0) cnt = (uint32_t)((rx1 - rx0 + 1.0) * (ry1 - ry0 + 1.0));
    a.count[o] = cnt;
    if (cnt == 0) return 0u;
    a.depth[o] = (float)P.z;
    a.rect[o] = (uint64_t)(uint32_t)rx0 | ((uint64_t)(uint32_t)ry0 << 16) | ((uint64_t)(uint32_t)rx1 << 32) |
                ((uint64_t)(uint32_t)ry1 << 48);
    return cnt;
}

// Colour of a Gaussian at position p seen by cam from its SH coefficients shv (Sec. 3.2).
template <int DEG>
__device__ __forceinline__ void sh_colour(const gs_camera& cam, float p0, float p1, float p2, const float* shv,
                                          float rgb[3]) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    float d[3];
    double len;
    view_dir(cam, p0, p1, p2, d, len);
    float Y[16];
    sh_basis(DEG, d[0], d[1], d[2], Y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < NB; ++k) acc += shv[k * 3 + c] * Y[k];
        // finite in FP32 (overflow saturates), so a zero weight always contributes zero
        rgb[c] = fminf(fmaxf(acc + 0.5f, 0.f), 3.402823466e38f);
    }
}

// the 64-byte record of entry o
__device__ __forceinline__ void write_record(const PreArgs& a, int64_t o, const Proj& P, double op,
                                             const float rgb[3]) {
    gs_splat s;
    s.u = P.u;
    s.v = P.v;
    s.ca = P.syy / P.det;
    s.cb = -P.sxy / P.det;
    s.cc = P.sxx / P.det;
    s.qmax = P.qmax;
    s.opacity = (float)op;
    s.rgb[0] = rgb[0];
    s.rgb[1] = rgb[1];
    s.rgb[2] = rgb[2];
    const double4* src = reinterpret_cast<const double4*>(&s);
    double4* dst = reinterpret_cast<double4*>(a.splat + o);
    dst[0] = src[0];
    dst[1] = src[1];
}

// One (view, entry) o of the lane's Gaussian (parameters gm, SH coefficients shv) seen by cam:
// count, depth, tile rectangle and the 64-byte record.
template <int DEG, bool COLOR>
__device__ __forceinline__ void project_one(const PreArgs& a, const gs_camera& cam, int64_t o, const Geom& gm,
                                            const float* shv) {
    Proj P;
    double op;
    if (project_geom(a, cam, o, gm, P, op) == 0u) return;
    float rgb[3] = {0.f, 0.f, 0.f};
    if (COLOR) sh_colour<DEG>(cam, gm.p[0], gm.p[1], gm.p[2], shv, rgb);
    write_record(a, o, P, op, rgb);
}

// DEG and COLOR are compile-time so the SH coefficients of the lane's Gaussian are loaded
// into registers together with the geometry, before the projection math: every load of the
// lane is in flight at once instead of the SH loads waiting behind the FP64 chain. The
// coefficient planes are read once per frame: streamed past the caches.
template <int DEG, bool COLOR>
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
    const int v = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n) return;
    const int64_t i = a.subset ? (int64_t)a.subset[j] : j;
    const int64_t o = (int64_t)v * a.n + j;
    if (i < 0 || i >= a.n_all) {  // a subset index outside the scene selects nothing
        a.count[o] = 0u;
        return;
    }
    const gs_camera cam = a.cams[v];
    constexpr int NB = (DEG + 1) * (DEG + 1);
    // every load of the lane is issued here, then waited for once
    const Geom gm = load_geom(a.mean, a.scale, a.quat, a.opac, a.n_all, i);
    float shv[COLOR ? NB * 3 : 1];
    if (COLOR) {
#pragma unroll
        for (int k = 0; k < NB * 3; ++k) shv[k] = __builtin_nontemporal_load(&a.sh[(int64_t)k * a.n_all + i]);
#pragma unroll
        for (int k = 0; k < NB * 3; ++k) asm volatile("" ::"v"(shv[k]));
    }
    project_one<DEG, COLOR>(a, cam, o, gm, shv);
}

// One view with colour: a workgroup takes 64 Gaussians with two waves. Wave 0 loads the geometry and
// runs the FP64 projection (count, depth, rectangle); wave 1 loads the positions and the SH
// coefficients and evaluates the colours into LDS; after one barrier wave 0 writes the records.
// Each wave holds half the registers of the one-wave form, and the two waves' loads and math
// overlap. The arithmetic of every value is that of k_preprocess.
template <int DEG>
__global__ __launch_bounds__(128) void k_preprocess_split(PreArgs a) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    __shared__ float s_rgb[3][64];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 64 + l;
    const bool inr = j < a.n;
    const int64_t i = inr ? (a.subset ? (int64_t)a.subset[j] : j) : -1;
    const bool valid = inr && i >= 0 && i < a.n_all;  // a subset index outside the scene selects nothing
    const gs_camera cam = a.cams[0];
    Proj P;
    double op = 0.0;
    uint32_t cnt = 0u;
    if (wv == 0) {
        if (valid) {
            const Geom gm = load_geom(a.mean, a.scale, a.quat, a.opac, a.n_all, i);
            cnt = project_geom(a, cam, j, gm, P, op);
        } else if (inr) {
            a.count[j] = 0u;
        }
    } else if (valid) {
        float shv[NB * 3];
#pragma unroll
        for (int k = 0; k < NB * 3; ++k) shv[k] = __builtin_nontemporal_load(&a.sh[(int64_t)k * a.n_all + i]);
        float rgb[3];
        sh_colour<DEG>(cam, a.mean[i], a.mean[a.n_all + i], a.mean[2 * a.n_all + i], shv, rgb);
#pragma unroll
        for (int c = 0; c < 3; ++c) s_rgb[c][l] = rgb[c];
    }
    __syncthreads();
    if (wv == 0 && cnt != 0u) {
        const float rgb[3] = {s_rgb[0][l], s_rgb[1][l], s_rgb[2][l]};
        write_record(a, j, P, op, rgb);
    }
}

// Several views: the lane reads its Gaussian's parameters and SH coefficients once and projects
// it into every view of the batch in turn (each view re-reading 236 bytes per Gaussian would
// move the batch's whole parameter set once per view).
template <int DEG, bool COLOR>
__global__ __launch_bounds__(256) void k_preprocess_views(PreArgs a) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n) return;
    const int64_t i = a.subset ? (int64_t)a.subset[j] : j;
    if (i < 0 || i >= a.n_all) {  // a subset index outside the scene selects nothing
        for (int v = 0; v < a.n_views; ++v) a.count[(int64_t)v * a.n + j] = 0u;
        return;
    }
    constexpr int NB = (DEG + 1) * (DEG + 1);
    const Geom gm = load_geom(a.mean, a.scale, a.quat, a.opac, a.n_all, i);
    float shv[COLOR ? NB * 3 : 1];
    if (COLOR) {
#pragma unroll
        for (int k = 0; k < NB * 3; ++k) shv[k] = __builtin_nontemporal_load(&a.sh[(int64_t)k * a.n_all + i]);
#pragma unroll
        for (int k = 0; k < NB * 3; ++k) asm volatile("" ::"v"(shv[k]));
    }
    for (int v = 0; v < a.n_views; ++v) project_one<DEG, COLOR>(a, a.cams[v], (int64_t)v * a.n + j, gm, shv);
}

// ---------------------------------------------------------------------------------------
// Reverse mode: chain per-(view, Gaussian) gradients of the 2D quantities (u, v, conic
// a, b, c, opacity, rgb) to the parameters. The per-entry 2D gradients are the sums of the
// entry's pair slots (the reverse traversal's per-(tile, entry) partial sums), formed here in a
// fixed order. One lane per Gaussian, looping over the views of the batch, so each Gaussian's
// gradient is owned by one lane (no atomics). The geometric kernels cover position (through u,
// v and J), scale, rotation and opacity; the colour part follows in k_preprocess_bwd_sh. Adding reads and writes only the gradients of
// Gaussians some pair contributes to; overwriting writes every one and reads none, which halves
// the gradient traffic where (as in random storage order) the visible Gaussians are spread over
// every cache line anyway.
// ---------------------------------------------------------------------------------------
struct PreBwdArgs {
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opac;
    const float* sh;
    int64_t n;
    int deg;
    const gs_camera* cams;
    int n_views;
    gs_params p;
    const uint32_t* count;   // [V][n]
    const float* g2;         // [9][V*n]: the colour fields 6..8, read by the SH kernel where count > 0
    // the pair slots, summed by the geometric kernels (entry o owns the nine-float slots
    // [eoff[o], eoff[o] + count[o])), which write the colour fields 6..8 of g2 (g2w)
    const uint32_t* eoff;
    const float* slots;
    uint64_t capacity;
    float* g2w;
    const uint32_t* overflow;  // nothing is added after a pair overflow (zeros written when overwriting)
    int overwrite;             // 1: write every gradient (=) instead of adding (+=)
    float* gmean;
    float* gscale;
    float* gquat;
    float* gopac;
    float* gsh;
};

// A wave-uniform row pointer held in scalar registers, in the global address space, and the
// element at byte offset lb (a 32-bit lane offset) of it: each access is a scalar base plus a
// vector offset, with no 64-bit address arithmetic per lane.
#define GS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GS_GLOBAL T* uniform_ptr(T* p) {
    const uint64_t x = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return reinterpret_cast<GS_GLOBAL T*>(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ GS_GLOBAL T& lane(GS_GLOBAL T* row, uint32_t lb) {
    static_assert(sizeof(T) == 4, "4-byte elements");
    return *(GS_GLOBAL T*)((GS_GLOBAL const char*)row + lb);
}

// the eleven parameters of the lane's Gaussian from rows at scalar addresses (i0: the wave's
// first Gaussian, lb: the lane's byte offset)
__device__ __forceinline__ Geom load_geom_rows(const PreBwdArgs& a, int64_t i0, uint32_t lb) {
    Geom g;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.p[k] = lane(uniform_ptr(a.mean + k * a.n + i0), lb);
        g.s[k] = lane(uniform_ptr(a.scale + k * a.n + i0), lb);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) g.q[k] = lane(uniform_ptr(a.quat + k * a.n + i0), lb);
    g.o = lane(uniform_ptr(a.opac + i0), lb);
    return g;
}

// The parameter chain's running sums of one Gaussian (FP64, over the views in order)
struct GeomAcc {
    double gp[3], gs[3], gq[4], go;
    bool any;  // some view's 2D gradients were not all zero
};

// One view's 2D gradients g6 = (u, v, conic a, b, c, opacity) of the Gaussian with parameters gm,
// seen by camera cam, chained to its parameters and added into A.
__device__ __forceinline__ void chain_step(const PreBwdArgs& a, const Geom& gm, const gs_camera& cam,
                                           const float (&g6)[6], GeomAcc& A) {
    const float gu = g6[0], gv = g6[1], gA = g6[2], gB = g6[3], gC = g6[4], gO = g6[5];
    if (gu == 0.f && gv == 0.f && gA == 0.f && gB == 0.f && gC == 0.f && gO == 0.f) return;
    A.any = true;
    Proj P;
    double op;
    if (!project_vals(cam, a.p, gm, P, op)) return;
    A.go += gO;
    const double idet = 1.0 / P.det;
    const double ca = P.syy * idet, cb = -P.sxy * idet, cc = P.sxx * idet;
    // conic Q = Sigma'^-1; for a symmetric perturbation dSigma', dQ = -Q dSigma' Q.
    // With G = [[gA, gB/2], [gB/2, gC]] the gradient w.r.t. Sigma' is -Q G Q.
    const double g00 = gA, g01 = 0.5 * gB, g11 = gC;
    const double QG00 = ca * g00 + cb * g01, QG01 = ca * g01 + cb * g11;
    const double QG10 = cb * g00 + cc * g01, QG11 = cb * g01 + cc * g11;
    const double H00 = -(QG00 * ca + QG01 * cb);
    const double H01 = -(QG00 * cb + QG01 * cc);
    const double H11 = -(QG10 * cb + QG11 * cc);
    const double H[2][2] = {{H00, H01}, {H01, H11}};
    // Sigma' = T Sigma T^T: dL/dSigma = T^T H T, dL/dT = 2 H T Sigma
    double GS[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            GS[r][c] = P.T[0][r] * (H[0][0] * P.T[0][c] + H[0][1] * P.T[1][c]) +
                       P.T[1][r] * (H[1][0] * P.T[0][c] + H[1][1] * P.T[1][c]);
    double HT[2][3], GT[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) HT[r][c] = H[r][0] * P.T[0][c] + H[r][1] * P.T[1][c];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            GT[r][c] = 2.0 * (HT[r][0] * P.Sg[0][c] + HT[r][1] * P.Sg[1][c] + HT[r][2] * P.Sg[2][c]);
    // T = J R with J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]: dL/dJ = GT R^T
    const float* Rc = cam.R;
    double GJ00 = 0, GJ02 = 0, GJ11 = 0, GJ12 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        GJ00 += GT[0][k] * Rc[0 * 3 + k];
        GJ02 += GT[0][k] * Rc[2 * 3 + k];
        GJ11 += GT[1][k] * Rc[1 * 3 + k];
        GJ12 += GT[1][k] * Rc[2 * 3 + k];
    }
    const double fx = cam.fx, fy = cam.fy, z = P.z, iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
    double gc[3];
    gc[0] = -fx * iz2 * GJ02 + fx * iz * gu;
    gc[1] = -fy * iz2 * GJ12 + fy * iz * gv;
    gc[2] = -fx * iz2 * GJ00 + 2.0 * fx * P.x * iz3 * GJ02 - fy * iz2 * GJ11 + 2.0 * fy * P.y * iz3 * GJ12 -
            fx * P.x * iz2 * gu - fy * P.y * iz2 * gv;
    // world mean: p_c = R p + t
#pragma unroll
    for (int k = 0; k < 3; ++k) A.gp[k] += Rc[k] * gc[0] + Rc[3 + k] * gc[1] + Rc[6 + k] * gc[2];
    // Sigma = M M^T with M = Rq diag(s): dL/dM = 2 GS M
    const double s[3] = {gm.s[0], gm.s[1], gm.s[2]};
    double GR[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double gm =
                2.0 * (GS[r][0] * P.Rq[0][c] * s[c] + GS[r][1] * P.Rq[1][c] * s[c] + GS[r][2] * P.Rq[2][c] * s[c]);
            A.gs[c] += gm * P.Rq[r][c];
            GR[r][c] = gm * s[c];
        }
    const double w = P.qh[0], x = P.qh[1], y = P.qh[2], zq = P.qh[3];
    double gw = 2.0 * (-zq * GR[0][1] + y * GR[0][2] + zq * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
    double gx = 2.0 * (y * GR[0][1] + zq * GR[0][2] + y * GR[1][0] - 2.0 * x * GR[1][1] - w * GR[1][2] +
                       zq * GR[2][0] + w * GR[2][1] - 2.0 * x * GR[2][2]);
    double gy = 2.0 * (-2.0 * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + zq * GR[1][2] -
                       w * GR[2][0] + zq * GR[2][1] - 2.0 * y * GR[2][2]);
    double gz = 2.0 * (-2.0 * zq * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2.0 * zq * GR[1][1] +
                       y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
    const double dot = w * gw + x * gx + y * gy + zq * gz;
    const double iqn = 1.0 / P.qn;
    A.gq[0] += (gw - w * dot) * iqn;
    A.gq[1] += (gx - x * dot) * iqn;
    A.gq[2] += (gy - y * dot) * iqn;
    A.gq[3] += (gz - zq * dot) * iqn;
    
}

// the chain's results: written (old = 0) or added onto the gradients held (old)
__device__ __forceinline__ void write_geom(const PreBwdArgs& a, int64_t i0, uint32_t lb, const float (&old)[11],
                                           const GeomAcc& A) {
    const int64_t n = a.n;
    auto grow = [&](float* base, int k) -> GS_GLOBAL float& { return lane(uniform_ptr(base + k * n + i0), lb); };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        grow(a.gmean, k) = old[k] + (float)A.gp[k];
        grow(a.gscale, k) = old[3 + k] + (float)A.gs[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) grow(a.gquat, k) = old[6 + k] + (float)A.gq[k];
    grow(a.gopac, 0) = old[10] + (float)A.go;
}

// The parameter chain of one Gaussian composited in the one view (byte offset lb from the row
// base i0), from the view's 2D gradients summed in LDS (sg), written (or added).
__device__ __forceinline__ void geom_chain(const PreBwdArgs& a, int64_t i0, uint32_t lb, bool acc,
                                           const float (*sg)[9]) {
    const int64_t n = a.n;
    auto grow = [&](float* base, int k) -> GS_GLOBAL float& { return lane(uniform_ptr(base + k * n + i0), lb); };
    GeomAcc A = {};
    // parameters and the gradients accumulated so far are requested together
    const Geom gm = load_geom_rows(a, i0, lb);
    float g6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) g6[k] = sg[lb >> 2][k];
    float old[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) old[k] = 0.f;
    if (acc) {
#pragma unroll
        for (int k = 0; k < 3; ++k) old[k] = grow(a.gmean, k), old[3 + k] = grow(a.gscale, k);
#pragma unroll
        for (int k = 0; k < 4; ++k) old[6 + k] = grow(a.gquat, k);
        old[10] = grow(a.gopac, 0);
    }
    chain_step(a, gm, a.cams[0], g6, A);
    if (!A.any && acc) return;
    write_geom(a, i0, lb, old, A);
}

// One view. One wave per workgroup takes BWD_CHUNK consecutive Gaussians. It first sums their
// pair slots: entry o owns the slots [eoff[o], eoff[o] + count[o]) and consecutive entries own
// consecutive runs, so the chunk's slots form one range, read 64 at a time (coalesced) and
// reduced by a segmented scan whose run ends add into the owner's sums in LDS, round after
// round (every sum formed in the same order on every call); the colour fields go to g2 for
// the SH kernel. It lists in LDS the Gaussians the view composited and runs the parameter chain
// on them 64 at a time, so the long FP64 chain runs on nearly full waves even where few
// Gaussians are visible (about one in five for a view of a large scene, spread over every
// wave in random storage order); the others get zeros when overwriting and nothing when adding.
constexpr int BWD_CHUNK = 256;

__global__ __launch_bounds__(64) void k_preprocess_bwd(PreBwdArgs a) {
    __shared__ uint16_t s_list[BWD_CHUNK];
    __shared__ uint32_t s_beg[BWD_CHUNK];
    __shared__ float s_g[BWD_CHUNK][9];
    __shared__ uint32_t s_end;
    const int64_t i0 = (int64_t)blockIdx.x * BWD_CHUNK;
    const uint32_t l = threadIdx.x;
    const int64_t n = a.n;
    const bool acc = !a.overwrite;
    auto zero = [&](uint32_t lb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lane(uniform_ptr(a.gmean + k * n + i0), lb) = 0.f;
            lane(uniform_ptr(a.gscale + k * n + i0), lb) = 0.f;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) lane(uniform_ptr(a.gquat + k * n + i0), lb) = 0.f;
        lane(uniform_ptr(a.gopac + i0), lb) = 0.f;
    };
    if (*a.overflow) {  // nothing is added after a pair overflow; zeros are written when overwriting
        if (acc) return;
        for (uint32_t li = l; li < BWD_CHUNK; li += 64)
            if (i0 + li < n) zero(li * 4u);
        return;
    }
    // the chunk's counts and first slots are requested together
    constexpr int NS = BWD_CHUNK / 64;
    const int last = (int)min((int64_t)BWD_CHUNK - 1, n - 1 - i0);  // the chunk's last Gaussian
    uint32_t cnt[NS], eo[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const uint32_t li = 64 * j + l;
        const bool valid = i0 + li < n;
        cnt[j] = valid ? lane(uniform_ptr(a.count + i0), li * 4u) : 0u;
        eo[j] = valid ? lane(uniform_ptr(a.eoff + i0), li * 4u) : 0u;
    }
    uint64_t act_mask[NS];
    uint32_t total = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const uint32_t li = 64 * j + l;
        const bool act = cnt[j] != 0;
        act_mask[j] = ballot(act);
        if (act) s_list[total + mask_rank(act_mask[j])] = (uint16_t)li;
        total += (uint32_t)__builtin_popcountll(act_mask[j]);
        if ((int)li <= last) s_beg[li] = eo[j];
        if ((int)li == last) s_end = eo[j] + cnt[j];
#pragma unroll
        for (int f = 0; f < 9; ++f) s_g[li][f] = 0.f;
    }
    __syncthreads();
    {
        const uint32_t S0 = s_beg[0], S1 = s_end;
        for (uint32_t base = S0; base < S1; base += 64) {  // the same for the whole wave
            const uint32_t sl = base + l;
            const bool in = sl < S1 && (uint64_t)sl < a.capacity;
            // owner: the largest Gaussian of the chunk whose run starts at or before sl (those
            // with no pairs share the next one's start, so the largest is the one with pairs)
            int L = 0;
#pragma unroll
            for (int step = BWD_CHUNK / 2; step > 0; step >>= 1)
                if (L + step <= last && s_beg[L + step] <= sl) L += step;
            if (!in) L = -1 - (int)l;  // unique: never merged with another lane
            float x[9];
#pragma unroll
            for (int f = 0; f < 9; ++f) x[f] = in ? a.slots[(uint64_t)sl * 9 + f] : 0.f;
            seg_scan9(L, x);
            const int Ln = __shfl_down(L, 1);
            if (in && (l == 63 || Ln != L)) {
#pragma unroll
                for (int f = 0; f < 9; ++f) s_g[L][f] += x[f];
            }
        }
        __syncthreads();
        // colour fields of the composited entries, for the SH kernel
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const uint32_t li = 64 * j + l;
            if (cnt[j] != 0) {
#pragma unroll
                for (int f = 6; f < 9; ++f) lane(uniform_ptr(a.g2w + f * n + i0), li * 4u) = s_g[li][f];
            }
        }
    }
    for (uint32_t b = 0; b < total; b += 64)
        if (b + l < total) geom_chain(a, i0, (uint32_t)s_list[b + l] * 4u, acc, s_g);
    // zeros for the rest, after the chain's loads so they do not wait behind these stores
    if (!acc) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const uint32_t li = 64 * j + l;
            if (i0 + li < n && !((act_mask[j] >> l) & 1)) zero(li * 4u);
        }
    }
}

// Several views: one wave per workgroup takes MV_CHUNK consecutive Gaussians and goes through
// the views in order. For each view it sums the chunk's pair slots of that view (one coalesced
// range, as the one-view kernel does), writes the colour sums for the SH kernel, lists the
// Gaussians that view composited and runs that view's chain step on them 64 at a time, the
// running FP64 sums of every Gaussian of the chunk held in LDS between views. So the FP64 step
// runs on nearly full waves although each view composites only some of the Gaussians, and each
// Gaussian's sums still run over the views in order.
constexpr int MV_CHUNK = 128;

__global__ __launch_bounds__(64) void k_preprocess_bwd_mv(PreBwdArgs a) {
    constexpr int NS = MV_CHUNK / 64;
    __shared__ uint32_t s_beg[MV_CHUNK];
    __shared__ float s_g[MV_CHUNK][9];
    __shared__ uint16_t s_list[MV_CHUNK];
    __shared__ double s_acc[11][MV_CHUNK];  // gp[3], gs[3], gq[4], go of each Gaussian
    __shared__ uint32_t s_any[MV_CHUNK];
    __shared__ uint32_t s_end;
    const int64_t i0 = (int64_t)blockIdx.x * MV_CHUNK;
    const uint32_t l = threadIdx.x;
    const int64_t n = a.n, VN = (int64_t)a.n_views * n;
    const bool acc = !a.overwrite;
    const int last = (int)min((int64_t)MV_CHUNK - 1, n - 1 - i0);  // the chunk's last Gaussian
    auto grow = [&](float* base, int k, uint32_t lb) -> GS_GLOBAL float& {
        return lane(uniform_ptr(base + k * n + i0), lb);
    };
    auto zero = [&](uint32_t lb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) grow(a.gmean, k, lb) = 0.f, grow(a.gscale, k, lb) = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) grow(a.gquat, k, lb) = 0.f;
        grow(a.gopac, 0, lb) = 0.f;
    };
    if (*a.overflow) {  // nothing is added after a pair overflow; zeros are written when overwriting
        if (acc) return;
        for (uint32_t li = l; li < MV_CHUNK; li += 64)
            if (i0 + li < n) zero(li * 4u);
        return;
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const uint32_t li = 64 * j + l;
#pragma unroll
        for (int k = 0; k < 11; ++k) s_acc[k][li] = 0.0;
        s_any[li] = 0u;
    }
    uint64_t seen[NS];  // composited in some view so far
#pragma unroll
    for (int j = 0; j < NS; ++j) seen[j] = 0;
    // counts and entry offsets of the view after the current one, requested before the current
    // view's chain so that their latency hides behind it
    uint32_t cnt_nx[NS], e_nx[NS];
    auto fetch = [&](int v) {
        const int64_t o0 = (int64_t)v * n + i0;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const uint32_t li = 64 * j + l;
            const bool valid = i0 + li < n;
            cnt_nx[j] = valid ? lane(uniform_ptr(a.count + o0), li * 4u) : 0u;
            e_nx[j] = valid ? lane(uniform_ptr(a.eoff + o0), li * 4u) : 0u;
        }
    };
    fetch(0);
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t o0 = (int64_t)v * n + i0;
        uint32_t cnt[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const uint32_t li = 64 * j + l;
            cnt[j] = cnt_nx[j];
            const uint32_t e = e_nx[j];
            if ((int)li <= last) s_beg[li] = e;
            if ((int)li == last) s_end = e + cnt[j];
#pragma unroll
            for (int f = 0; f < 9; ++f) s_g[li][f] = 0.f;
        }
        __syncthreads();
        const uint32_t S0 = s_beg[0], S1 = s_end;
        for (uint32_t base = S0; base < S1; base += 64) {  // the same for the whole wave
            const uint32_t sl = base + l;
            const bool in = sl < S1 && (uint64_t)sl < a.capacity;
            int L = 0;  // owner: the largest Gaussian of the chunk whose run starts at or before sl
#pragma unroll
            for (int step = MV_CHUNK / 2; step > 0; step >>= 1)
                if (L + step <= last && s_beg[L + step] <= sl) L += step;
            if (!in) L = -1 - (int)l;  // unique: never merged with another lane
            float x[9];
#pragma unroll
            for (int f = 0; f < 9; ++f) x[f] = in ? a.slots[(uint64_t)sl * 9 + f] : 0.f;
            seg_scan9(L, x);
            const int Ln = __shfl_down(L, 1);
            if (in && (l == 63 || Ln != L)) {
#pragma unroll
                for (int f = 0; f < 9; ++f) s_g[L][f] += x[f];
            }
        }
        __syncthreads();
        // colour sums of this view's composited entries; the list of them
        uint32_t total = 0;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const uint32_t li = 64 * j + l;
            const bool c = cnt[j] != 0;
            if (c) {
#pragma unroll
                for (int f = 6; f < 9; ++f) lane(uniform_ptr(a.g2w + f * VN + o0), li * 4u) = s_g[li][f];
            }
            const uint64_t m = ballot(c);
            if (c) s_list[total + mask_rank(m)] = (uint16_t)li;
            total += (uint32_t)__builtin_popcountll(m);
            seen[j] |= m;
        }
        __syncthreads();
        if (v + 1 < a.n_views) fetch(v + 1);
        const gs_camera cam = a.cams[v];
        for (uint32_t b = 0; b < total; b += 64) {
            if (b + l < total) {
                const uint32_t li = s_list[b + l];
                const Geom gm = load_geom_rows(a, i0, li * 4u);
                GeomAcc A;
#pragma unroll
                for (int k = 0; k < 3; ++k) A.gp[k] = s_acc[k][li], A.gs[k] = s_acc[3 + k][li];
#pragma unroll
                for (int k = 0; k < 4; ++k) A.gq[k] = s_acc[6 + k][li];
                A.go = s_acc[10][li];
                A.any = s_any[li] != 0u;
                float g6[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) g6[k] = s_g[li][k];
                chain_step(a, gm, cam, g6, A);
#pragma unroll
                for (int k = 0; k < 3; ++k) s_acc[k][li] = A.gp[k], s_acc[3 + k][li] = A.gs[k];
#pragma unroll
                for (int k = 0; k < 4; ++k) s_acc[6 + k][li] = A.gq[k];
                s_acc[10][li] = A.go;
                s_any[li] = A.any ? 1u : 0u;
            }
        }
        __syncthreads();  // the sums and lists are rewritten for the next view
    }
    // the results, written (or added) for the Gaussians some view composited; zeros for the rest
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const uint32_t li = 64 * j + l, lb = li * 4u;
        if (i0 + li >= n) continue;
        if ((seen[j] >> l) & 1) {
            GeomAcc A;
#pragma unroll
            for (int k = 0; k < 3; ++k) A.gp[k] = s_acc[k][li], A.gs[k] = s_acc[3 + k][li];
#pragma unroll
            for (int k = 0; k < 4; ++k) A.gq[k] = s_acc[6 + k][li];
            A.go = s_acc[10][li];
            A.any = s_any[li] != 0u;
            if (!A.any && acc) continue;
            float old[11];
#pragma unroll
            for (int k = 0; k < 11; ++k) old[k] = 0.f;
            if (acc) {
#pragma unroll
                for (int k = 0; k < 3; ++k) old[k] = grow(a.gmean, k, lb), old[3 + k] = grow(a.gscale, k, lb);
#pragma unroll
                for (int k = 0; k < 4; ++k) old[6 + k] = grow(a.gquat, k, lb);
                old[10] = grow(a.gopac, 0, lb);
            }
            write_geom(a, i0, lb, old, A);
        } else if (!acc) {
            zero(lb);
        }
    }
}

// Colour part of the reverse mode: SH coefficient gradients and the mean gradient through
// the view direction. Split from the geometric part so that neither kernel carries the
// other's registers. A workgroup takes 64 G Gaussians with 3 G waves: wave (c, s) holds colour
// channel c's coefficients of Gaussians [64 s, 64 s + 64) of them (16 values at SH-3 instead of
// 48), so the G waves of a channel read and write 256 G contiguous bytes of each coefficient
// plane together (G = 4 measured fastest for one view, G = 1 for several, where each lane
// walks every view). The channels' mean-gradient parts are added through LDS at the end, onto
// what the geometric part left (written or added). The kernel streams the coefficient planes
// (read once, written once), so what bounds it is the memory requests in flight: the register
// budget is held to six waves per SIMD, two workgroups per CU at G = 4, and the gradient rows
// are stored past the caches.
template <int DEG, int G>
__global__ __launch_bounds__(192 * G) __attribute__((amdgpu_waves_per_eu(6))) void k_preprocess_bwd_sh(PreBwdArgs a) {
    constexpr int NB = (DEG + 1) * (DEG + 1);
    __shared__ float s_gp[3][3][64 * G];
    __shared__ uint32_t s_any[3][64 * G];
    // channel and sub-block are wave-uniform, so every plane's row of a wave's 64 Gaussians is a
    // scalar address and the lanes index it with their lane number
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int c = wv / G, sub = wv % G;
    const uint32_t l = threadIdx.x & 63u;
    const int64_t i0 = (int64_t)blockIdx.x * (64 * G) + sub * 64, i = i0 + l;
    const int ls = sub * 64 + (int)l;  // the Gaussian within the workgroup
    const bool acc = !a.overwrite;
    const int64_t n = a.n;
    auto row = [&](float* base, int k) { return uniform_ptr(base + (int64_t)(k * 3 + c) * n + i0); };
    auto crow = [&](const float* base, int k) { return uniform_ptr(base + (int64_t)(k * 3 + c) * n + i0); };
    const uint32_t lb = l * 4u;  // the lane's byte offset in a row
    if (*a.overflow) {  // the same for the whole workgroup
        if (!acc && i < n) {
#pragma unroll
            for (int k = 0; k < NB; ++k) lane(row(a.gsh, k), lb) = 0.f;
        }
        return;
    }
    const bool valid = i < n;
    const int64_t VN = (int64_t)a.n_views * n;
    float shv[NB], gsh[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        shv[k] = valid ? __builtin_nontemporal_load(&lane(crow(a.sh, k), lb)) : 0.f;
        gsh[k] = 0.f;
    }
    float px = 0.f, py = 0.f, pz = 0.f;
    // the first view's count and colour gradient are requested together with the parameters
    uint32_t cnt0 = 0;
    float gc0 = 0.f;
    const int64_t g2o = (6 + c) * VN + i0;  // colour gradient of channel c, view 0
    if (valid) {
        px = lane(uniform_ptr(a.mean + i0), lb);
        py = lane(uniform_ptr(a.mean + n + i0), lb);
        pz = lane(uniform_ptr(a.mean + 2 * n + i0), lb);
        cnt0 = lane(uniform_ptr(a.count + i0), lb);
        gc0 = lane(uniform_ptr(a.g2 + g2o), lb);
    }
    double gp[3] = {0, 0, 0};
    bool any = false;
    // the next view's count and colour gradient are requested before this view's math, so
    // their latency hides behind it (the gradient is read whatever the count; it is used
    // only where the count is not zero)
    uint32_t cnt_next = cnt0;
    float gc_next = gc0;
    for (int v = 0; valid && v < a.n_views; ++v) {
        const uint32_t cnt = cnt_next;
        const float gc = gc_next;
        if (v + 1 < a.n_views) {
            const int64_t o = (int64_t)(v + 1) * n;
            cnt_next = lane(uniform_ptr(a.count + o + i0), lb);
            gc_next = lane(uniform_ptr(a.g2 + g2o + o), lb);
        }
        if (cnt == 0) continue;
        if (gc == 0.f) continue;
        any = true;
        const gs_camera cam = a.cams[v];
        float d[3];
        double len;
        view_dir(cam, px, py, pz, d, len);
        float Y[16];
        sh_basis(DEG, d[0], d[1], d[2], Y);
        float accv = 0.f;
#pragma unroll
        for (int k = 0; k < NB; ++k) accv += shv[k] * Y[k];
        if (!(accv + 0.5f > 0.f)) continue;  // colour clamped at 0: no gradient
#pragma unroll
        for (int k = 0; k < NB; ++k) gsh[k] += gc * Y[k];
        float gd[3];
        sh_wgrad(DEG, d[0], d[1], d[2], shv, gc, gd);
        // d(d)/d(mean) = (I - d d^T) / len
        const double dd = (double)d[0] * gd[0] + (double)d[1] * gd[1] + (double)d[2] * gd[2];
        const double il = 1.0 / len;
#pragma unroll
        for (int k = 0; k < 3; ++k) gp[k] += ((double)gd[k] - (double)d[k] * dd) * il;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) s_gp[c][k][ls] = (float)gp[k];
    s_any[c][ls] = any ? 1u : 0u;
    // written rows are not read again here: streamed past the caches. (Two branches, so that
    // no read of the old gradient is speculated into the writing one.)
    if (valid && acc && any) {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            GS_GLOBAL float& q = lane(row(a.gsh, k), lb);
            q = q + gsh[k];
        }
    } else if (valid && !acc) {
#pragma unroll
        for (int k = 0; k < NB; ++k) __builtin_nontemporal_store(0.f + gsh[k], &lane(row(a.gsh, k), lb));
    }
    __syncthreads();
    if (c == 0 && valid && (s_any[0][ls] | s_any[1][ls] | s_any[2][ls])) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            lane(uniform_ptr(a.gmean + k * n + i0), lb) += s_gp[0][k][ls] + s_gp[1][k][ls] + s_gp[2][k][ls];
    }
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------
gs_status launch_preprocess(const gs_gaussians* g, const gs_views* views, const gs_params* p,
                            const int32_t* subset, int64_t n, int want_color, gs_projected* out,
                            hipStream_t stream) {
    if (n == 0) return GS_OK;
    PreArgs a;
    a.mean = g->mean;
    a.scale = g->scale;
    a.quat = g->quat;
    a.opac = g->opacity;
    a.sh = g->sh;
    a.n_all = g->n;
    a.deg = g->sh_degree;
    a.cams = views->cams;
    a.p = *p;
    a.tile_w = views->tile_w;
    a.tile_h = views->tile_h;
    a.subset = subset;
    a.n = n;
    a.want_color = want_color;
    a.splat = out->splat;
    a.depth = out->depth;
    a.rect = out->rect;
    a.count = out->count;
    a.n_views = views->n_views;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (views->n_views == 1) {
        const dim3 grid(blocks, 1);
        const unsigned blocks64 = (unsigned)((n + 63) / 64);
        if (!want_color) {
            hipLaunchKernelGGL((k_preprocess<0, false>), grid, dim3(256), 0, stream, a);
        } else {
            switch (g->sh_degree) {
                case 0: hipLaunchKernelGGL((k_preprocess<0, true>), grid, dim3(256), 0, stream, a); break;
                case 1: hipLaunchKernelGGL((k_preprocess<1, true>), grid, dim3(256), 0, stream, a); break;
                case 2: hipLaunchKernelGGL((k_preprocess_split<2>), dim3(blocks64), dim3(128), 0, stream, a); break;
                default: hipLaunchKernelGGL((k_preprocess_split<3>), dim3(blocks64), dim3(128), 0, stream, a); break;
            }
        }
    } else {
        if (!want_color) {
            hipLaunchKernelGGL((k_preprocess_views<0, false>), dim3(blocks), dim3(256), 0, stream, a);
        } else {
            switch (g->sh_degree) {
                case 0: hipLaunchKernelGGL((k_preprocess_views<0, true>), dim3(blocks), dim3(256), 0, stream, a); break;
                case 1: hipLaunchKernelGGL((k_preprocess_views<1, true>), dim3(blocks), dim3(256), 0, stream, a); break;
                case 2: hipLaunchKernelGGL((k_preprocess_views<2, true>), dim3(blocks), dim3(256), 0, stream, a); break;
                default: hipLaunchKernelGGL((k_preprocess_views<3, true>), dim3(blocks), dim3(256), 0, stream, a); break;
            }
        }
    }
    return check_launch("preprocess");
}

template <int DEG>
static void launch_bwd_sh(bool one_view, int64_t n, hipStream_t stream, const PreBwdArgs& a) {
    if (one_view)
        hipLaunchKernelGGL((k_preprocess_bwd_sh<DEG, 4>), dim3((unsigned)((n + 255) / 256)), dim3(768), 0, stream, a);
    else
        hipLaunchKernelGGL((k_preprocess_bwd_sh<DEG, 1>), dim3((unsigned)((n + 63) / 64)), dim3(192), 0, stream, a);
}

gs_status launch_preprocess_bwd(const gs_gaussians* g, const gs_views* views, const gs_params* p,
                                const gs_projected* proj, const gs_bins* bins, const float* slots, float* g2,
                                gs_gaussians_grad* grad, hipStream_t stream) {
    if (g->n == 0) return GS_OK;
    PreBwdArgs a;
    a.mean = g->mean;
    a.scale = g->scale;
    a.quat = g->quat;
    a.opac = g->opacity;
    a.sh = g->sh;
    a.n = g->n;
    a.deg = g->sh_degree;
    a.cams = views->cams;
    a.n_views = views->n_views;
    a.p = *p;
    a.count = proj->count;
    a.g2 = g2;
    a.eoff = bins->entry_offset;
    a.slots = slots;
    a.capacity = bins->capacity;
    a.g2w = g2;
    a.overflow = bins->overflow;
    a.overwrite = grad->overwrite;
    a.gmean = grad->mean;
    a.gscale = grad->scale;
    a.gquat = grad->quat;
    a.gopac = grad->opacity;
    a.gsh = grad->sh;
    const dim3 grid((unsigned)((g->n + BWD_CHUNK - 1) / BWD_CHUNK));
    if (views->n_views == 1)
        hipLaunchKernelGGL(k_preprocess_bwd, grid, dim3(64), 0, stream, a);
    else
        hipLaunchKernelGGL(k_preprocess_bwd_mv, dim3((unsigned)((g->n + MV_CHUNK - 1) / MV_CHUNK)), dim3(64), 0, stream,
                           a);
    // colour part: 64 G Gaussians x 3 channels per workgroup
    switch (g->sh_degree) {
        case 0: launch_bwd_sh<0>(views->n_views == 1, g->n, stream, a); break;
        case 1: launch_bwd_sh<1>(views->n_views == 1, g->n, stream, a); break;
        case 2: launch_bwd_sh<2>(views->n_views == 1, g->n, stream, a); break;
        default: launch_bwd_sh<3>(views->n_views == 1, g->n, stream, a); break;
    }
    return check_launch("preprocess_bwd");
}

}  // namespace gs
