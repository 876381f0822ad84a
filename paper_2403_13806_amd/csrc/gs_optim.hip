// Adam step over the parameter planes of the point representation (the optimisation of phi in
// Sec. 3.2), fused with clearing the gradients: one HBM-bound pass over every element of
// every group, reading parameter, gradient and both moments and writing parameter, moments
// and a zero gradient.
//
// A group's parameter is optimised in one of three parametrisations of the stored value x:
//   linear  u = x
//   log     u = log x         (x > 0; positive scales: multiplicative steps)
//   logit   u = log(x/(1-x))  (x in (0, 1); opacities), x clamped to [1e-6, 1 - 1e-6] first
// with du = dx * x (log) or dx * x (1 - x) (logit); Adam runs on u and x is mapped back.
#include <cmath>
#include <cstdint>

#include "gs_device.hpp"

namespace gs {

namespace {

constexpr int GROUPS_PER_LAUNCH = 16;
constexpr int NT = 256;
constexpr int PER_THREAD = 16;
constexpr int CHUNK = NT * PER_THREAD;  // elements per workgroup, all of one group
typedef float f4 __attribute__((ext_vector_type(4)));

struct AdamTable {
    float* p[GROUPS_PER_LAUNCH];
    float* g[GROUPS_PER_LAUNCH];
    float* m[GROUPS_PER_LAUNCH];
    float* v[GROUPS_PER_LAUNCH];
    int64_t count[GROUPS_PER_LAUNCH];
    int64_t blk[GROUPS_PER_LAUNCH + 1];  // first workgroup of each group
    float lr[GROUPS_PER_LAUNCH];
    int32_t mode[GROUPS_PER_LAUNCH];
    int32_t vec[GROUPS_PER_LAUNCH];  // all four planes 16-byte aligned: 4-element loads and stores
    int32_t count_groups;
    int32_t zero_grad;
    float b1, b2, omb1, omb2, eps, inv_bc1, inv_sqrt_bc2;  // omb = 1 - b, formed in FP64
};

// one element: parameter x, gradient dx and moments m, v in; new x, m, v out
__device__ __forceinline__ void adam1(const AdamTable& t, int mode, float lr, float& x, float dx, float& m, float& v) {
    float xv = x, uu = xv, du = dx;
    if (mode == GS_ADAM_LOG) {
        uu = logf(xv);
        du = dx * xv;
    } else if (mode == GS_ADAM_LOGIT) {
        xv = fminf(fmaxf(xv, 1e-6f), 1.f - 1e-6f);
        uu = logf(xv / (1.f - xv));
        du = dx * xv * (1.f - xv);
    }
    m = t.b1 * m + t.omb1 * du;
    v = t.b2 * v + t.omb2 * du * du;
    uu -= lr * (m * t.inv_bc1) / (sqrtf(v) * t.inv_sqrt_bc2 + t.eps);
    if (mode == GS_ADAM_LOG)
        xv = expf(uu);
    else if (mode == GS_ADAM_LOGIT)
        xv = 1.f / (1.f + expf(-uu));
    else
        xv = uu;
    x = xv;
}

// One workgroup = CHUNK consecutive elements of one group (group, pointers and mode are
// uniform). Aligned groups: each lane takes PER_THREAD / 4 runs of 4 consecutive elements
// (NT runs apart: each wave instruction moves 1 KB), all loads of the lane issued before any
// arithmetic, every plane read and written once with streaming (nontemporal) accesses; the
// tail of a group shorter than 4 goes element by element. Otherwise PER_THREAD single
// elements NT apart. The arithmetic per element is the same in both.
__global__ __launch_bounds__(NT) void k_adam(AdamTable t) {
    const int64_t b = blockIdx.x;
    int k = 0;
    while (b >= t.blk[k + 1]) ++k;
    const int64_t n = t.count[k];
    float* __restrict__ P = t.p[k];
    float* __restrict__ G = t.g[k];
    float* __restrict__ M = t.m[k];
    float* __restrict__ V = t.v[k];
    const int mode = t.mode[k];
    const float lr = t.lr[k];
    if (t.vec[k]) {
        constexpr int R = PER_THREAD / 4;
        const int64_t q0 = (b - t.blk[k]) * (CHUNK / 4) + threadIdx.x;  // first run of the lane
        f4 x[R], dx[R], m[R], v[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t e = 4 * (q0 + u * NT);
            if (e + 3 < n) {
                x[u] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(P + e));
                dx[u] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(G + e));
                m[u] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(M + e));
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(V + e));
            }
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int64_t e = 4 * (q0 + u * NT);
            if (e + 3 < n) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float xc = x[u][c], mc = m[u][c], vc = v[u][c];
                    adam1(t, mode, lr, xc, dx[u][c], mc, vc);
                    x[u][c] = xc, m[u][c] = mc, v[u][c] = vc;
                }
                __builtin_nontemporal_store(x[u], reinterpret_cast<f4*>(P + e));
                __builtin_nontemporal_store(m[u], reinterpret_cast<f4*>(M + e));
                __builtin_nontemporal_store(v[u], reinterpret_cast<f4*>(V + e));
                if (t.zero_grad) __builtin_nontemporal_store(f4(0.f), reinterpret_cast<f4*>(G + e));
            } else {
                for (int64_t j = e; j < n && j < e + 4; ++j) {
                    float xj = P[j], mj = M[j], vj = V[j];
                    adam1(t, mode, lr, xj, G[j], mj, vj);
                    P[j] = xj, M[j] = mj, V[j] = vj;
                    if (t.zero_grad) G[j] = 0.f;
                }
            }
        }
        return;
    }
    const int64_t base = (b - t.blk[k]) * CHUNK + threadIdx.x;
    float x[PER_THREAD], dx[PER_THREAD], m0[PER_THREAD], v0[PER_THREAD];
#pragma unroll
    for (int u = 0; u < PER_THREAD; ++u) {
        const int64_t j = base + u * NT;
        x[u] = dx[u] = m0[u] = v0[u] = 0.f;
        if (j < n) x[u] = P[j], dx[u] = G[j], m0[u] = M[j], v0[u] = V[j];
    }
#pragma unroll
    for (int u = 0; u < PER_THREAD; ++u) {
        const int64_t j = base + u * NT;
        if (j >= n) continue;
        adam1(t, mode, lr, x[u], dx[u], m0[u], v0[u]);
        P[j] = x[u];
        M[j] = m0[u];
        V[j] = v0[u];
        if (t.zero_grad) G[j] = 0.f;
    }
}

}  // namespace

gs_status launch_adam(const gs_adam_group* groups, int32_t n_groups, double b1, double b2, double eps, int64_t step,
                      int32_t zero_grad, hipStream_t s) {
    const double bc1 = 1.0 - std::pow(b1, (double)step), bc2 = 1.0 - std::pow(b2, (double)step);
    AdamTable t{};
    auto flush = [&]() -> gs_status {
        if (t.count_groups == 0) return GS_OK;
        t.zero_grad = zero_grad;
        t.b1 = (float)b1, t.b2 = (float)b2, t.eps = (float)eps;
        t.omb1 = (float)(1.0 - b1), t.omb2 = (float)(1.0 - b2);
        t.inv_bc1 = (float)(1.0 / bc1);
        t.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
        for (int c = t.count_groups + 1; c <= GROUPS_PER_LAUNCH; ++c) t.blk[c] = t.blk[t.count_groups];
        const int64_t blocks = t.blk[t.count_groups];
        hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(NT), 0, s, t);
        t = AdamTable{};
        return check_launch("adam_step");
    };
    for (int k = 0; k < n_groups; ++k) {
        if (groups[k].count == 0) continue;
        const int c = t.count_groups++;
        t.p[c] = groups[k].param, t.g[c] = groups[k].grad, t.m[c] = groups[k].m, t.v[c] = groups[k].v;
        t.count[c] = groups[k].count;
        t.blk[c + 1] = t.blk[c] + (groups[k].count + CHUNK - 1) / CHUNK;
        t.lr[c] = groups[k].lr;
        t.mode[c] = groups[k].mode;
        t.vec[c] = ((reinterpret_cast<uintptr_t>(t.p[c]) | reinterpret_cast<uintptr_t>(t.g[c]) |
                     reinterpret_cast<uintptr_t>(t.m[c]) | reinterpret_cast<uintptr_t>(t.v[c])) & 15u) == 0;
        if (t.count_groups == GROUPS_PER_LAUNCH) {
            gs_status st = flush();
            if (st != GS_OK) return st;
        }
    }
    return flush();
}

}  // namespace gs
