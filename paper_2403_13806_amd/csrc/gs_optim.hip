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

#include "gs_device.hpp"

namespace gs {

namespace {

constexpr int GROUPS_PER_LAUNCH = 16;
constexpr int NT = 256;

struct AdamTable {
    float* p[GROUPS_PER_LAUNCH];
    float* g[GROUPS_PER_LAUNCH];
    float* m[GROUPS_PER_LAUNCH];
    float* v[GROUPS_PER_LAUNCH];
    int64_t end[GROUPS_PER_LAUNCH];  // prefix sums of the group sizes
    float lr[GROUPS_PER_LAUNCH];
    int32_t mode[GROUPS_PER_LAUNCH];
    int32_t count;
    int32_t zero_grad;
    float b1, b2, omb1, omb2, eps, inv_bc1, inv_sqrt_bc2;  // omb = 1 - b, formed in FP64
};

__global__ __launch_bounds__(NT) void k_adam(AdamTable t) {
    const int64_t total = t.end[t.count - 1];
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        int k = 0;
        while (i >= t.end[k]) ++k;
        const int64_t j = i - (k ? t.end[k - 1] : 0);
        float x = t.p[k][j], dx = t.g[k][j];
        float u = x, du = dx;
        if (t.mode[k] == GS_ADAM_LOG) {
            u = logf(x);
            du = dx * x;
        } else if (t.mode[k] == GS_ADAM_LOGIT) {
            x = fminf(fmaxf(x, 1e-6f), 1.f - 1e-6f);
            u = logf(x / (1.f - x));
            du = dx * x * (1.f - x);
        }
        const float m = t.b1 * t.m[k][j] + t.omb1 * du;
        const float v = t.b2 * t.v[k][j] + t.omb2 * du * du;
        u -= t.lr[k] * (m * t.inv_bc1) / (sqrtf(v) * t.inv_sqrt_bc2 + t.eps);
        if (t.mode[k] == GS_ADAM_LOG)
            x = expf(u);
        else if (t.mode[k] == GS_ADAM_LOGIT)
            x = 1.f / (1.f + expf(-u));
        else
            x = u;
        t.p[k][j] = x;
        t.m[k][j] = m;
        t.v[k][j] = v;
        if (t.zero_grad) t.g[k][j] = 0.f;
    }
}

}  // namespace

gs_status launch_adam(const gs_adam_group* groups, int32_t n_groups, double b1, double b2, double eps, int64_t step,
                      int32_t zero_grad, hipStream_t s) {
    const double bc1 = 1.0 - std::pow(b1, (double)step), bc2 = 1.0 - std::pow(b2, (double)step);
    AdamTable t{};
    int64_t acc = 0;
    auto flush = [&]() -> gs_status {
        if (t.count == 0) return GS_OK;
        t.zero_grad = zero_grad;
        t.b1 = (float)b1, t.b2 = (float)b2, t.eps = (float)eps;
        t.omb1 = (float)(1.0 - b1), t.omb2 = (float)(1.0 - b2);
        t.inv_bc1 = (float)(1.0 / bc1);
        t.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
        const int64_t blocks = std::min<int64_t>((acc + NT - 1) / NT, 8192);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(NT), 0, s, t);
        t = AdamTable{};
        acc = 0;
        return check_launch("adam_step");
    };
    for (int k = 0; k < n_groups; ++k) {
        if (groups[k].count == 0) continue;
        const int c = t.count++;
        t.p[c] = groups[k].param, t.g[c] = groups[k].grad, t.m[c] = groups[k].m, t.v[c] = groups[k].v;
        acc += groups[k].count;
        t.end[c] = acc;
        t.lr[c] = groups[k].lr;
        t.mode[c] = groups[k].mode;
        if (t.count == GROUPS_PER_LAUNCH) {
            gs_status st = flush();
            if (st != GS_OK) return st;
        }
    }
    return flush();
}

}  // namespace gs
