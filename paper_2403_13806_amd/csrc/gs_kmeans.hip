// Lloyd iterations of k-means on the device, for camera sets too large for the host loop
// (Sec. 3.4 clusters the input camera centres with k-means). FP64 throughout.
//
// One iteration is two launches, each of which returns at once when the clustering has
// converged (a flag in the workspace), so the host enqueues max_iter iterations without
// waiting on the device:
//   k_km_assign  one lane per point: nearest centre (centres in LDS), squared distance as
//                (dx dx + dy dy) + dz dz without fused multiply-add, ties to the lowest centre;
//                whether any assignment changed; per workgroup the point farthest from its
//                centre (largest distance, ties to the lowest index) and, for every cluster, the
//                sums and count of the workgroup's points in it, added in index order from LDS
//   k_km_update  converged (no assignment changed after the first iteration): set the flag;
//                otherwise one workgroup per cluster sums the workgroup partials (each lane a
//                fixed stride in order, then a fixed tree) and moves the centre to the mean; a
//                centre with no points moves to the farthest point
// A last k_km_assign assigns the points to the final centres. The order of every FP64 sum is
// fixed, so results do not change from run to run; they differ from a sequential sum in the
// last bits only. The farthest point is a maximum with a lowest-index tie rule, exact in any
// order.
#include <algorithm>

#include "gs_device.hpp"

namespace gs {

namespace {

constexpr int KT = 256;          // threads per workgroup, points per assignment workgroup
constexpr int KM_KMAX = 2048;    // centres held in LDS by the assignment pass (48 KiB)
constexpr int KM_GROUPS = 8;     // runs of points per workgroup in the partial sums

struct KmState {
    int32_t done;
};

struct KmFar {
    double d;
    int64_t i;
};

struct KmPart {
    double x, y, z;
    int64_t n;
};

struct KmLayout {
    KmState* st;
    int32_t* changed;  // [max_iter]: an assignment changed in iteration it
    KmFar* far;        // [assign workgroups]
    KmPart* part;      // [assign workgroups][k]
};

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }
int64_t km_blocks(int64_t m) { return (m + KT - 1) / KT; }

KmLayout km_layout(void* ws, int64_t m, int32_t k, int32_t max_iter) {
    KmLayout L;
    char* p = static_cast<char*>(ws);
    L.st = reinterpret_cast<KmState*>(p);
    p += a256(sizeof(KmState));
    L.changed = reinterpret_cast<int32_t*>(p);
    p += a256(sizeof(int32_t) * (size_t)max_iter);
    L.far = reinterpret_cast<KmFar*>(p);
    p += a256(sizeof(KmFar) * (size_t)km_blocks(m));
    L.part = reinterpret_cast<KmPart*>(p);
    return L;
}

__device__ __forceinline__ double sq3(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ bool farther(double d, int64_t i, double bd, int64_t bi) {
    return d > bd || (d == bd && i < bi);
}

__global__ void __launch_bounds__(KT) k_km_init(int32_t* __restrict__ assign, int64_t m,
                                                int32_t* __restrict__ changed, int32_t max_iter,
                                                KmState* __restrict__ st, int32_t* __restrict__ iterations) {
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    if (i < m) assign[i] = -1;
    if (i < max_iter) changed[i] = 0;
    if (i == 0) {
        st->done = 0;
        if (iterations) *iterations = 0;
    }
}

__global__ void __launch_bounds__(KT) k_km_assign(const double* __restrict__ pos, int64_t m,
                                                  const double* __restrict__ centres, int32_t k,
                                                  int32_t* __restrict__ assign, int32_t* __restrict__ changed,
                                                  KmFar* __restrict__ far, KmPart* __restrict__ part,
                                                  const KmState* __restrict__ st, int last) {
    extern __shared__ double s_c[];  // [k][3]
    __shared__ double s_x[3][KT];
    __shared__ int32_t s_a[KT];
    __shared__ KmPart s_q[KT];
    __shared__ KmFar s_far[KT / GS_WAVE];
    __shared__ int s_any;
    if (!last && st->done) return;
    const int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x;
    // the point and its previous assignment are loaded before the centres are staged
    double px = 0, py = 0, pz = 0;
    int32_t old = -1;
    if (i < m) {
        px = pos[3 * i];
        py = pos[3 * i + 1];
        pz = pos[3 * i + 2];
        if (!last) old = assign[i];
    }
    for (int j = threadIdx.x; j < 3 * k; j += KT) s_c[j] = centres[j];
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    double bd = -1.0;
    int64_t bi = i;
    int32_t best = -1;
    if (i < m) {
        best = 0;
        bd = sq3(px - s_c[0], py - s_c[1], pz - s_c[2]);
        for (int32_t c = 1; c < k; ++c) {
            const double d = sq3(px - s_c[3 * c], py - s_c[3 * c + 1], pz - s_c[3 * c + 2]);
            if (d < bd) {
                bd = d;
                best = c;
            }
        }
        if (!last && old != best) s_any = 1;
        assign[i] = best;
        s_x[0][threadIdx.x] = px;
        s_x[1][threadIdx.x] = py;
        s_x[2][threadIdx.x] = pz;
    }
    if (last) return;
    s_a[threadIdx.x] = best;  // -1 past the end of the points
    // farthest point of the workgroup
#pragma unroll
    for (int o = GS_WAVE / 2; o > 0; o >>= 1) {
        const double od = __shfl_xor(bd, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (farther(od, oi, bd, bi)) {
            bd = od;
            bi = oi;
        }
    }
    const int w = threadIdx.x / GS_WAVE;
    if ((threadIdx.x & (GS_WAVE - 1)) == 0) s_far[w] = KmFar{bd, bi};
    __syncthreads();
    if (threadIdx.x == 0) {
        KmFar f = s_far[0];
        for (int v = 1; v < KT / GS_WAVE; ++v)
            if (farther(s_far[v].d, s_far[v].i, f.d, f.i)) f = s_far[v];
        far[blockIdx.x] = f;
        if (s_any) *changed = 1;
    }
    // per cluster, the sums of the workgroup's points in index order. With kp = k rounded up to a
    // power of two (at most KT), `groups` sets of kp lanes each cover one run of consecutive
    // points, lane c of a set taking cluster c; the runs' sums are then added in run order
    int kp = 1;
    while (kp < k && kp < KT) kp <<= 1;
    const int groups = std::min(KT / kp, KM_GROUPS), run = KT / groups;
    const int n_here = (int)std::min<int64_t>(KT, m - (int64_t)blockIdx.x * KT);
    if ((int)threadIdx.x < groups * kp) {
        const int q = threadIdx.x / kp, j0 = q * run, j1 = std::min(j0 + run, n_here);
        for (int32_t c = threadIdx.x % kp; c < k; c += kp) {
            double x = 0, y = 0, z = 0;
            int64_t n = 0;
#pragma unroll 8
            for (int j = j0; j < j1; ++j) {
                const bool hit = s_a[j] == c;
                x += hit ? s_x[0][j] : 0.0;
                y += hit ? s_x[1][j] : 0.0;
                z += hit ? s_x[2][j] : 0.0;
                n += hit;
            }
            if (groups == 1)
                part[(int64_t)blockIdx.x * k + c] = KmPart{x, y, z, n};
            else
                s_q[q * kp + c] = KmPart{x, y, z, n};
        }
    }
    if (groups > 1) {
        __syncthreads();
        for (int32_t c = threadIdx.x; c < k; c += KT) {
            KmPart p = s_q[c];
            for (int q = 1; q < groups; ++q) {
                p.x += s_q[q * kp + c].x;
                p.y += s_q[q * kp + c].y;
                p.z += s_q[q * kp + c].z;
                p.n += s_q[q * kp + c].n;
            }
            part[(int64_t)blockIdx.x * k + c] = p;
        }
    }
}

__global__ void __launch_bounds__(KT) k_km_update(const double* __restrict__ pos, double* __restrict__ centres,
                                                  int32_t k, const KmPart* __restrict__ part,
                                                  const KmFar* __restrict__ far, int64_t n_blocks,
                                                  const int32_t* __restrict__ changed, int32_t it,
                                                  KmState* __restrict__ st, int32_t* __restrict__ iterations) {
    __shared__ KmPart s_p[KT / GS_WAVE];
    __shared__ KmFar s_far[KT / GS_WAVE];
    __shared__ int64_t s_n;
    if (st->done) return;
    if (it > 0 && *changed == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 1;
        return;
    }
    const int32_t c = blockIdx.x;
    const int w = threadIdx.x / GS_WAVE;
    double x = 0, y = 0, z = 0;
    int64_t n = 0;
    for (int64_t b = threadIdx.x; b < n_blocks; b += KT) {
        const KmPart p = part[b * k + c];
        x += p.x;
        y += p.y;
        z += p.z;
        n += p.n;
    }
#pragma unroll
    for (int o = GS_WAVE / 2; o > 0; o >>= 1) {
        x += __shfl_xor(x, o);
        y += __shfl_xor(y, o);
        z += __shfl_xor(z, o);
        n += __shfl_xor(n, o);
    }
    if ((threadIdx.x & (GS_WAVE - 1)) == 0) s_p[w] = KmPart{x, y, z, n};
    __syncthreads();
    if (threadIdx.x == 0) {
        KmPart p = s_p[0];
        for (int v = 1; v < KT / GS_WAVE; ++v) {
            p.x += s_p[v].x;
            p.y += s_p[v].y;
            p.z += s_p[v].z;
            p.n += s_p[v].n;
        }
        s_n = p.n;
        if (p.n > 0) {
            const double dn = (double)p.n;
            centres[3 * c] = p.x / dn;
            centres[3 * c + 1] = p.y / dn;
            centres[3 * c + 2] = p.z / dn;
        }
        if (c == 0 && iterations) *iterations = it + 1;
    }
    __syncthreads();
    if (s_n > 0) return;
    // an empty cluster: the point farthest from its centre over the whole assignment
    double fd = -1.0;
    int64_t fi = 0;
    for (int64_t b = threadIdx.x; b < n_blocks; b += KT)
        if (farther(far[b].d, far[b].i, fd, fi)) {
            fd = far[b].d;
            fi = far[b].i;
        }
#pragma unroll
    for (int o = GS_WAVE / 2; o > 0; o >>= 1) {
        const double od = __shfl_xor(fd, o);
        const int64_t oi = __shfl_xor(fi, o);
        if (farther(od, oi, fd, fi)) {
            fd = od;
            fi = oi;
        }
    }
    if ((threadIdx.x & (GS_WAVE - 1)) == 0) s_far[w] = KmFar{fd, fi};
    __syncthreads();
    if (threadIdx.x == 0) {
        KmFar f = s_far[0];
        for (int v = 1; v < KT / GS_WAVE; ++v)
            if (farther(s_far[v].d, s_far[v].i, f.d, f.i)) f = s_far[v];
        centres[3 * c] = pos[3 * f.i];
        centres[3 * c + 1] = pos[3 * f.i + 1];
        centres[3 * c + 2] = pos[3 * f.i + 2];
    }
}

}  // namespace

int32_t kmeans_max_centres() { return KM_KMAX; }

size_t kmeans_workspace_bytes(int64_t m, int32_t k, int32_t max_iter) {
    if (m < 1 || k < 1 || max_iter < 1) return 0;
    return a256(sizeof(KmState)) + a256(sizeof(int32_t) * (size_t)max_iter) + a256(sizeof(KmFar) * km_blocks(m)) +
           a256(sizeof(KmPart) * (size_t)k * km_blocks(m));
}

gs_status launch_kmeans_lloyd(const double* pos, int64_t m, int32_t k, int32_t max_iter, double* centres,
                              int32_t* assign, int32_t* iterations, void* ws, hipStream_t s) {
    const KmLayout L = km_layout(ws, m, k, max_iter);
    const int64_t nb = km_blocks(m);
    const unsigned ni = (unsigned)((std::max<int64_t>(m, max_iter) + KT - 1) / KT);
    const size_t lds = sizeof(double) * 3 * (size_t)k;
    hipLaunchKernelGGL(k_km_init, dim3(ni), dim3(KT), 0, s, assign, m, L.changed, max_iter, L.st, iterations);
    for (int32_t it = 0; it < max_iter; ++it) {
        int32_t* ch = L.changed + it;
        hipLaunchKernelGGL(k_km_assign, dim3((unsigned)nb), dim3(KT), lds, s, pos, m, centres, k, assign, ch, L.far,
                           L.part, L.st, 0);
        hipLaunchKernelGGL(k_km_update, dim3((unsigned)k), dim3(KT), 0, s, pos, centres, k, L.part, L.far, nb, ch, it,
                           L.st, iterations);
    }
    hipLaunchKernelGGL(k_km_assign, dim3((unsigned)nb), dim3(KT), lds, s, pos, m, centres, k, assign, L.changed,
                       L.far, L.part, L.st, 1);
    return check_launch("kmeans_lloyd");
}

}  // namespace gs
