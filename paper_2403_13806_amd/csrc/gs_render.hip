// Per-tile front-to-back compositing (eq. render-gs) and the two passes built on the same
// traversal: the max-over-rays importance score (eq. importance-score) and per-cluster
// visibility bits (eq. importance-score-vis); plus the reverse traversal that gives the
// gradients of the 2D quantities.
//
// One workgroup per tile, one pixel per lane. Each wave owns an 8x8 pixel block. The
// tile's sorted list is streamed through LDS in batches of DEPTH records per lane (64-byte
// records, coalesced loads); while a batch is staged, each loading lane marks which wave
// blocks its record's support box meets, and each wave then walks only its hits (ballot
// masks and scalar bit scans), so records that miss a block cost that wave nothing. The
// support test d^T conic d <= q_max runs in FP64 -- same issue rate as FP32 on CDNA4 -- so
// it agrees with an FP64 evaluation; the exponential and the transmittance are FP32.
//
// One workgroup per tile. Workgroup b takes tile b, or, in the longest-first (LPT) order,
// the b-th entry of a list of tiles sorted by decreasing list length: workgroups are
// dispatched in increasing b as resources free up, so the dispatcher itself hands out the
// longest tiles first, with no queue counter to reset between launches or graph replays.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "gs_device.hpp"
#include "gs_tile_sort.hpp"

namespace gs {

// MODE_FWD_COUNT is the forward pass that also counts the entries composited into each pixel
// (gs_render_fwd with n_contrib); the count costs two VALU instructions per hit, so the plain
// forward leaves it out
enum { MODE_FWD = 0, MODE_IMPORTANCE = 1, MODE_VISIBILITY = 2, MODE_FWD_COUNT = 3 };

struct RenderArgs {
    const gs_splat* splat;
    const uint32_t* vals;
    const uint32_t* ranges;
    const int32_t* tile_offset;
    const int64_t* pixel_offset;
    const gs_camera* cams;
    int n_views;
    int64_t n;
    gs_params p;
    float* rgb;
    float* t_final;
    uint32_t* n_last;
    uint32_t* n_contrib;
    float* h;
    uint32_t* bits;
    const int32_t* view_cluster;
    int64_t words;
    float t_cluster;
    int k_clusters;  // rows of bits; views with a cluster id outside [0, k) set nothing
    // backward
    const float* dl_drgb;
    const float* t_in;
    const uint32_t* last_in;
    const uint64_t* rect;          // [n_views * n] tile rectangles
    const uint32_t* entry_offset;  // [n_views * n] first emission slot of each entry
    uint64_t capacity;             // slots
    float* slots;                  // [capacity][9] per-pair partial gradients
    // longest-first order
    const uint32_t* queue;  // tiles, longest list first, or NULL
};

// bit w set when the support ellipse d^T conic d <= q_max meets the rectangle spanned by
// the pixel centres of wave w's 8x8 block (waves tile the TW x TH tile row-major in 8x8
// blocks; (ox, oy) is the centre of the tile's first pixel). q is a positive-definite
// quadratic with its minimum at the projected mean, so over a rectangle that does not hold
// the mean its minimum lies on an edge facing the mean: the vertical edge at x = clamp(u)
// or the horizontal edge at y = clamp(v). Along a vertical edge at offset ex the minimum is
// at the offset -(b/c) ex clamped to the edge, along a horizontal edge at -(b/a) ey. Both
// candidate points lie in the rectangle and one of them is the minimiser, so the smaller
// of the two values is the minimum of q over the rectangle. The relative and absolute
// margins cover the rounding of these evaluations against the per-pixel test, so a block
// that holds a covered pixel centre is always marked.
// QUARTERS: test the four 4x4 quarters of every wave block instead (bit 4 w + quarter,
// quarters numbered row-major inside the block).
// the support test over the rectangle [x0, x1] x [y0, y1] of pixel-centre offsets from the
// mean (see above); kx = -b/c, ky = -b/a, lim = q_max with the rounding margins
__device__ __forceinline__ bool rect_hit(const gs_splat& s, double x0, double x1, double y0, double y1, double kx,
                                         double ky, double lim) {
    const double ex = fmin(fmax(0.0, x0), x1), ey = fmin(fmax(0.0, y0), y1);
    const double fy = fmin(fmax(kx * ex, y0), y1), fx = fmin(fmax(ky * ey, x0), x1);
    const double q1 = s.ca * ex * ex + 2.0 * s.cb * ex * fy + s.cc * fy * fy;
    const double q2 = s.ca * fx * fx + 2.0 * s.cb * fx * ey + s.cc * ey * ey;
    return fmin(q1, q2) <= lim;
}

// bit w set when the support meets wave w's block of (8 PXW) x 8 pixels (blocks row-major)
template <int TW, int TH, int PXW>
__device__ __forceinline__ uint64_t wave_hits(const gs_splat& s, double ox, double oy) {
    constexpr int BW = 8 * PXW, WPR = TW / BW, NB = WPR * (TH / 8);
    const double kx = -s.cb / s.cc, ky = -s.cb / s.ca;
    const double lim = s.qmax * (1.0 + 1e-9) + 1e-12;
    uint64_t m = 0;
#pragma unroll 1
    for (int w = 0; w < NB; ++w) {
        const double x0 = ox + (double)((w % WPR) * BW) - s.u;
        const double y0 = oy + (double)((w / WPR) * 8) - s.v;
        if (rect_hit(s, x0, x0 + (BW - 1), y0, y0 + 7.0, kx, ky, lim)) m |= 1ull << w;
    }
    return m;
}

// px: the lane's first pixel; with PXW pixels per lane it holds px .. px + PXW - 1 of row py
struct TileGeom {
    int view, W, H, tx, ty, px, py, wave;
    double ox, oy;   // centre of the tile's first pixel
};

template <int TW, int TH, int PXW = 1>
__device__ __forceinline__ TileGeom tile_geom(const RenderArgs& a, int tile) {
    TileGeom g;
    g.view = view_of_tile(a.tile_offset, a.n_views, tile);
    g.W = a.cams[g.view].width;
    g.H = a.cams[g.view].height;
    const int tiles_x = div_up(g.W, TW);
    const int local = tile - a.tile_offset[g.view];
    const int tx = local % tiles_x, ty = local / tiles_x;
    g.tx = tx;
    g.ty = ty;
    const int t = threadIdx.x, l = t & 63;
    g.wave = t >> 6;
    constexpr int BW = 8 * PXW, WPR = TW / BW;
    const int bx = (g.wave % WPR) * BW, by = (g.wave / WPR) * 8;
    g.px = tx * TW + bx + (l & 7) * PXW;
    g.py = ty * TH + by + (l >> 3);
    g.ox = (double)(tx * TW) + 0.5;
    g.oy = (double)(ty * TH) + 0.5;
    return g;
}

// d^T conic d at the offset (dx, dy) of a pixel centre from the projected mean: FP64, one
// fixed order of operations shared by every traversal, so the forward pass, the importance
// pass and the reverse traversal take identical support and opacity decisions
__device__ __forceinline__ double quad(const gs_splat& s, double dx, double dy) {
    return fma(s.cc * dy, dy, dx * fma(2.0 * s.cb, dy, s.ca * dx));
}

// min(alpha_max, o G) for o G >= 0 in one instruction
__device__ __forceinline__ float clamp_alpha(float og, float amax) { return __builtin_amdgcn_fmed3f(og, 0.f, amax); }

// exp(-q/2) in FP32, as 2^(q * (-log2(e) / 2))
__device__ __forceinline__ float falloff(double q) {
    return __builtin_amdgcn_exp2f((float)q * -0.72134752044448170368f);
}

template <int TW, int TH, int DEPTH, int PXW = 1>
struct Smem {
    static constexpr int NT = TW * TH / PXW;  // threads
    static constexpr int BD = NT * DEPTH;     // records per batch
    gs_splat rec[BD];
    uint32_t gid[BD];
    uint16_t hit[BD];   // bit w: the record meets wave w's 8x8 block (up to 16 waves)
    uint32_t hacc[BD];  // importance: max weight bits per staged record; visibility: flag
    uint32_t top;
};

// The reverse traversal: each lane holds a cluster of PXW x PXH neighbouring pixels, a wave an
// (8 PXW) x (8 PXH) block of the tile, and each row of 16 lanes (a quarter of the wave) a
// (4 PXW) x (4 PXH) part of it. It stages BB records per batch and keeps, per wave and staged
// record, the nine 2D-gradient sums of that wave's pixels: the waves' sums are combined in
// wave order when the batch is flushed, so every per-pair sum is formed in a fixed order.
template <int TW, int TH, int PXW, int PXH>
struct BwdShape {
    static constexpr int P = PXW * PXH;           // pixels per lane
    static constexpr int NT = TW * TH / P;        // threads
    static constexpr int NW = NT / 64;            // waves
    static constexpr int BW = 8 * PXW, BH = 8 * PXH;  // wave block
    static constexpr int WPR = TW / BW;           // waves per row of blocks
    static constexpr int BB = NT < 128 ? NT : 128;  // records per batch
    static constexpr int SH = NT / BB;              // threads staging one record (each tests every SH-th block)
    static_assert(TW % BW == 0 && TH % BH == 0 && NW >= 1, "tile not a whole number of wave blocks");
    static_assert(NW * 4 <= 64, "quarter masks hold 64 bits");
};

template <int TW, int TH, int PXW, int PXH>
struct SmemBwd {
    using S = BwdShape<TW, TH, PXW, PXH>;
    gs_splat rec[S::BB];
    uint64_t hitq[S::SH][S::BB];  // quarter masks, bit 4 w + quarter, in SH parts (OR-ed when read)
    uint32_t gid[S::BB];
    float acc[S::NW * S::BB * 9];  // [wave][record][field]
    uint32_t top;
};

// stage records [base, base + cnt) of the tile's list; mark the wave blocks each one meets
template <int TW, int TH, int DEPTH, int PXW>
__device__ __forceinline__ void stage(Smem<TW, TH, DEPTH, PXW>& sm, const RenderArgs& a, const gs_splat* sp,
                                      uint32_t base, uint32_t cnt, const TileGeom& g) {
    constexpr int NT = Smem<TW, TH, DEPTH, PXW>::NT;
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
        const uint32_t q = threadIdx.x + d * NT;
        uint64_t hm = 0;
        const uint32_t id = q < cnt ? a.vals[base + q] : 0xffffffffu;
        if ((int64_t)id < a.n) {  // (out of range only in the output of a timed-out sort)
            const gs_splat s = sp[id];
            sm.rec[q] = s;
            sm.gid[q] = id;
            hm = wave_hits<TW, TH, PXW>(s, g.ox, g.oy);
        }
        sm.hit[q] = (uint16_t)hm;
    }
}

// the backward's staging: records [base, base + cnt) with their quarter masks
template <int TW, int TH, int PXW, int PXH>
__device__ __forceinline__ void stage_q(SmemBwd<TW, TH, PXW, PXH>& sm, const RenderArgs& a, const gs_splat* sp,
                                        uint32_t base, uint32_t cnt, double ox, double oy) {
    using S = BwdShape<TW, TH, PXW, PXH>;
    // SH threads per record (all of the workgroup's threads when it has more than BB): thread
    // part h tests the quarters 4 w + qd = h, h + SH, ...; the FP64 tests are the staging's
    // critical path, so splitting them shortens every batch's wait at the barrier
    const uint32_t q = threadIdx.x % S::BB, h = threadIdx.x / S::BB;
    uint64_t hm = 0;
    const uint32_t id = q < cnt ? a.vals[base + q] : 0xffffffffu;
    if ((int64_t)id < a.n) {  // (out of range only in the output of a timed-out sort)
        const gs_splat s = sp[id];
        if (h == 0) sm.rec[q] = s;
        const double kx = -s.cb / s.cc, ky = -s.cb / s.ca;
        const double lim = s.qmax * (1.0 + 1e-9) + 1e-12;
#pragma unroll 1
        for (int bit = (int)h; bit < 4 * S::NW; bit += S::SH) {
            const int w = bit >> 2, qd = bit & 3;
            const double x0 = ox + (double)((w % S::WPR) * S::BW + (qd & 1) * 4 * PXW) - s.u;
            const double y0 = oy + (double)((w / S::WPR) * S::BH + (qd >> 1) * 4 * PXH) - s.v;
            if (rect_hit(s, x0, x0 + (4 * PXW - 1), y0, y0 + (4 * PXH - 1), kx, ky, lim)) hm |= 1ull << bit;
        }
    }
    if (h == 0) sm.gid[q] = (int64_t)id < a.n ? id : 0xffffffffu;
    sm.hitq[h][q] = hm;
}

// emission slot of the pair (tile (tx, ty) of its view, entry o): entry o's pairs are
// numbered from entry_offset[o] over the tiles of its rectangle in row-major order
__device__ __forceinline__ uint64_t pair_slot(const RenderArgs& a, int64_t o, int tx, int ty) {
    const uint64_t r = a.rect[o];
    const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff;
    return (uint64_t)a.entry_offset[o] + (uint64_t)((uint32_t)ty - y0) * (x1 - x0 + 1u) + ((uint32_t)tx - x0);
}

template <int TW, int TH, int DEPTH, int MODE, int PXW>
__device__ void fwd_tile(Smem<TW, TH, DEPTH, PXW>& sm, const RenderArgs& a, int tile) {
    using SM = Smem<TW, TH, DEPTH, PXW>;
    constexpr int NT = SM::NT, BD = SM::BD;
    const TileGeom g = tile_geom<TW, TH, PXW>(a, tile);
    const int l = threadIdx.x & 63, w = g.wave;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const double yc = (double)g.py + 0.5;
    const float amax = a.p.alpha_max, tmin = a.p.t_min;
    const gs_splat* sp = a.splat + (int64_t)g.view * a.n;
    // T < t_min marks a finished ray; pixels outside the view start finished (T = -1, t_min >= 0)
    double xc[PXW];
    float T[PXW], C0[PXW], C1[PXW], C2[PXW];
    uint32_t last[PXW], ncomp[PXW];
#pragma unroll
    for (int i = 0; i < PXW; ++i) {
        xc[i] = (double)(g.px + i) + 0.5;
        T[i] = (g.px + i < g.W && g.py < g.H) ? 1.f : -1.f;
        C0[i] = C1[i] = C2[i] = 0.f;
        last[i] = start;
        ncomp[i] = 0;
    }
    int cluster = 0;
    bool cluster_ok = true;
    if (MODE == MODE_VISIBILITY) {
        cluster = a.view_cluster[g.view];
        cluster_ok = (unsigned)cluster < (unsigned)a.k_clusters;
    }
    for (uint32_t base = start; base < end; base += BD) {
        bool alive = false;
#pragma unroll
        for (int i = 0; i < PXW; ++i) alive |= T[i] >= tmin;
        if (__syncthreads_and(!alive)) break;
        const uint32_t cnt = min((uint32_t)BD, end - base);
        stage<TW, TH, DEPTH, PXW>(sm, a, sp, base, cnt, g);
        if (MODE == MODE_IMPORTANCE || MODE == MODE_VISIBILITY) {
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) sm.hacc[threadIdx.x + d * NT] = 0u;
        }
        __syncthreads();
        // each wave walks only the entries that meet its block, in list order
#pragma unroll 1
        for (int c = 0; c < BD / 64; ++c) {
            uint64_t m = ballot((sm.hit[c * 64 + l] >> w) & 1u);
            while (m) {
                const int j = c * 64 + (int)__builtin_ctzll(m);
                m &= m - 1;
                // the whole record is read up front and the body is branch-free apart from the
                // wave-uniform skip, so no LDS wait sits inside a divergent region
                const gs_splat s = sm.rec[j];
                // opacity and colour are requested together with the geometry
                asm volatile("" ::"v"(s.opacity), "v"(s.rgb[0]), "v"(s.rgb[1]), "v"(s.rgb[2]));
                double q[PXW];
                bool in[PXW];
                bool any = false;
#pragma unroll
                for (int i = 0; i < PXW; ++i) {
                    q[i] = quad(s, xc[i] - s.u, yc - s.v);
                    in[i] = (q[i] <= s.qmax) & (T[i] >= tmin);
                    any |= in[i];
                }
                if (ballot(any) == 0) continue;
                float wmax = 0.f;
                bool above = false;
#pragma unroll
                for (int i = 0; i < PXW; ++i) {
                    const float al = in[i] ? clamp_alpha(s.opacity * falloff(q[i]), amax) : 0.f;
                    const float wgt = al * T[i];
                    if (MODE == MODE_FWD || MODE == MODE_FWD_COUNT) {  // colours are finite: wgt = 0 adds nothing
                        C0[i] = fmaf(wgt, s.rgb[0], C0[i]);
                        C1[i] = fmaf(wgt, s.rgb[1], C1[i]);
                        C2[i] = fmaf(wgt, s.rgb[2], C2[i]);
                    }
                    T[i] = T[i] * (1.f - al);
                    last[i] = in[i] ? base + j + 1 : last[i];
                    if (MODE == MODE_FWD_COUNT) ncomp[i] += in[i] ? 1u : 0u;
                    wmax = fmaxf(wmax, wgt);
                    above |= wgt > a.t_cluster;
                }
                // per staged record, combined over the workgroup's waves in LDS
                if (MODE == MODE_IMPORTANCE) {
                    if (ballot(wmax > 0.f)) {
                        const float mx = wave_max_nonneg(wmax);
                        if (l == 0) atomicMax(&sm.hacc[j], __float_as_uint(mx));
                    }
                }
                if (MODE == MODE_VISIBILITY) {
                    if (ballot(above) != 0 && l == 0) atomicOr(&sm.hacc[j], 1u);
                }
            }
            bool alive2 = false;
#pragma unroll
            for (int i = 0; i < PXW; ++i) alive2 |= T[i] >= tmin;
            if (ballot(alive2) == 0) break;
        }
        if (MODE == MODE_IMPORTANCE || MODE == MODE_VISIBILITY) {
            // one device-wide atomic per (tile, record) at most, and none when the value held
            // already covers it (a stale read can only cause a redundant atomic)
            __syncthreads();
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
                const uint32_t qq = threadIdx.x + d * NT;
                const uint32_t v = sm.hacc[qq];
                if (qq < cnt && v != 0u && cluster_ok) {
                    const uint32_t id = sm.gid[qq];
                    if (MODE == MODE_IMPORTANCE) {
                        unsigned int* hp = reinterpret_cast<unsigned int*>(a.h) + id;
                        if (v > *hp) atomicMax(hp, v);
                    } else {
                        uint32_t* bp = a.bits + (int64_t)cluster * a.words + (id >> 5);
                        const uint32_t bit = 1u << (id & 31);
                        if (!(*bp & bit)) atomicOr(bp, bit);
                    }
                }
            }
        }
    }
    if (MODE == MODE_FWD || MODE == MODE_FWD_COUNT) {
        const int64_t plane = (int64_t)g.W * g.H, poff = a.pixel_offset[g.view];
#pragma unroll
        for (int i = 0; i < PXW; ++i) {
            if (g.px + i < g.W && g.py < g.H) {
                const int64_t pix = poff + (int64_t)g.py * g.W + g.px + i;
                float* out = a.rgb + 3 * poff + (int64_t)g.py * g.W + g.px + i;
                out[0] = C0[i] + T[i] * a.p.bg[0];
                out[plane] = C1[i] + T[i] * a.p.bg[1];
                out[2 * plane] = C2[i] + T[i] * a.p.bg[2];
                a.t_final[pix] = T[i];
                a.n_last[pix] = last[i];
                if (MODE == MODE_FWD_COUNT) a.n_contrib[pix] = ncomp[i];
            }
        }
    }
}

// Nine per-lane values summed over each row of 16 lanes by a transposing butterfly: at
// every step a lane adds its partner's copy of half of the fields it still holds and keeps
// that half, so after four steps each lane holds the row sum of one field. Lane i keeps
// the upper half at the steps pairing it with i^1, i^2, i^7 and i^15 when s1 = b0^b2,
// s2 = b1^b2, s3 = b2^b3 and s4 = b3 are set (b the bits of i within the row): partners
// differ in the selector of their own step and agree in every earlier one, so they hold the
// same fields when they exchange. The field ends up as f = s1 + 2 s2 + 4 s3 + 8 s4; fields
// 9..15 are zero padding. Must be called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ float pair_add(float x) {
    return x + __int_as_float(dpp<CTRL>(__float_as_int(x)));
}

__device__ __forceinline__ int row_sum9_field(int lane) {
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    return (b0 ^ b2) + 2 * (b1 ^ b2) + 4 * (b2 ^ b3) + 8 * b3;
}

__device__ __forceinline__ float row_sum9(const float (&v)[9], int lane) {
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
    const bool s1 = b0 ^ b2, s2 = b1 ^ b2, s3 = b2 ^ b3, s4 = b3;
    // every cross-lane add is computed by all lanes before the selects (a DPP read inside a
    // divergent branch would see inactive source lanes)
    float w[5], x[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float lo = pair_add<0xB1>(v[2 * k]), hi = pair_add<0xB1>(v[2 * k + 1]);
        w[k] = s1 ? hi : lo;
    }
    const float w4 = pair_add<0xB1>(v[8]);
    w[4] = s1 ? 0.f : w4;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float lo = pair_add<0x4E>(w[2 * k]), hi = pair_add<0x4E>(w[2 * k + 1]);
        x[k] = s2 ? hi : lo;
    }
    const float x2 = pair_add<0x4E>(w[4]);
    x[2] = s2 ? 0.f : x2;
    const float y0l = pair_add<0x141>(x[0]), y0h = pair_add<0x141>(x[1]), y1l = pair_add<0x141>(x[2]);
    const float y0 = s3 ? y0h : y0l, y1 = s3 ? 0.f : y1l;
    const float zl = pair_add<0x140>(y0), zh = pair_add<0x140>(y1);
    return s4 ? zh : zl;
}

// Reverse traversal. For pixel entries in back-to-front order, with T the transmittance
// after entry j and S the colour composited behind it (S starts at T_final * bg):
//   T_j = T / (1 - alpha_j), w_j = alpha_j T_j,
//   dL/dc_j = dL/dC * w_j,  dL/dalpha_j = sum_c dL/dC_c (T_j c_jc - S_c / (1 - alpha_j)),
// kept per pixel as U = dL/dC . S (U += w_j Q_j with Q_j = dL/dC . c_j, so that
// dL/dalpha_j = T_j Q_j - U / (1 - alpha_j)),
// then alpha = o G (unless clamped), G = exp(-q/2), q = a dx^2 + 2 b dx dy + c dy^2,
// dx = xc - u. Each row of 16 lanes holds a 4x4 quarter of the wave's block and walks only
// the entries that meet its quarter, so one iteration serves up to four entries; the nine
// per-entry sums are reduced over the row and added into the wave's own LDS accumulator of
// the entry. When a batch is done, its records' wave sums are added in wave order and
// stored (plain stores) into each pair's emission slot; pairs behind every pixel's last
// entry get zeros. Each Gaussian's slots are then summed by the parameter chains.
template <int TW, int TH, int PXW, int PXH>
__device__ void bwd_tile(SmemBwd<TW, TH, PXW, PXH>& sm, const RenderArgs& a, int tile) {
    using S = BwdShape<TW, TH, PXW, PXH>;
    constexpr int NT = S::NT, BB = S::BB, NW = S::NW, P = S::P;
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int fld = row_sum9_field(l);
    const int view = view_of_tile(a.tile_offset, a.n_views, tile);
    const int W = a.cams[view].width, H = a.cams[view].height;
    const int tiles_x = div_up(W, TW);
    const int local = tile - a.tile_offset[view];
    const int tx = local % tiles_x, ty = local / tiles_x;
    // lane (lx, ly) of the wave's 8 x 8 lane grid: quarter qd = l / 16 (row-major 2 x 2), 4 x 4
    // lanes each; its pixels are the PXW x PXH cluster at (px0, py0)
    const int qd = l >> 4, sl = l & 15;
    const int lx = (qd & 1) * 4 + (sl & 3), ly = (qd >> 1) * 4 + (sl >> 2);
    const int px0 = tx * TW + (w % S::WPR) * S::BW + lx * PXW;
    const int py0 = ty * TH + (w / S::WPR) * S::BH + ly * PXH;
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const float amax = a.p.alpha_max;
    const gs_splat* sp = a.splat + (int64_t)view * a.n;
    const int64_t plane = (int64_t)W * H, poff = a.pixel_offset[view];
    double xc[PXW], yc[PXH];
#pragma unroll
    for (int i = 0; i < PXW; ++i) xc[i] = (double)(px0 + i) + 0.5;
#pragma unroll
    for (int j = 0; j < PXH; ++j) yc[j] = (double)(py0 + j) + 0.5;
    float T[P], dC[P][3], U[P];
    uint32_t last[P];
    bool inside[P];
    uint32_t lmax = start;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int px = px0 + p % PXW, py = py0 + p / PXW;
        inside[p] = px < W && py < H;
        T[p] = 1.f;
        last[p] = start;
#pragma unroll
        for (int c = 0; c < 3; ++c) dC[p][c] = 0.f;
        U[p] = 0.f;
        if (inside[p]) {
            const int64_t pix = poff + (int64_t)py * W + px;
            T[p] = a.t_in[pix];
            last[p] = a.last_in[pix];
            const float* d = a.dl_drgb + 3 * poff + (int64_t)py * W + px;
#pragma unroll
            for (int c = 0; c < 3; ++c) dC[p][c] = d[c * plane];
            U[p] = T[p] * (dC[p][0] * a.p.bg[0] + dC[p][1] * a.p.bg[1] + dC[p][2] * a.p.bg[2]);
        }
        // never read outside the tile's list, whatever n_last holds
        last[p] = min(max(last[p], start), end);
        lmax = max(lmax, inside[p] ? last[p] : start);
    }
    if (t == 0) sm.top = start;
    __syncthreads();
    if (lmax > start) atomicMax(&sm.top, lmax);
    __syncthreads();
    const uint32_t top = sm.top;
    // each quarter's last composited entry (max over its pixels): entries behind it are skipped
    int ql = (int)lmax;
    ql = max(ql, dpp<0xB1>(ql));
    ql = max(ql, dpp<0x4E>(ql));
    ql = max(ql, dpp<0x141>(ql));
    ql = max(ql, dpp<0x140>(ql));
    int64_t qlast[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qlast[k] = (int64_t)(uint32_t)__builtin_amdgcn_readlane(ql, 16 * k);
    const int64_t vbase = (int64_t)view * a.n;
    const double ox = (double)(tx * TW) + 0.5, oy = (double)(ty * TH) + 0.5;
    const int accw = w * (BB * 9);  // this wave's accumulators in sm.acc
    for (int q = t; q < NW * BB * 9; q += NT) sm.acc[q] = 0.f;
    for (uint32_t hi = top; hi > start;) {
        const uint32_t lo = (hi - start > (uint32_t)BB) ? hi - BB : start;
        __syncthreads();
        stage_q<TW, TH, PXW, PXH>(sm, a, sp, lo, hi - lo, ox, oy);
        __syncthreads();
        // entries that meet this wave's block, back to front
#pragma unroll 1
        for (int c = BB / 64 - 1; c >= 0; --c) {
            // each quarter (one row of 16 lanes) walks the entries that meet its pixels
            // the four quarters' masks are wave-uniform: their bit walks run on the scalar unit
            uint64_t hm = sm.hitq[0][c * 64 + l];
#pragma unroll
            for (int h = 1; h < S::SH; ++h) hm |= sm.hitq[h][c * 64 + l];
            const uint32_t hq = (uint32_t)(hm >> (4 * w));
            uint64_t mq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t m = ballot((hq >> k) & 1u);
                const int64_t lim = qlast[k] - (int64_t)(lo + c * 64);
                mq[k] = lim <= 0 ? 0ull : (lim >= 64 ? m : m & ((1ull << lim) - 1ull));
            }
            while (mq[0] | mq[1] | mq[2] | mq[3]) {
                // byte k of pk: quarter k's record (highest set bit), or 128 when it has none
                uint32_t pk = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t bk = mq[k] ? 63u - (uint32_t)__builtin_clzll(mq[k]) : 128u;
                    mq[k] &= ~(1ull << (bk & 63u));  // (no change when empty)
                    pk |= bk << (8 * k);
                }
                const uint32_t braw = (pk >> (8 * qd)) & 255u;
                const bool act = braw < 64u;
                const int b = (int)(braw & 63u);
                const int j = c * 64 + b;
                const uint32_t pos = lo + j;
                // whole record up front; branch-free body apart from the wave-uniform skip
                const gs_splat s = sm.rec[j];
                asm volatile("" ::"v"(s.opacity), "v"(s.rgb[0]), "v"(s.rgb[1]), "v"(s.rgb[2]));
                double q[P];
                bool con[P];
                bool any = false;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    q[p] = quad(s, xc[p % PXW] - s.u, yc[p / PXW] - s.v);
                    con[p] = act & (q[p] <= s.qmax) & inside[p] & (pos < last[p]);
                    any |= con[p];
                }
                if (ballot(any) == 0) continue;
                // the first pixel's terms start the sums (no adds onto zeros)
                float v[9];
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float G = falloff(q[p]);
                    const float og = s.opacity * G;
                    // where p does not contribute al = 0 and wt = 0: U and the colour sums stay as
                    // they are without a select (inputs are finite)
                    const float al = con[p] ? clamp_alpha(og, amax) : 0.f;
                    const float r = __builtin_amdgcn_rcpf(1.f - al);
                    T[p] = con[p] ? T[p] * r : T[p];
                    const float wt = al * T[p];
                    const float Q = dC[p][0] * s.rgb[0] + dC[p][1] * s.rgb[1] + dC[p][2] * s.rgb[2];
                    const float dA = T[p] * Q - U[p] * r;
                    U[p] = fmaf(wt, Q, U[p]);  // wt = 0 where p does not contribute
                    // dq dx, dq dy (turned into the u, v gradients with the conic once per record
                    // in the flush), a b c o r g b; the geometric terms vanish where alpha is clamped
                    // (the constant factors of dq/dalpha, -1/2, and of the b term, 2, are applied
                    // to the sums in the flush: scaling by powers of two is exact)
                    const bool free_a = con[p] & (og < amax);
                    const float dx = (float)(xc[p % PXW] - s.u), dy = (float)(yc[p / PXW] - s.v);
                    const float dq = free_a ? al * dA : 0.f;
                    const float a0 = dq * dx, a1 = dq * dy;
                    const float t9[9] = {a0,          a1,          a0 * dx, a0 * dy, a1 * dy, free_a ? dA * G : 0.f,
                                         dC[p][0] * wt, dC[p][1] * wt, dC[p][2] * wt};
#pragma unroll
                    for (int f = 0; f < 9; ++f) v[f] = p == 0 ? t9[f] : v[f] + t9[f];
                }
                // per-quarter sums, one field per lane, added into this wave's sums of that
                // entry (lanes of one instruction that meet at one address are applied in a
                // fixed order, so the result does not depend on timing)
                const float z = row_sum9(v, l);
                if (act & (fld < 9)) atomicAdd(&sm.acc[accw + j * 9 + fld], z);
            }
        }
        __syncthreads();
        // one slot per (tile, record): each (record, field) sum of the waves is formed in wave
        // order (into wave 0's accumulator), then each record's nine sums are stored with plain
        // stores; the sums of dq dx and dq dy become dL/du = -2 (a sx + b sy), dL/dv = -2 (b sx + c sy)
        for (int q = t; q < BB * 9; q += NT) {
            float sum = sm.acc[q];
#pragma unroll 1
            for (int ww = 1; ww < NW; ++ww) {
                sum += sm.acc[ww * BB * 9 + q];
                sm.acc[ww * BB * 9 + q] = 0.f;
            }
            sm.acc[q] = sum;
        }
        __syncthreads();
        const uint32_t cnt = hi - lo;
        if (t < BB) {
            float f9[9];
#pragma unroll
            for (int f = 0; f < 9; ++f) {
                f9[f] = sm.acc[t * 9 + f];
                sm.acc[t * 9 + f] = 0.f;
            }
            const uint32_t id = sm.gid[t];
            if ((uint32_t)t < cnt && id != 0xffffffffu) {
                // the sums are of al dA times (dx, dy, dx^2, dx dy, dy^2); with dq = -al dA / 2,
                // dL/du = -2 (a Sx + b Sy) and dL/d(a, b, c) = (Sxx, 2 Sxy, Syy) over sums of dq
                // are a sx + b sy and (-sxx / 2, -sxy, -syy / 2) over these
                const float sx = f9[0], sy = f9[1];
                f9[0] = (float)sm.rec[t].ca * sx + (float)sm.rec[t].cb * sy;
                f9[1] = (float)sm.rec[t].cb * sx + (float)sm.rec[t].cc * sy;
                f9[2] = -0.5f * f9[2];
                f9[3] = -f9[3];
                f9[4] = -0.5f * f9[4];
                const uint64_t slot = pair_slot(a, vbase + id, tx, ty);
                if (slot < a.capacity) {
                    float* dst = a.slots + slot * 9;
#pragma unroll
                    for (int f = 0; f < 9; ++f) dst[f] = f9[f];
                }
            }
        }
        hi = lo;
    }
    // pairs behind every pixel's last composited entry contribute nothing
    for (uint32_t pos = top + t; pos < end; pos += NT) {
        const uint32_t id = a.vals[pos];
        if ((int64_t)id >= a.n) continue;
        const uint64_t slot = pair_slot(a, vbase + id, tx, ty);
        if (slot < a.capacity) {
            float* dst = a.slots + slot * 9;
#pragma unroll
            for (int f = 0; f < 9; ++f) dst[f] = 0.f;
        }
    }
}

// tile of this workgroup: its own, or the entry of the longest-first list at its position
__device__ __forceinline__ int tile_of_block(const RenderArgs& a) {
    return a.queue ? (int)a.queue[blockIdx.x] : (int)blockIdx.x;
}

// single-depth batches of one pixel per lane: at most 64 VGPRs, so that eight waves fit on
// each SIMD
template <int TW, int TH, int DEPTH, int MODE, int PXW>
__global__ __launch_bounds__(TW* TH / PXW) __attribute__((amdgpu_waves_per_eu(DEPTH == 1 && PXW == 1 ? 8 : 1, 8)))
void k_render(RenderArgs a) {
    __shared__ Smem<TW, TH, DEPTH, PXW> sm;
    fwd_tile<TW, TH, DEPTH, MODE, PXW>(sm, a, tile_of_block(a));
}

// Sorting and compositing in one launch: each workgroup first sorts its tile's list (as the
// binning's sort launch would, writing the keys and values) and then composites it, reusing the
// same LDS. Tiles whose lists are sorted early start compositing while others still sort, and
// the launch between the two is gone. For the tile shapes whose workgroup has the sort's TS_T
// threads.
template <int TW, int TH, int DEPTH, int MODE, int PXW>
__global__ __launch_bounds__(TW* TH / PXW) void k_sort_render(RenderArgs a, TileSortArgs ta) {
    static_assert(TW * TH / PXW == TS_T, "one thread of the sort per compositing thread");
    __shared__ union {
        TileSortLds s;
        Smem<TW, TH, DEPTH, PXW> r;
    } u;
    const int tile = tile_of_block(a);
    if (ta.sticky && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t o = *ta.overflow;
        if (o) atomicOr(ta.sticky, o);
    }
    sort_tile(u.s, ta, tile);
    __syncthreads();  // the LDS changes hands; the tile's sorted values are read back below
    fwd_tile<TW, TH, DEPTH, MODE, PXW>(u.r, a, tile);
}

// Tile order of the reverse traversal: workgroups go to the 8 XCDs round-robin, so workgroup b
// runs on XCD b mod 8; here each XCD takes pairs of neighbouring tiles (2m, 2m + 1) in
// consecutive slots, so that the slots of a Gaussian's pairs in two neighbouring tiles (adjacent
// in emission order) are written through one L2. The last n mod 16 tiles keep their place.
__device__ __forceinline__ int bwd_tile_of_block(const RenderArgs& a) {
    if (a.queue) return (int)a.queue[blockIdx.x];
    const int b = (int)blockIdx.x, n16 = (int)gridDim.x & ~15;
    if (b >= n16) return b;
    const int x = b & 7, s = b >> 3;
    return 2 * (8 * (s >> 1) + x) + (s & 1);
}

template <int TW, int TH, int PXW, int PXH>
__global__ __launch_bounds__(TW* TH / (PXW * PXH)) void k_render_bwd(RenderArgs a) {
    __shared__ SmemBwd<TW, TH, PXW, PXH> sm;
    bwd_tile<TW, TH, PXW, PXH>(sm, a, bwd_tile_of_block(a));
}

// L1 loss and its gradient: grid-stride over the elements, one atomic per workgroup for
// the loss (the grid is bounded, so the loss word sees at most a few thousand atomics)
__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ rgb, const float* __restrict__ tgt, int64_t n,
                                            float scale, float* __restrict__ dl, float* __restrict__ loss) {
    __shared__ float part[4];
    float e = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = rgb[i] - tgt[i];
        dl[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
        e += fabsf(d);
    }
    const float s = wave_sum(e);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, scale * ((part[0] + part[1]) + (part[2] + part[3])));
}

gs_status launch_l1(const float* rgb, const float* tgt, int64_t n, float scale, float* dl, float* loss,
                    hipStream_t s) {
    if (n == 0) return GS_OK;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_l1, dim3(grid), dim3(256), 0, s, rgb, tgt, n, scale, dl, loss);
    return check_launch("l1_loss_grad");
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------
// workgroups of a persistent launch: CUs x resident workgroups of this kernel per CU. The
// device queries run on the first launch of each kernel on each device and are cached, so
// later launches (for instance inside a captured graph) make no runtime query.
int persistent_grid(const void* fn, int threads, int64_t n_tiles) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return n_tiles;
    int slots = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find({fn, dev});
        if (it != cache.end()) slots = it->second;
    }
    if (slots == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        slots = cus * per_cu;
        std::lock_guard<std::mutex> lock(mu);
        cache[{fn, dev}] = slots;
    }
    return (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, slots));
}

template <typename K>
static void launch_tiles(K kernel, const RenderArgs& a, int threads, int n_tiles, hipStream_t s) {
    hipLaunchKernelGGL(kernel, dim3(n_tiles), dim3(threads), 0, s, a);
}

// pixels per lane of the forward traversals: 1, 2 (2 x 1) where the tile is at least 16 wide, or
// 4 (4 x 1) where it is at least 32 wide
template <int MODE>
static bool launch_mode(const RenderArgs& a, int tw, int th, int depth, int px, int n_tiles, hipStream_t s) {
#define GS_CASE(W_, H_, D_, P_)                                                                  \
    if (tw == W_ && th == H_ && depth == D_ && px == P_) {                                       \
        launch_tiles(k_render<W_, H_, D_, MODE, P_>, a, W_ * H_ / P_, n_tiles, s);               \
        return true;                                                                             \
    }
    GS_CASE(8, 8, 1, 1) GS_CASE(8, 8, 2, 1)
    GS_CASE(16, 8, 1, 1) GS_CASE(16, 8, 2, 1)
    GS_CASE(8, 16, 1, 1) GS_CASE(8, 16, 2, 1)
    GS_CASE(16, 16, 1, 1) GS_CASE(16, 16, 2, 1)
    GS_CASE(32, 8, 1, 1) GS_CASE(32, 8, 2, 1)
    GS_CASE(8, 32, 1, 1) GS_CASE(8, 32, 2, 1)
    GS_CASE(32, 16, 1, 1) GS_CASE(32, 16, 2, 1)
    GS_CASE(16, 32, 1, 1) GS_CASE(16, 32, 2, 1)
    GS_CASE(32, 32, 1, 1)
    GS_CASE(16, 8, 1, 2) GS_CASE(16, 16, 1, 2) GS_CASE(32, 8, 1, 2) GS_CASE(32, 16, 1, 2) GS_CASE(16, 32, 1, 2)
    GS_CASE(32, 32, 1, 2)
    GS_CASE(16, 8, 2, 2) GS_CASE(16, 16, 2, 2) GS_CASE(32, 8, 2, 2) GS_CASE(32, 16, 2, 2) GS_CASE(16, 32, 2, 2)
    GS_CASE(32, 16, 1, 4) GS_CASE(32, 16, 2, 4) GS_CASE(32, 32, 1, 4)
#undef GS_CASE
    return false;
}

// as asked (4 is a row of four pixels where the tile is at least 32 wide, else two), else 2 for
// tiles of at least 512 pixels: at 1256 x 828 and 1M Gaussians, 16 x 32 tiles composite in
// 138 us at two pixels per lane against 150 us at one; 16 x 16 tiles gain nothing and their
// importance pass loses 8%
static int fwd_pixels_per_lane(const gs_views* v) {
    const int p = v->pixels_per_lane;
    if (p == 1 || p == 2) return p;
    if (p == 4) return v->tile_w >= 32 ? 4 : 2;
    return v->tile_w >= 16 && v->tile_w * v->tile_h >= 512 ? 2 : 1;
}

// pixels per lane of the reverse traversal: as asked, else 2 where the tile is at least 16 wide
static int bwd_pixels_per_lane(const gs_views* v) {
    if (v->pixels_per_lane) return v->pixels_per_lane;
    return v->tile_w >= 16 ? 2 : 1;
}

// pixels per lane of the reverse traversal: 1 (1 x 1), 2 (2 x 1) or 4 (2 x 2); a tile must hold
// whole wave blocks of 8 x 8 lanes
static bool launch_bwd(const RenderArgs& a, int tw, int th, int px, int n_tiles, hipStream_t s) {
#define GS_CASE(W_, H_, PW_, PH_)                                                                \
    if (tw == W_ && th == H_ && px == PW_ * PH_) {                                               \
        launch_tiles(k_render_bwd<W_, H_, PW_, PH_>, a, W_ * H_ / (PW_ * PH_), n_tiles, s);      \
        return true;                                                                             \
    }
    GS_CASE(8, 8, 1, 1) GS_CASE(16, 8, 1, 1) GS_CASE(8, 16, 1, 1) GS_CASE(16, 16, 1, 1) GS_CASE(32, 8, 1, 1)
    GS_CASE(8, 32, 1, 1) GS_CASE(32, 16, 1, 1) GS_CASE(16, 32, 1, 1) GS_CASE(32, 32, 1, 1)
    GS_CASE(16, 8, 2, 1) GS_CASE(16, 16, 2, 1) GS_CASE(32, 8, 2, 1) GS_CASE(32, 16, 2, 1) GS_CASE(16, 32, 2, 1)
    GS_CASE(32, 32, 2, 1)
    GS_CASE(16, 16, 2, 2) GS_CASE(32, 16, 2, 2) GS_CASE(16, 32, 2, 2) GS_CASE(32, 32, 2, 2)
#undef GS_CASE
    return false;
}

static RenderArgs base_args(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                            const gs_params* p) {
    RenderArgs a = {};
    a.splat = proj->splat;
    a.vals = bins->vals;
    a.ranges = bins->ranges;
    a.tile_offset = views->tile_offset;
    a.pixel_offset = views->pixel_offset;
    a.cams = views->cams;
    a.n_views = views->n_views;
    a.n = proj->n;
    a.p = *p;
    a.queue = views->lpt ? bins->queue : nullptr;
    return a;
}

static gs_status finish(bool launched, const char* what) {
    if (!launched) return set_error(GS_ERR_UNSUPPORTED, "%s: no kernel for this tile size and batch depth", what);
    return check_launch(what);
}

gs_status launch_render_fwd(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                            float* rgb, float* t_final, uint32_t* n_last, uint32_t* n_contrib, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.rgb = rgb;
    a.t_final = t_final;
    a.n_last = n_last;
    a.n_contrib = n_contrib;
    const int px = fwd_pixels_per_lane(views);
    const bool ok = n_contrib ? launch_mode<MODE_FWD_COUNT>(a, views->tile_w, views->tile_h, views->batch_depth, px,
                                                            views->n_tiles, s)
                              : launch_mode<MODE_FWD>(a, views->tile_w, views->tile_h, views->batch_depth, px,
                                                      views->n_tiles, s);
    return finish(ok, "render_fwd");
}

void launch_tile_sort(const TileSortArgs& ta, hipStream_t stream);
gs_status launch_importance(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, float*,
                            hipStream_t);
gs_status launch_visibility(const gs_projected*, const gs_views*, const gs_bins*, const gs_params*, const int32_t*,
                            int32_t, float, uint32_t*, hipStream_t);

template <int MODE>
static bool launch_sort_mode(const RenderArgs& a, const TileSortArgs& ta, int tw, int th, int depth, int px,
                             int n_tiles, hipStream_t s) {
#define GS_CASE(W_, H_, D_, P_)                                                                          \
    if (tw == W_ && th == H_ && depth == D_ && px == P_) {                                               \
        hipLaunchKernelGGL((k_sort_render<W_, H_, D_, MODE, P_>), dim3(n_tiles), dim3(W_ * H_ / P_), 0, s, a, ta); \
        return true;                                                                                     \
    }
    GS_CASE(16, 16, 1, 1) GS_CASE(16, 16, 2, 1)
    GS_CASE(32, 8, 1, 1) GS_CASE(32, 8, 2, 1)
    GS_CASE(8, 32, 1, 1) GS_CASE(8, 32, 2, 1)
    GS_CASE(32, 16, 1, 2) GS_CASE(16, 32, 1, 2) GS_CASE(32, 16, 2, 2) GS_CASE(16, 32, 2, 2)
    GS_CASE(32, 32, 1, 4)
#undef GS_CASE
    return false;
}

// compositing of lists whose per-tile sort is still to be done (ta, from the binning): in the
// compositing launch where the tile shape allows, else the sort launch and then compositing
gs_status launch_render_fwd_sorted(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                                   const gs_params* p, float* rgb, float* t_final, uint32_t* n_last,
                                   uint32_t* n_contrib, const TileSortArgs& ta, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.rgb = rgb;
    a.t_final = t_final;
    a.n_last = n_last;
    a.n_contrib = n_contrib;
    const int px = fwd_pixels_per_lane(views);
    const bool fused =
        n_contrib ? launch_sort_mode<MODE_FWD_COUNT>(a, ta, views->tile_w, views->tile_h, views->batch_depth, px,
                                                     views->n_tiles, s)
                  : launch_sort_mode<MODE_FWD>(a, ta, views->tile_w, views->tile_h, views->batch_depth, px,
                                               views->n_tiles, s);
    if (fused) return check_launch("bin_sort_render_fwd");
    launch_tile_sort(ta, s);
    return launch_render_fwd(proj, views, bins, p, rgb, t_final, n_last, n_contrib, s);
}

// the importance and cluster-visibility traversals over lists whose per-tile sort is still to
// be done (ta), as launch_render_fwd_sorted does for compositing
gs_status launch_importance_sorted(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                                   const gs_params* p, float* h, const TileSortArgs& ta, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.h = h;
    if (launch_sort_mode<MODE_IMPORTANCE>(a, ta, views->tile_w, views->tile_h, views->batch_depth,
                                          fwd_pixels_per_lane(views), views->n_tiles, s))
        return check_launch("bin_sort_importance");
    launch_tile_sort(ta, s);
    return launch_importance(proj, views, bins, p, h, s);
}

gs_status launch_visibility_sorted(const gs_projected* proj, const gs_views* views, const gs_bins* bins,
                                   const gs_params* p, const int32_t* view_cluster, int32_t k, float t_cluster,
                                   uint32_t* bits, const TileSortArgs& ta, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.bits = bits;
    a.view_cluster = view_cluster;
    a.k_clusters = k;
    a.words = (proj->n + 31) / 32;
    a.t_cluster = t_cluster;
    if (launch_sort_mode<MODE_VISIBILITY>(a, ta, views->tile_w, views->tile_h, views->batch_depth,
                                          fwd_pixels_per_lane(views), views->n_tiles, s))
        return check_launch("bin_sort_cluster_visibility");
    launch_tile_sort(ta, s);
    return launch_visibility(proj, views, bins, p, view_cluster, k, t_cluster, bits, s);
}

gs_status launch_importance(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                            float* h, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.h = h;
    return finish(
        launch_mode<MODE_IMPORTANCE>(a, views->tile_w, views->tile_h, views->batch_depth, fwd_pixels_per_lane(views),
                                     views->n_tiles, s),
        "importance");
}

gs_status launch_visibility(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                            const int32_t* view_cluster, int32_t k, float t_cluster, uint32_t* bits, hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.bits = bits;
    a.view_cluster = view_cluster;
    a.k_clusters = k;
    a.words = (proj->n + 31) / 32;
    a.t_cluster = t_cluster;
    return finish(
        launch_mode<MODE_VISIBILITY>(a, views->tile_w, views->tile_h, views->batch_depth, fwd_pixels_per_lane(views),
                                     views->n_tiles, s),
        "cluster_visibility");
}

gs_status launch_render_bwd(const gs_projected* proj, const gs_views* views, const gs_bins* bins, const gs_params* p,
                            const float* t_final, const uint32_t* n_last, const float* dl_drgb, float* slots,
                            hipStream_t s) {
    if (views->n_tiles == 0) return GS_OK;
    RenderArgs a = base_args(proj, views, bins, p);
    a.t_in = t_final;
    a.last_in = n_last;
    a.dl_drgb = dl_drgb;
    a.rect = proj->rect;
    a.entry_offset = bins->entry_offset;
    a.capacity = bins->capacity;
    a.slots = slots;
    if (!launch_bwd(a, views->tile_w, views->tile_h, bwd_pixels_per_lane(views), views->n_tiles, s))
        return finish(false, "render_bwd");
    return check_launch("render_bwd");
}

}  // namespace gs
