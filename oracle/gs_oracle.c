/*
 * FP64 CPU oracle of the Gaussian-splatting model used by RadSplat.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file; it exists so the tests and the benchmark's CPU baseline can check
 * the GPU path against a plain, slow, obviously correct definition. It shares
 * no code, header or constant with the GPU library.
 *
 * What it computes (paper Sec. 3.2, eq. render-gs; Sec. 3.3, eq. importance-score;
 * Sec. 3.4, eq. importance-score-vis), for one pinhole camera at a time:
 *   - each Gaussian's projection: camera-space mean, EWA 2D covariance
 *     Sigma' = J M Sigma M^T J^T (+ low-pass), its inverse (the conic), the
 *     support radius q_max, the footprint's bounding box and tile rectangle,
 *     the FP32 depth key and the SH colour for the view direction;
 *   - per pixel, tile-free: every Gaussian whose footprint covers the pixel
 *     centre, ordered by (FP32 depth, index), composited front to back with
 *     weights w_j = alpha_j * prod_{k<j} (1 - alpha_k); the ray ends right
 *     after the first entry that takes the transmittance below t_min (that
 *     entry is still composited, so every Gaussian that influences a pixel has
 *     a positive weight there);
 *   - the importance score h_i = max over pixels of w_ij (eq. importance-score);
 *   - the exact a.e. derivative of the image with respect to every Gaussian
 *     parameter, with every discrete decision (support, order, stop, clamps)
 *     held fixed.
 * All arithmetic is FP64. Inputs are FP32 values widened exactly to FP64 by the
 * caller.
 *
 * Camera array (20 doubles): R[9] (world->camera, row-major), t[3], fx, fy, cx,
 * cy, width, height, znear, unused.
 * Parameter array (9 doubles): lowpass, kappa, alpha_min, alpha_max, t_min,
 * guard, bg[3].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Per-Gaussian projection record: NPROJ doubles, field order below. */
enum {
    PJ_VIS = 0,   /* 1 if the Gaussian passes the culls */
    PJ_X, PJ_Y, PJ_Z,          /* camera-space mean */
    PJ_U, PJ_V,                /* projected mean in pixels */
    PJ_SXX, PJ_SXY, PJ_SYY,    /* 2D covariance incl. low-pass */
    PJ_CA, PJ_CB, PJ_CC,       /* conic = inverse 2D covariance (a, b, c) */
    PJ_QMAX,                   /* support radius in squared Mahalanobis units */
    PJ_HX, PJ_HY,              /* half extents of the support's bounding box */
    PJ_R, PJ_G, PJ_B,          /* colour after clamp */
    PJ_RAWR, PJ_RAWG, PJ_RAWB, /* colour before clamp (sum k*Y + 0.5) */
    PJ_DEPTH32,                /* camera z rounded to FP32 (the depth key) */
    PJ_TX0, PJ_TY0, PJ_TX1, PJ_TY1, /* tile rectangle, inclusive */
    PJ_COUNT,                  /* number of tiles in the rectangle */
    PJ_OPAC,                   /* opacity */
    PJ_DX, PJ_DY, PJ_DZ,       /* unit view direction (world) */
    PJ_DLEN,                   /* distance camera centre -> mean */
    NPROJ
};

/* ------------------------------------------------------------------ */
/* Real spherical harmonics, orthonormal, Condon-Shortley phase.       */
/* Y_lm(d) = N * P_l^(|m|)(d_z) * A_m(d_x, d_y), where P_l^(m) is the   */
/* m-th derivative of the Legendre polynomial P_l, A_m = Re (x+iy)^m    */
/* for m > 0, Im (x+iy)^|m| for m < 0, 1 for m = 0, and                 */
/* N = sqrt(2) K_l^|m| (-1)^m (m != 0), N = K_l^0 (m = 0),              */
/* K_l^m = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!).                         */
/* On the unit sphere (1-z^2)^(m/2) cos(m phi) = Re (x+iy)^m, so this is */
/* the associated-Legendre definition written in Cartesian form.        */
/* ------------------------------------------------------------------ */

static double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    return factorial(n) / (factorial(k) * factorial(n - k));
}

/* coefficients c[p] of t^p of the m-th derivative of P_l (p = 0..l) */
static void legendre_deriv_coeffs(int l, int m, double* c) {
    double base[8];
    for (int p = 0; p <= l; ++p) base[p] = 0.0;
    /* P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k, l) t^(l-2k) */
    for (int k = 0; 2 * k <= l; ++k)
        base[l - 2 * k] = ldexp(((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l), -l);
    for (int d = 0; d < m; ++d) {
        for (int p = 0; p < l; ++p) base[p] = base[p + 1] * (double)(p + 1);
        base[l] = 0.0;
    }
    for (int p = 0; p <= l; ++p) c[p] = base[p];
}

static double poly_eval(const double* c, int deg, double t) {
    double s = 0.0;
    for (int p = deg; p >= 0; --p) s = s * t + c[p];
    return s;
}

/* Re and Im of (x + i y)^m */
static void cpow_xy(double x, double y, int m, double* re, double* im) {
    double a = 1.0, b = 0.0;
    for (int k = 0; k < m; ++k) {
        double na = a * x - b * y;
        double nb = a * y + b * x;
        a = na;
        b = nb;
    }
    *re = a;
    *im = b;
}

static double sh_norm(int l, int m) {
    int am = m < 0 ? -m : m;
    double k = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
    if (m == 0) return k;
    return sqrt(2.0) * k * ((am & 1) ? -1.0 : 1.0);
}

/* Y[idx] for idx = l*l + l + m, and optionally its gradient (as a function on R^3
 * extended off the sphere by the same formula) in grad[3*idx..]. */
static void sh_eval(int degree, const double d[3], double* Y, double* grad) {
    for (int l = 0; l <= degree; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            int idx = l * l + l + m;
            double c[8], cd[8];
            legendre_deriv_coeffs(l, am, c);
            legendre_deriv_coeffs(l, am + 1, cd);
            double pz = poly_eval(c, l, d[2]);
            double dpz = poly_eval(cd, l, d[2]);
            double re, im, re1 = 0.0, im1 = 0.0;
            cpow_xy(d[0], d[1], am, &re, &im);
            if (am > 0) cpow_xy(d[0], d[1], am - 1, &re1, &im1);
            double A, dAx, dAy;
            if (m > 0) {        /* Re (x+iy)^m: d/dx = m Re(.)^(m-1), d/dy = -m Im(.)^(m-1) */
                A = re; dAx = am * re1; dAy = -am * im1;
            } else if (m < 0) { /* Im (x+iy)^m: d/dx = m Im(.)^(m-1), d/dy = m Re(.)^(m-1) */
                A = im; dAx = am * im1; dAy = am * re1;
            } else {
                A = 1.0; dAx = 0.0; dAy = 0.0;
            }
            double nrm = sh_norm(l, m);
            Y[idx] = nrm * pz * A;
            if (grad) {
                grad[3 * idx + 0] = nrm * pz * dAx;
                grad[3 * idx + 1] = nrm * pz * dAy;
                grad[3 * idx + 2] = nrm * dpz * A;
            }
        }
    }
}

/* Exposed for the basis checks. */
void or_sh_basis(int degree, const double* dirs, int64_t m, double* out) {
    int nb = (degree + 1) * (degree + 1);
    for (int64_t j = 0; j < m; ++j) sh_eval(degree, dirs + 3 * j, out + nb * j, NULL);
}

void or_sh_basis_grad(int degree, const double* dirs, int64_t m, double* out) {
    int nb = (degree + 1) * (degree + 1);
    double Y[16];
    for (int64_t j = 0; j < m; ++j) sh_eval(degree, dirs + 3 * j, Y, out + 3 * nb * j);
}

/* ------------------------------------------------------------------ */
/* Projection (Sec. 3.2: Sigma = R S S^T R^T, Sigma' = J M Sigma M^T J^T)*/
/* Evaluation order of every key-determining quantity (z, u, v, the    */
/* diagonal of Sigma', q_max, half extents) is spelled out operation by */
/* operation so that it is reproducible.                                */
/* ------------------------------------------------------------------ */

static void quat_to_rot(double w, double x, double y, double z, double R[3][3]) {
    R[0][0] = 1.0 - 2.0 * ((y * y) + (z * z));
    R[0][1] = 2.0 * ((x * y) - (w * z));
    R[0][2] = 2.0 * ((x * z) + (w * y));
    R[1][0] = 2.0 * ((x * y) + (w * z));
    R[1][1] = 1.0 - 2.0 * ((x * x) + (z * z));
    R[1][2] = 2.0 * ((y * z) - (w * x));
    R[2][0] = 2.0 * ((x * z) - (w * y));
    R[2][1] = 2.0 * ((y * z) + (w * x));
    R[2][2] = 1.0 - 2.0 * ((x * x) + (y * y));
}

void or_project(const double* mean, const double* scale, const double* quat, const double* opac, const double* sh,
                int64_t n, int sh_degree, const double* cam, const double* prm, int tile_w, int tile_h,
                double* out) {
    const double* R = cam;
    const double* t = cam + 9;
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    double W = cam[16], H = cam[17], znear = cam[18];
    double lowpass = prm[0], kappa = prm[1], amin = prm[2], guard = prm[5];
    int tiles_x = ((int)W + tile_w - 1) / tile_w;
    int tiles_y = ((int)H + tile_h - 1) / tile_h;
    int nb = (sh_degree + 1) * (sh_degree + 1);
    /* camera centre C = -R^T t */
    double C[3];
    for (int k = 0; k < 3; ++k) C[k] = -(((R[0 * 3 + k] * t[0]) + (R[1 * 3 + k] * t[1])) + (R[2 * 3 + k] * t[2]));

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* o = out + NPROJ * i;
        for (int f = 0; f < NPROJ; ++f) o[f] = 0.0;
        double p[3] = {mean[i], mean[n + i], mean[2 * n + i]};
        double s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
        double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
        double op = opac[i];
        int finite = 1;
        for (int k = 0; k < 3; ++k) finite &= isfinite(p[k]) && isfinite(s[k]);
        for (int k = 0; k < 4; ++k) finite &= isfinite(q[k]);
        finite &= isfinite(op);
        if (!finite) continue;
        double x = (((R[0] * p[0]) + (R[1] * p[1])) + (R[2] * p[2])) + t[0];
        double y = (((R[3] * p[0]) + (R[4] * p[1])) + (R[5] * p[2])) + t[1];
        double z = (((R[6] * p[0]) + (R[7] * p[1])) + (R[8] * p[2])) + t[2];
        if (!(z > znear)) continue;
        if (!(op >= amin)) continue;
        double u = ((fx * x) / z) + cx;
        double v = ((fy * y) / z) + cy;
        double hw = 0.5 * W, hh = 0.5 * H;
        if (!(fabs(u - hw) <= guard * hw)) continue;
        if (!(fabs(v - hh) <= guard * hh)) continue;
        double qn = sqrt((((q[0] * q[0]) + (q[1] * q[1])) + (q[2] * q[2])) + (q[3] * q[3]));
        if (!(qn > 0.0)) continue;
        double Rq[3][3];
        quat_to_rot(q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn, Rq);
        double s2[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
        double Sg[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Sg[a][b] = (((Rq[a][0] * s2[0]) * Rq[b][0]) + ((Rq[a][1] * s2[1]) * Rq[b][1])) +
                           ((Rq[a][2] * s2[2]) * Rq[b][2]);
        /* J: Jacobian of the perspective projection at the camera-space mean */
        double J00 = fx / z, J02 = -((fx * x) / (z * z));
        double J11 = fy / z, J12 = -((fy * y) / (z * z));
        double T[2][3];
        for (int k = 0; k < 3; ++k) {
            T[0][k] = (J00 * R[0 * 3 + k]) + (J02 * R[2 * 3 + k]);
            T[1][k] = (J11 * R[1 * 3 + k]) + (J12 * R[2 * 3 + k]);
        }
        double Mx[2][3];
        for (int a = 0; a < 2; ++a)
            for (int l = 0; l < 3; ++l)
                Mx[a][l] = ((T[a][0] * Sg[0][l]) + (T[a][1] * Sg[1][l])) + (T[a][2] * Sg[2][l]);
        double Sp[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) Sp[a][b] = ((Mx[a][0] * T[b][0]) + (Mx[a][1] * T[b][1])) + (Mx[a][2] * T[b][2]);
        double sxx = Sp[0][0] + lowpass, syy = Sp[1][1] + lowpass, sxy = Sp[0][1];
        double det = (sxx * syy) - (sxy * sxy);
        if (!(det > 0.0)) continue;
        double qmax = kappa * kappa;
        double ql = 2.0 * log(op / amin);
        if (ql < qmax) qmax = ql;
        double hx = sqrt(qmax * sxx), hy = sqrt(qmax * syy);
        /* tile rectangle of the support's bounding box, widened by 2^-16 px */
        const double eps = 1.0 / 65536.0;
        double fx0 = floor(((u - hx) - eps) / (double)tile_w);
        double fx1 = floor(((u + hx) + eps) / (double)tile_w);
        double fy0 = floor(((v - hy) - eps) / (double)tile_h);
        double fy1 = floor(((v + hy) + eps) / (double)tile_h);
        if (fx0 < 0.0) fx0 = 0.0;
        if (fy0 < 0.0) fy0 = 0.0;
        if (fx1 > (double)(tiles_x - 1)) fx1 = (double)(tiles_x - 1);
        if (fy1 > (double)(tiles_y - 1)) fy1 = (double)(tiles_y - 1);
        double count = 0.0;
        if (fx1 >= fx0 && fy1 >= fy0) count = (fx1 - fx0 + 1.0) * (fy1 - fy0 + 1.0);
        /* colour: SH evaluated at the unit direction from the camera centre to the mean */
        double dv[3] = {p[0] - C[0], p[1] - C[1], p[2] - C[2]};
        double dl = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        double d[3] = {dv[0] / dl, dv[1] / dl, dv[2] / dl};
        double Y[16];
        sh_eval(sh_degree, d, Y, NULL);
        double raw[3];
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < nb; ++k) acc += sh[(int64_t)(k * 3 + c) * n + i] * Y[k];
            raw[c] = acc + 0.5;
        }
        o[PJ_VIS] = 1.0;
        o[PJ_X] = x; o[PJ_Y] = y; o[PJ_Z] = z;
        o[PJ_U] = u; o[PJ_V] = v;
        o[PJ_SXX] = sxx; o[PJ_SXY] = sxy; o[PJ_SYY] = syy;
        o[PJ_CA] = syy / det; o[PJ_CB] = -sxy / det; o[PJ_CC] = sxx / det;
        o[PJ_QMAX] = qmax; o[PJ_HX] = hx; o[PJ_HY] = hy;
        for (int c = 0; c < 3; ++c) {
            o[PJ_RAWR + c] = raw[c];
            o[PJ_R + c] = raw[c] > 0.0 ? raw[c] : 0.0;
        }
        o[PJ_DEPTH32] = (double)(float)z;
        o[PJ_TX0] = fx0; o[PJ_TY0] = fy0; o[PJ_TX1] = fx1; o[PJ_TY1] = fy1;
        o[PJ_COUNT] = count;
        o[PJ_OPAC] = op;
        o[PJ_DX] = d[0]; o[PJ_DY] = d[1]; o[PJ_DZ] = d[2];
        o[PJ_DLEN] = dl;
    }
}

/* ------------------------------------------------------------------ */
/* Per-pixel compositing (eq. render-gs)                               */
/* ------------------------------------------------------------------ */

typedef struct {
    float depth;
    int64_t idx;
    double qd;
} entry;

static int entry_cmp(const void* a, const void* b) {
    const entry* x = (const entry*)a;
    const entry* y = (const entry*)b;
    if (x->depth < y->depth) return -1;
    if (x->depth > y->depth) return 1;
    if (x->idx < y->idx) return -1;
    if (x->idx > y->idx) return 1;
    return 0;
}

/* support set of pixel (px,py), sorted by (depth32, index); returns its size */
static int64_t pixel_support(const double* proj, int64_t n, int px, int py, double qmax_scale, entry* list) {
    double xc = (double)px + 0.5, yc = (double)py + 0.5;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double* o = proj + NPROJ * i;
        if (o[PJ_VIS] == 0.0) continue;
        double dx = xc - o[PJ_U], dy = yc - o[PJ_V];
        double qd = o[PJ_CA] * dx * dx + 2.0 * o[PJ_CB] * dx * dy + o[PJ_CC] * dy * dy;
        if (qd <= o[PJ_QMAX] * qmax_scale) {
            list[m].depth = (float)o[PJ_DEPTH32];
            list[m].idx = i;
            list[m].qd = qd;
            ++m;
        }
    }
    qsort(list, (size_t)m, sizeof(entry), entry_cmp);
    return m;
}

/*
 * Render m pixels (px[j], py[j]) of one view from a projection table.
 * Outputs: rgb[3*j+c], T_final[j], n_comp[j] (number of composited entries),
 * optional fingerprint[j] (hash of the composited list and clamp states, used to
 * detect discrete-decision changes), optional h[n] (max-accumulated weights).
 * qmax_scale and tmin_scale move the support and stop thresholds (1.0 nominal).
 */
void or_render(const double* proj, int64_t n, const double* prm, const int32_t* px, const int32_t* py, int64_t m,
               double qmax_scale, double tmin_scale, double* rgb, double* T_final, int32_t* n_comp,
               int64_t* fingerprint, double* h) {
    double amax = prm[3], tmin = prm[4] * tmin_scale;
    const double* bg = prm + 6;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double* hloc = NULL;
    if (h) hloc = (double*)calloc((size_t)nthreads * (size_t)n, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        entry* list = (entry*)malloc(sizeof(entry) * (size_t)(n > 0 ? n : 1));
        double* hl = h ? hloc + (size_t)tid * (size_t)n : NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < m; ++j) {
            int64_t cnt = pixel_support(proj, n, px[j], py[j], qmax_scale, list);
            double T = 1.0, C[3] = {0.0, 0.0, 0.0};
            int32_t nc = 0;
            uint64_t fp = 1469598103934665603ULL;
            for (int64_t k = 0; k < cnt; ++k) {
                const double* o = proj + NPROJ * list[k].idx;
                double a = o[PJ_OPAC] * exp(-0.5 * list[k].qd);
                int clamped = 0;
                if (a >= amax) { a = amax; clamped = 1; }
                double w = a * T;
                for (int c = 0; c < 3; ++c) C[c] += w * o[PJ_R + c];
                if (hl && w > hl[list[k].idx]) hl[list[k].idx] = w;
                fp = (fp ^ (uint64_t)(list[k].idx * 8 + clamped * 4 + (o[PJ_RAWR] > 0.0) * 2 + (o[PJ_RAWG] > 0.0))) *
                     1099511628211ULL;
                fp = (fp ^ (uint64_t)(o[PJ_RAWB] > 0.0)) * 1099511628211ULL;
                T = T * (1.0 - a);
                ++nc;
                if (T < tmin) break; /* this entry was composited; the ray ends here */
            }
            for (int c = 0; c < 3; ++c) rgb[3 * j + c] = C[c] + T * bg[c];
            T_final[j] = T;
            n_comp[j] = nc;
            if (fingerprint) fingerprint[j] = (int64_t)(fp >> 1);
        }
        free(list);
    }
    if (h) {
        for (int tt = 0; tt < nthreads; ++tt)
            for (int64_t i = 0; i < n; ++i)
                if (hloc[(size_t)tt * (size_t)n + i] > h[i]) h[i] = hloc[(size_t)tt * (size_t)n + i];
        free(hloc);
    }
}

/* ------------------------------------------------------------------ */
/* Backward: exact derivative with every discrete decision held fixed. */
/* ------------------------------------------------------------------ */

enum { G2_U = 0, G2_V, G2_A, G2_B, G2_C, G2_O, G2_R, G2_G, G2_BL, NG2 };

/*
 * Accumulate dL/d(2D quantities) of one view: for m pixels with upstream
 * gradients dl_drgb[3*j+c], add into g2[NG2*i + f] for each Gaussian i.
 * The suffix sums S_j = sum_{k>j} w_k c_k + T_final bg are formed directly from
 * the composited list (no division).
 */
void or_render_bwd_2d(const double* proj, int64_t n, const double* prm, const int32_t* px, const int32_t* py,
                      int64_t m, const double* dl_drgb, double* g2) {
    double amax = prm[3], tmin = prm[4];
    const double* bg = prm + 6;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double* gl = (double*)calloc((size_t)nthreads * (size_t)n * NG2, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        entry* list = (entry*)malloc(sizeof(entry) * (size_t)(n > 0 ? n : 1));
        double* al = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* Tl = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        int* cl = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
        double* g = gl + (size_t)tid * (size_t)n * NG2;
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < m; ++j) {
            const double* dC = dl_drgb + 3 * j;
            if (dC[0] == 0.0 && dC[1] == 0.0 && dC[2] == 0.0) continue;
            int64_t cnt = pixel_support(proj, n, px[j], py[j], 1.0, list);
            double T = 1.0;
            int64_t nc = 0;
            for (int64_t k = 0; k < cnt; ++k) {
                const double* o = proj + NPROJ * list[k].idx;
                double a = o[PJ_OPAC] * exp(-0.5 * list[k].qd);
                int clamped = 0;
                if (a >= amax) { a = amax; clamped = 1; }
                al[k] = a;
                Tl[k] = T;
                cl[k] = clamped;
                T = T * (1.0 - a);
                ++nc;
                if (T < tmin) break;
            }
            /* suffix sums, from the back */
            double S[3] = {T * bg[0], T * bg[1], T * bg[2]};
            for (int64_t k = nc - 1; k >= 0; --k) {
                int64_t i = list[k].idx;
                const double* o = proj + NPROJ * i;
                double a = al[k], Tk = Tl[k];
                double* gi = g + NG2 * i;
                /* dL/dcolour_k = dC * w_k */
                for (int c = 0; c < 3; ++c) gi[G2_R + c] += dC[c] * a * Tk;
                /* dL/dalpha_k = sum_c dC_c (T_k c_k - S_c / (1 - alpha_k)) */
                double dA = 0.0;
                for (int c = 0; c < 3; ++c) dA += dC[c] * (Tk * o[PJ_R + c] - S[c] / (1.0 - a));
                for (int c = 0; c < 3; ++c) S[c] += a * Tk * o[PJ_R + c];
                if (cl[k]) continue;
                double G = exp(-0.5 * list[k].qd);
                gi[G2_O] += dA * G;
                double dq = dA * (-0.5 * a); /* d alpha / d qd = -alpha/2 */
                double dx = ((double)px[j] + 0.5) - o[PJ_U], dy = ((double)py[j] + 0.5) - o[PJ_V];
                gi[G2_A] += dq * dx * dx;
                gi[G2_B] += dq * 2.0 * dx * dy;
                gi[G2_C] += dq * dy * dy;
                /* qd = a dx^2 + 2 b dx dy + c dy^2, dx = xc - u */
                gi[G2_U] += dq * (-2.0) * (o[PJ_CA] * dx + o[PJ_CB] * dy);
                gi[G2_V] += dq * (-2.0) * (o[PJ_CB] * dx + o[PJ_CC] * dy);
            }
        }
        free(list);
        free(al);
        free(Tl);
        free(cl);
    }
    for (int tt = 0; tt < nthreads; ++tt)
        for (int64_t q = 0; q < n * NG2; ++q) g2[q] += gl[(size_t)tt * (size_t)n * NG2 + q];
    free(gl);
}

/*
 * Chain the 2D gradients of one view to the Gaussian parameters and add them
 * into dmean[3][n], dscale[3][n], dquat[4][n], dopac[n], dsh[rows][n].
 */
void or_project_bwd(const double* mean, const double* scale, const double* quat, const double* sh, int64_t n,
                    int sh_degree, const double* cam, const double* proj, const double* g2, double* dmean,
                    double* dscale, double* dquat, double* dopac, double* dsh) {
    (void)mean; /* the camera-space mean is taken from the projection table */
    const double* R = cam;
    double fx = cam[12], fy = cam[13];
    int nb = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* o = proj + NPROJ * i;
        const double* gi = g2 + NG2 * i;
        if (o[PJ_VIS] == 0.0) continue;
        double x = o[PJ_X], y = o[PJ_Y], z = o[PJ_Z];
        double s[3] = {scale[i], scale[n + i], scale[2 * n + i]};
        double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
        double Rq[3][3];
        quat_to_rot(qh[0], qh[1], qh[2], qh[3], Rq);
        /* M = Rq diag(s), Sigma = M M^T */
        double Mm[3][3], Sg[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Mm[a][b] = Rq[a][b] * s[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += Mm[a][k] * Mm[b][k];
                Sg[a][b] = acc;
            }
        double J00 = fx / z, J02 = -fx * x / (z * z), J11 = fy / z, J12 = -fy * y / (z * z);
        double Jm[2][3] = {{J00, 0.0, J02}, {0.0, J11, J12}};
        double T[2][3];
        for (int a = 0; a < 2; ++a)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int l = 0; l < 3; ++l) acc += Jm[a][l] * R[l * 3 + k];
                T[a][k] = acc;
            }
        /* conic Q and its gradient as a symmetric matrix */
        double Q[2][2] = {{o[PJ_CA], o[PJ_CB]}, {o[PJ_CB], o[PJ_CC]}};
        double GQ[2][2] = {{gi[G2_A], 0.5 * gi[G2_B]}, {0.5 * gi[G2_B], gi[G2_C]}};
        /* dL/dSigma' = -Q GQ Q */
        double QG[2][2], GS2[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) QG[a][b] = Q[a][0] * GQ[0][b] + Q[a][1] * GQ[1][b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) GS2[a][b] = -(QG[a][0] * Q[0][b] + QG[a][1] * Q[1][b]);
        /* Sigma' = T Sigma T^T: dL/dSigma = T^T GS2 T, dL/dT = 2 GS2 T Sigma */
        double GS3[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int d2 = 0; d2 < 2; ++d2) acc += T[c][a] * GS2[c][d2] * T[d2][b];
                GS3[a][b] = acc;
            }
        double GT[2][3];
        for (int a = 0; a < 2; ++a)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int l = 0; l < 3; ++l) acc += 2.0 * GS2[a][c] * T[c][l] * Sg[l][k];
                GT[a][k] = acc;
            }
        /* T = J R: dL/dJ = GT R^T */
        double GJ[2][3];
        for (int a = 0; a < 2; ++a)
            for (int l = 0; l < 3; ++l) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += GT[a][k] * R[l * 3 + k];
                GJ[a][l] = acc;
            }
        /* camera-space mean gradient from J and from (u, v) */
        double gpc[3] = {0.0, 0.0, 0.0};
        double z2 = z * z, z3 = z2 * z;
        gpc[2] += GJ[0][0] * (-fx / z2);
        gpc[0] += GJ[0][2] * (-fx / z2);
        gpc[2] += GJ[0][2] * (2.0 * fx * x / z3);
        gpc[2] += GJ[1][1] * (-fy / z2);
        gpc[1] += GJ[1][2] * (-fy / z2);
        gpc[2] += GJ[1][2] * (2.0 * fy * y / z3);
        gpc[0] += gi[G2_U] * (fx / z);
        gpc[2] += gi[G2_U] * (-fx * x / z2);
        gpc[1] += gi[G2_V] * (fy / z);
        gpc[2] += gi[G2_V] * (-fy * y / z2);
        /* world mean: p_c = R p + t */
        double gp[3];
        for (int k = 0; k < 3; ++k) gp[k] = R[0 * 3 + k] * gpc[0] + R[1 * 3 + k] * gpc[1] + R[2 * 3 + k] * gpc[2];
        /* Sigma = M M^T: dL/dM = 2 GS3 M */
        double GM[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += 2.0 * GS3[a][k] * Mm[k][b];
                GM[a][b] = acc;
            }
        double gs[3] = {0.0, 0.0, 0.0}, GR[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                gs[b] += GM[a][b] * Rq[a][b];
                GR[a][b] = GM[a][b] * s[b];
            }
        /* rotation matrix entries as functions of the unit quaternion (w,x,y,z) */
        double w = qh[0], qx = qh[1], qy = qh[2], qz = qh[3];
        double gqh[4] = {0.0, 0.0, 0.0, 0.0};
        /* R00 = 1 - 2(y^2+z^2) */
        gqh[2] += GR[0][0] * (-4.0 * qy); gqh[3] += GR[0][0] * (-4.0 * qz);
        /* R01 = 2(xy - wz) */
        gqh[1] += GR[0][1] * 2.0 * qy; gqh[2] += GR[0][1] * 2.0 * qx; gqh[0] += GR[0][1] * (-2.0 * qz); gqh[3] += GR[0][1] * (-2.0 * w);
        /* R02 = 2(xz + wy) */
        gqh[1] += GR[0][2] * 2.0 * qz; gqh[3] += GR[0][2] * 2.0 * qx; gqh[0] += GR[0][2] * 2.0 * qy; gqh[2] += GR[0][2] * 2.0 * w;
        /* R10 = 2(xy + wz) */
        gqh[1] += GR[1][0] * 2.0 * qy; gqh[2] += GR[1][0] * 2.0 * qx; gqh[0] += GR[1][0] * 2.0 * qz; gqh[3] += GR[1][0] * 2.0 * w;
        /* R11 = 1 - 2(x^2+z^2) */
        gqh[1] += GR[1][1] * (-4.0 * qx); gqh[3] += GR[1][1] * (-4.0 * qz);
        /* R12 = 2(yz - wx) */
        gqh[2] += GR[1][2] * 2.0 * qz; gqh[3] += GR[1][2] * 2.0 * qy; gqh[0] += GR[1][2] * (-2.0 * qx); gqh[1] += GR[1][2] * (-2.0 * w);
        /* R20 = 2(xz - wy) */
        gqh[1] += GR[2][0] * 2.0 * qz; gqh[3] += GR[2][0] * 2.0 * qx; gqh[0] += GR[2][0] * (-2.0 * qy); gqh[2] += GR[2][0] * (-2.0 * w);
        /* R21 = 2(yz + wx) */
        gqh[2] += GR[2][1] * 2.0 * qz; gqh[3] += GR[2][1] * 2.0 * qy; gqh[0] += GR[2][1] * 2.0 * qx; gqh[1] += GR[2][1] * 2.0 * w;
        /* R22 = 1 - 2(x^2+y^2) */
        gqh[1] += GR[2][2] * (-4.0 * qx); gqh[2] += GR[2][2] * (-4.0 * qy);
        /* normalisation qh = q/|q|: dL/dq = (g - qh (qh . g)) / |q| */
        double dotg = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
        double gq[4];
        for (int k = 0; k < 4; ++k) gq[k] = (gqh[k] - qh[k] * dotg) / qn;
        /* colour: c = max(0, sum k Y(d) + 0.5), d = (p - C)/|p - C| */
        double d[3] = {o[PJ_DX], o[PJ_DY], o[PJ_DZ]};
        double Y[16], dY[48];
        sh_eval(sh_degree, d, Y, dY);
        double gd[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            if (!(o[PJ_RAWR + c] > 0.0)) continue;
            double gc = gi[G2_R + c];
            for (int k = 0; k < nb; ++k) {
                dsh[(int64_t)(k * 3 + c) * n + i] += gc * Y[k];
                double kc = sh[(int64_t)(k * 3 + c) * n + i];
                for (int e = 0; e < 3; ++e) gd[e] += gc * kc * dY[3 * k + e];
            }
        }
        double dotd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
        for (int e = 0; e < 3; ++e) gp[e] += (gd[e] - d[e] * dotd) / o[PJ_DLEN];
        for (int k = 0; k < 3; ++k) {
            dmean[(int64_t)k * n + i] += gp[k];
            dscale[(int64_t)k * n + i] += gs[k];
        }
        for (int k = 0; k < 4; ++k) dquat[(int64_t)k * n + i] += gq[k];
        dopac[i] += gi[G2_O];
    }
}

int or_nproj(void) { return NPROJ; }
int or_ng2(void) { return NG2; }
