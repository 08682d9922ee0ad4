/* CPU oracle of the tracking correspondence search.  TEST INFRASTRUCTURE ONLY:
 * see ft_oracle.h for scope, conventions and what it shares (nothing) with the
 * device path.  Build: gcc -O2 -ffp-contract=off -fno-fast-math. */
#include "ft_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Hamming distance of two 256-bit ORB descriptors (Section II-A: each keypoint
 * is described by a binary descriptor; similarity is the number of differing
 * bits).  Pinned in tests by the +-1 dot-product identity and numpy unpackbits. */
int oracle_hamming(const uint8_t *a, const uint8_t *b)
{
    int h = 0;
    for (int q = 0; q < 32; ++q)
        h += __builtin_popcount((unsigned)(a[q] ^ b[q]));
    return h;
}

/* Resolve two queries that claimed one target: the claim with the smaller
 * (distance, query index) keeps it, the others become unmatched.  The paper
 * treats every query as independent (Section IV-C, IV-E), so this rule is the
 * reading that makes the result unique without ordering between queries. */
static void resolve_conflicts(int nQ, const int32_t *target, const int32_t *dist,
                              int nT, uint8_t *alive)
{
    int64_t *best = (int64_t *)malloc(sizeof(int64_t) * (nT > 0 ? nT : 1));
    for (int j = 0; j < nT; ++j) best[j] = INT64_MAX;
    for (int i = 0; i < nQ; ++i) {
        if (!alive[i]) continue;
        int64_t key = ((int64_t)dist[i] << 32) | (int64_t)i;
        if (key < best[target[i]]) best[target[i]] = key;
    }
    for (int i = 0; i < nQ; ++i) {
        if (!alive[i]) continue;
        int64_t key = ((int64_t)dist[i] << 32) | (int64_t)i;
        if (best[target[i]] != key) alive[i] = 0;
    }
    free(best);
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Centre-subtracted sum of absolute differences between the (2w+1)^2 patch of
 * the left level image centred at (su, sv) and the right patches centred at
 * (su0 + k, sv) for k = -L..L (rectified images: same row).  Returns 0 and
 * leaves sad untouched when any accessed pixel lies outside the level image.
 * Pinned by a numpy brute force and by exact integer shifts. */
int oracle_sad_window(const uint8_t *IL, const uint8_t *IR, int Wl, int Hl,
                      int su, int sv, int su0, int w, int L, int *sad)
{
    if (su - w < 0 || su + w >= Wl || sv - w < 0 || sv + w >= Hl ||
        su0 - L - w < 0 || su0 + L + w >= Wl)
        return 0;
    const int cL = IL[(size_t)sv * Wl + su];
    for (int k = -L; k <= L; ++k) {
        const int cR = IR[(size_t)sv * Wl + su0 + k];
        int acc = 0;
        for (int dy = -w; dy <= w; ++dy)
            for (int dx = -w; dx <= w; ++dx) {
                const int a = (int)IL[(size_t)(sv + dy) * Wl + su + dx] - cL;
                const int c = (int)IR[(size_t)(sv + dy) * Wl + su0 + k + dx] - cR;
                acc += abs(a - c);
            }
        sad[k + L] = acc;
    }
    return 1;
}

/* Best shift (smallest SAD, ties to the smaller shift) and the vertex offset
 * of the parabola through the three SAD values around it.  Returns 0 when the
 * best shift sits on the border of the range or the offset exceeds one pixel.
 * Pinned by closed forms (the vertex of an exact parabola, |delta| <= 1/2). */
int oracle_subpixel(const int *sad, int L, int *kbest, int *sad_best, float *delta)
{
    int kb = -L, best = sad[0];
    for (int k = -L + 1; k <= L; ++k)
        if (sad[k + L] < best) { best = sad[k + L]; kb = k; }
    if (kb == -L || kb == L) return 0;
    const int a = sad[kb + L - 1], c = sad[kb + L], e = sad[kb + L + 1];
    const float num = (float)(a - e);
    const float den = (float)(2 * (a + e - 2 * c));
    const float d = num / den;
    if (d < -1.0f || d > 1.0f) return 0;
    *kbest = kb; *sad_best = c; *delta = d;
    return 1;
}

/* Outlier rejection after stereo refinement: m = the SAD at position n/2 of the
 * ascending order; keep[i] = (den * sad[i] < num * m).  Returns m, or -1 when
 * n = 0.  Pinned by hand-built lists (n = 0, 1, m = 0, ties). */
int oracle_median_keep(int n, const int32_t *sad, int num, int den, uint8_t *keep)
{
    if (n <= 0) return -1;
    int *v = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) v[i] = sad[i];
    qsort(v, n, sizeof(int), cmp_int);
    const int m = v[n / 2];
    free(v);
    for (int i = 0; i < n; ++i) keep[i] = (int64_t)den * sad[i] < (int64_t)num * m;
    return m;
}

/* Predicted pyramid level of a map point seen at distance dist: the smallest
 * level whose scale reaches dmax/dist (the level where it would have been
 * observed at its creation distance), capped at the top level.  Pinned against
 * ceil(log(ratio)/log(scale factor)). */
int oracle_predict_level(float ratio, const float *sf, int n_levels)
{
    for (int l = 0; l < n_levels; ++l)
        if (sf[l] >= ratio) return l;
    return n_levels - 1;
}

/* ------------------------------------------------------------------------ */
/* Rectified pinhole stereo (Section II-B, IV-C): the right match of a left  */
/* keypoint lies on its epipolar line, so only right keypoints whose row    */
/* band contains the left row are searched; the best one is then refined   */
/* among nearby pixels.                                                     */
/* ------------------------------------------------------------------------ */
void oracle_stereo_pinhole(
    int nL, const float *xL, const float *yL, const uint8_t *oL, const uint8_t *dL,
    int nR, const float *xR, const float *yR, const uint8_t *oR, const uint8_t *dR,
    const uint8_t *pyrL, const uint8_t *pyrR, const int64_t *lv_off,
    const int32_t *lv_w, const int32_t *lv_h, const float *sf, const float *inv_sf,
    float bf, float b, int rows, const int32_t *ip, float band,
    int32_t *out_j, int32_t *out_h, float *out_ur, float *out_depth, int32_t *out_sad,
    int64_t *stats)
{
    const int th_orb = ip[0], w = ip[1], L = ip[2], lw = ip[3];
    const int med_num = ip[4], med_den = ip[5];
    const float minD = 0.0f;
    const float maxD = bf / b;
    int64_t n_ham = 0, n_ref = 0, n_ref_ok = 0;

    int32_t *cj = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    int32_t *ch = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    int32_t *cs = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    float *cu = (float *)malloc(sizeof(float) * (nL > 0 ? nL : 1));
    float *cd = (float *)malloc(sizeof(float) * (nL > 0 ? nL : 1));
    uint8_t *alive = (uint8_t *)calloc(nL > 0 ? nL : 1, 1);
    int *sadv = (int *)malloc(sizeof(int) * (2 * L + 1));

    for (int i = 0; i < nL; ++i) {
        out_j[i] = -1; out_h[i] = -1; out_ur[i] = -1.0f; out_depth[i] = -1.0f; out_sad[i] = -1;
        const int row = (int)yL[i];
        const float minU = xL[i] - maxD;
        const float maxU = xL[i] - minD;
        if (maxU < 0.0f) continue;
        const int oi = oL[i];
        int best_h = 1000, best_j = -1;
        for (int j = 0; j < nR; ++j) {
            const float r = band * sf[oR[j]];
            int lo = (int)floorf(yR[j] - r);
            int hi = (int)ceilf(yR[j] + r);
            if (lo < 0) lo = 0;
            if (hi > rows - 1) hi = rows - 1;
            if (row < lo || row > hi) continue;
            const int oj = oR[j];
            if (oj < oi - lw || oj > oi + lw) continue;
            if (!(xR[j] >= minU && xR[j] <= maxU)) continue;
            const int h = oracle_hamming(dL + 32 * (size_t)i, dR + 32 * (size_t)j);
            ++n_ham;
            if (h < best_h) { best_h = h; best_j = j; }
        }
        if (best_j < 0 || !(best_h < th_orb)) continue;

        /* refinement: sliding-window SAD at the left keypoint's pyramid level */
        ++n_ref;
        const int l = oi;
        const float s = inv_sf[l];
        const int su = (int)roundf(xL[i] * s);
        const int sv = (int)roundf(yL[i] * s);
        const int su0 = (int)roundf(xR[best_j] * s);
        if (!oracle_sad_window(pyrL + lv_off[l], pyrR + lv_off[l], lv_w[l], lv_h[l],
                               su, sv, su0, w, L, sadv))
            continue;
        int kb, c;
        float delta;
        if (!oracle_subpixel(sadv, L, &kb, &c, &delta)) continue;
        float uR = sf[l] * (((float)su0 + (float)kb) + delta);
        float disp = xL[i] - uR;
        if (!(disp >= minD && disp < maxD)) continue;
        if (disp <= 0.0f) {
            disp = 0.01f;
            uR = (float)((double)xL[i] - 0.01);
        }
        ++n_ref_ok;
        cj[i] = best_j; ch[i] = best_h; cs[i] = c; cu[i] = uR; cd[i] = bf / disp;
        alive[i] = 1;
    }

    resolve_conflicts(nL, cj, ch, nR, alive);
    int n_alive = 0;
    for (int i = 0; i < nL; ++i) n_alive += alive[i];
    int32_t *sv_alive = (int32_t *)malloc(sizeof(int32_t) * (n_alive > 0 ? n_alive : 1));
    uint8_t *keep = (uint8_t *)malloc(n_alive > 0 ? n_alive : 1);
    int q = 0;
    for (int i = 0; i < nL; ++i) if (alive[i]) sv_alive[q++] = cs[i];
    const int median = oracle_median_keep(n_alive, sv_alive, med_num, med_den, keep);
    int n_final = 0;
    q = 0;
    for (int i = 0; i < nL; ++i) {
        if (!alive[i]) continue;
        if (!keep[q++]) continue;
        out_j[i] = cj[i]; out_h[i] = ch[i]; out_ur[i] = cu[i]; out_depth[i] = cd[i];
        out_sad[i] = cs[i];
        ++n_final;
    }
    free(sv_alive); free(keep);
    if (stats) {
        stats[0] = n_ham; stats[1] = n_ref; stats[2] = n_ref_ok; stats[3] = n_alive;
        stats[4] = median; stats[5] = n_final;
    }
    free(cj); free(ch); free(cs); free(cu); free(cd); free(alive); free(sadv);
}

/* ------------------------------------------------------------------------ */
/* Kannala-Brandt fisheye model: theta_d = theta (1 + k1 t^2 + k2 t^4 +      */
/* k3 t^6 + k4 t^8), image radius = f * theta_d.                            */
/* ------------------------------------------------------------------------ */
/* Level sizes and packed offsets of the image pyramid (see ft_oracle.h). */
int64_t oracle_pyramid_layout(int W, int H, const float *inv_sf, int n_levels,
                              int32_t *w, int32_t *h, int64_t *off)
{
    int64_t acc = 0;
    for (int l = 0; l < n_levels; ++l) {
        const float fw = (float)W * inv_sf[l];
        const float fh = (float)H * inv_sf[l];
        w[l] = (int32_t)floorf(fw + 0.5f);
        h[l] = (int32_t)floorf(fh + 0.5f);
        off[l] = acc;
        acc += (int64_t)w[l] * h[l];
    }
    return acc;
}

/* Source pixel and 8-bit weight of output index x of a level n_out wide from a
 * source n_in wide: s = ((2x + 1) * n_in - n_out) / (2 * n_out), i.e.
 * (x + 1/2) * n_in / n_out - 1/2, as an exact fraction. */
static void pyramid_tap(int x, int n_in, int n_out, int *i0, int *wt)
{
    const int64_t num = (int64_t)(2 * x + 1) * n_in - n_out;
    const int64_t den = 2 * (int64_t)n_out;
    if (num <= 0) {                         /* left of the first pixel centre */
        *i0 = 0;
        *wt = 0;
        return;
    }
    int64_t q = num / den;
    int64_t r = num % den;
    int64_t wq = (256 * r) / den;           /* floor(256 * frac(s)) */
    if (q >= n_in - 1) {                    /* right of the last pixel centre */
        q = n_in - 1;
        wq = 0;
    }
    *i0 = (int)q;
    *wt = (int)wq;
}

void oracle_pyramid(const uint8_t *img, int W, int H, int pitch, const float *inv_sf, int n_levels,
                    uint8_t *out)
{
    int32_t w[64], h[64];
    int64_t off[64];
    if (n_levels > 64) return;
    oracle_pyramid_layout(W, H, inv_sf, n_levels, w, h, off);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) out[(size_t)y * W + x] = img[(size_t)y * pitch + x];
    for (int l = 1; l < n_levels; ++l) {
        uint8_t *dst = out + off[l];
        for (int y = 0; y < h[l]; ++y) {
            int y0, b;
            pyramid_tap(y, H, h[l], &y0, &b);
            const int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
            for (int x = 0; x < w[l]; ++x) {
                int x0, a;
                pyramid_tap(x, W, w[l], &x0, &a);
                const int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
                const int p00 = img[(size_t)y0 * pitch + x0], p01 = img[(size_t)y0 * pitch + x1];
                const int p10 = img[(size_t)y1 * pitch + x0], p11 = img[(size_t)y1 * pitch + x1];
                const int top = (256 - a) * p00 + a * p01;
                const int bot = (256 - a) * p10 + a * p11;
                const int v = (256 - b) * top + b * bot;
                dst[(size_t)y * w[l] + x] = (uint8_t)((v + 32768) >> 16);
            }
        }
    }
}

static double kb_distort(const float *kb, double th)
{
    const double k1 = kb[4], k2 = kb[5], k3 = kb[6], k4 = kb[7];
    const double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    return th * ((((1.0 + k1 * t2) + k2 * t4) + k3 * t6) + k4 * t8);
}

void oracle_kb_project(const float *kb, const double *X, double *uv)
{
    const double fx = kb[0], fy = kb[1], cx = kb[2], cy = kb[3];
    const double rho = sqrt(X[0] * X[0] + X[1] * X[1]);
    if (rho == 0.0) { uv[0] = cx; uv[1] = cy; return; }
    const double th = atan2(rho, X[2]);
    const double thd = kb_distort(kb, th);
    uv[0] = fx * ((thd * X[0]) / rho) + cx;
    uv[1] = fy * ((thd * X[1]) / rho) + cy;
}

/* Newton's method on theta_d(theta) = r, started at theta = r. Returns 0 when
 * the ray is rejected (theta at or beyond max_theta). */
int oracle_kb_unproject(const float *kb, float u, float v, int iters, double tol,
                        double max_theta, double *ray)
{
    const double fx = kb[0], fy = kb[1], cx = kb[2], cy = kb[3];
    const double k1 = kb[4], k2 = kb[5], k3 = kb[6], k4 = kb[7];
    const double xp = ((double)u - cx) / fx;
    const double yp = ((double)v - cy) / fy;
    double thd = sqrt(xp * xp + yp * yp);
    const double half_pi = 1.5707963267948966;
    if (thd > half_pi) thd = half_pi;
    if (!(thd > 1e-8)) { ray[0] = xp; ray[1] = yp; ray[2] = 1.0; return 1; }
    double th = thd;
    for (int it = 0; it < iters; ++it) {
        const double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
        const double f = th * ((((1.0 + k1 * t2) + k2 * t4) + k3 * t6) + k4 * t8) - thd;
        const double fp = (((1.0 + 3.0 * k1 * t2) + 5.0 * k2 * t4) + 7.0 * k3 * t6) + 9.0 * k4 * t8;
        const double step = f / fp;
        th = th - step;
        if (fabs(step) < tol) break;
    }
    if (!(th < max_theta)) return 0;
    const double scale = tan(th) / thd;
    ray[0] = xp * scale; ray[1] = yp * scale; ray[2] = 1.0;
    return 1;
}

static double det3(const double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
         - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
         + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

/* Linear least-squares triangulation of two rays with the homogeneous
 * coordinate fixed to 1: camera 1 is [I|0] (left), camera 2 is [R_rl|t_rl]
 * with R_rl = R_lr^T, t_rl = -R_lr^T t_lr.  Each view contributes the rows
 * p.x P3 - P1 and p.y P3 - P2 (p = the ray scaled to z = 1); the 3x3 normal
 * equations are solved by Cramer's rule.  Returns 0 on a singular system. */
int oracle_triangulate(const double *r1, const double *r2, const float *R_lr,
                       const float *t_lr, double *X)
{
    double Rrl[3][3], trl[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rrl[r][c] = (double)R_lr[3 * c + r];
    for (int r = 0; r < 3; ++r)
        trl[r] = -(((Rrl[r][0] * (double)t_lr[0]) + Rrl[r][1] * (double)t_lr[1]) + Rrl[r][2] * (double)t_lr[2]);
    const double p1x = r1[0] / r1[2], p1y = r1[1] / r1[2];
    const double p2x = r2[0] / r2[2], p2y = r2[1] / r2[2];
    double A[4][3], bb[4];
    A[0][0] = -1.0; A[0][1] = 0.0; A[0][2] = p1x; bb[0] = 0.0;
    A[1][0] = 0.0; A[1][1] = -1.0; A[1][2] = p1y; bb[1] = 0.0;
    for (int c = 0; c < 3; ++c) {
        A[2][c] = p2x * Rrl[2][c] - Rrl[0][c];
        A[3][c] = p2y * Rrl[2][c] - Rrl[1][c];
    }
    bb[2] = -(p2x * trl[2] - trl[0]);
    bb[3] = -(p2y * trl[2] - trl[1]);
    double M[3][3], v[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc = acc + A[k][r] * A[k][c];
            M[r][c] = acc;
        }
        double acc = 0.0;
        for (int k = 0; k < 4; ++k) acc = acc + A[k][r] * bb[k];
        v[r] = acc;
    }
    const double D = det3(M);
    if (D == 0.0 || !isfinite(D)) return 0;
    for (int c = 0; c < 3; ++c) {
        double Mc[3][3];
        memcpy(Mc, M, sizeof(Mc));
        for (int r = 0; r < 3; ++r) Mc[r][c] = v[r];
        X[c] = det3(Mc) / D;
    }
    return 1;
}

/* Fisheye stereo (Section II-B, IV-C): brute force over the right keypoints of
 * the overlap region, two nearest neighbours by Hamming distance, a ratio test,
 * then a parallax / triangulation / reprojection check of the best pair. */
void oracle_stereo_fisheye(
    int nL, const float *xL, const float *yL, const uint8_t *oL, const uint8_t *dL,
    int nR, const float *xR, const float *yR, const uint8_t *oR, const uint8_t *dR,
    const float *kbL, const float *kbR, const float *R_lr, const float *t_lr,
    const float *ovl, const float *ovr, const float *sigma2,
    const int32_t *ip, const double *dp,
    int32_t *out_j, int32_t *out_h, float *out_depth, float *out_xyz, int32_t *out_h2,
    int64_t *stats)
{
    const int ratio_num = ip[0], ratio_den = ip[1], iters = ip[2];
    const double cos_max = dp[0], chi2 = dp[1], max_theta = dp[2], tol = dp[3];
    int64_t nQ = 0, nT = 0, n_ratio = 0, n_tri = 0;
    int64_t n_par = 0, n_dep = 0, n_rep = 0;   /* rejections by the parallax, depth and reprojection tests */
    int32_t *cj = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    int32_t *ch = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    float *cdep = (float *)malloc(sizeof(float) * (nL > 0 ? nL : 1));
    float *cx3 = (float *)malloc(sizeof(float) * 3 * (nL > 0 ? nL : 1));
    uint8_t *alive = (uint8_t *)calloc(nL > 0 ? nL : 1, 1);

    for (int j = 0; j < nR; ++j)
        if (xR[j] >= ovr[0] && xR[j] <= ovr[1]) ++nT;
    for (int i = 0; i < nL; ++i) {
        out_j[i] = -1; out_h[i] = -1; out_depth[i] = -1.0f;
        out_xyz[3 * i] = 0.0f; out_xyz[3 * i + 1] = 0.0f; out_xyz[3 * i + 2] = 0.0f;
        if (out_h2) out_h2[i] = -1;
        if (!(xL[i] >= ovl[0] && xL[i] <= ovl[1])) continue;
        ++nQ;
        if (nT < 2) continue;
        int h1 = 1000, j1 = -1, h2 = 1000;
        for (int j = 0; j < nR; ++j) {
            if (!(xR[j] >= ovr[0] && xR[j] <= ovr[1])) continue;
            const int h = oracle_hamming(dL + 32 * (size_t)i, dR + 32 * (size_t)j);
            if (h < h1) { h2 = h1; h1 = h; j1 = j; }
            else if (h < h2) { h2 = h; }
        }
        if (out_h2) out_h2[i] = h2;
        if (!(ratio_den * h1 < ratio_num * h2)) continue;
        ++n_ratio;
        double r1[3], r2[3];
        if (!oracle_kb_unproject(kbL, xL[i], yL[i], iters, tol, max_theta, r1)) continue;
        if (!oracle_kb_unproject(kbR, xR[j1], yR[j1], iters, tol, max_theta, r2)) continue;
        double r21[3];
        for (int r = 0; r < 3; ++r)
            r21[r] = (((double)R_lr[3 * r] * r2[0]) + (double)R_lr[3 * r + 1] * r2[1]) + (double)R_lr[3 * r + 2] * r2[2];
        const double n1 = sqrt((r1[0] * r1[0] + r1[1] * r1[1]) + r1[2] * r1[2]);
        const double n2 = sqrt((r21[0] * r21[0] + r21[1] * r21[1]) + r21[2] * r21[2]);
        const double cosp = ((r1[0] * r21[0] + r1[1] * r21[1]) + r1[2] * r21[2]) / (n1 * n2);
        if (!(cosp <= cos_max)) { ++n_par; continue; }
        double X[3];
        if (!oracle_triangulate(r1, r2, R_lr, t_lr, X)) continue;
        if (!(X[2] > 0.0)) { ++n_dep; continue; }
        double X2[3];
        for (int r = 0; r < 3; ++r) {
            /* right-camera coordinates: R_lr^T (X - t_lr) */
            X2[r] = (((double)R_lr[r] * (X[0] - (double)t_lr[0])) +
                     (double)R_lr[3 + r] * (X[1] - (double)t_lr[1])) +
                    (double)R_lr[6 + r] * (X[2] - (double)t_lr[2]);
        }
        if (!(X2[2] > 0.0)) { ++n_dep; continue; }
        /* reprojection error in each view against that keypoint's own octave */
        double uv[2];
        oracle_kb_project(kbL, X, uv);
        double ex = uv[0] - (double)xL[i], ey = uv[1] - (double)yL[i];
        if (!(ex * ex + ey * ey <= chi2 * (double)sigma2[oL[i]])) { ++n_rep; continue; }
        oracle_kb_project(kbR, X2, uv);
        ex = uv[0] - (double)xR[j1]; ey = uv[1] - (double)yR[j1];
        if (!(ex * ex + ey * ey <= chi2 * (double)sigma2[oR[j1]])) { ++n_rep; continue; }
        ++n_tri;
        cj[i] = j1; ch[i] = h1; cdep[i] = (float)X[2];
        cx3[3 * i] = (float)X[0]; cx3[3 * i + 1] = (float)X[1]; cx3[3 * i + 2] = (float)X[2];
        alive[i] = 1;
    }
    resolve_conflicts(nL, cj, ch, nR, alive);
    int64_t n_final = 0;
    for (int i = 0; i < nL; ++i) {
        if (!alive[i]) continue;
        out_j[i] = cj[i]; out_h[i] = ch[i]; out_depth[i] = cdep[i];
        out_xyz[3 * i] = cx3[3 * i]; out_xyz[3 * i + 1] = cx3[3 * i + 1];
        out_xyz[3 * i + 2] = cx3[3 * i + 2];
        ++n_final;
    }
    if (stats) {
        stats[0] = nQ; stats[1] = nT; stats[2] = n_ratio; stats[3] = n_tri; stats[4] = n_final;
        stats[5] = n_par; stats[6] = n_dep; stats[7] = n_rep;
    }
    free(cj); free(ch); free(cdep); free(cx3); free(alive);
}

/* ------------------------------------------------------------------------ */
/* Search by projection (Section II-D, IV-E): project each local map point   */
/* with the frame pose, keep it if it is in view at a plausible distance and */
/* viewing angle, predict its pyramid level, then take the best and second  */
/* best keypoints by Hamming distance inside a level- and angle-dependent    */
/* window around the projection.                                             */
/* ------------------------------------------------------------------------ */
void oracle_search_local_points(
    int nM, const float *pos, const float *normal, const float *dmin, const float *dmax,
    const uint8_t *mdesc,
    int nK, const float *kx, const float *ky, const uint8_t *ko, const uint8_t *kdesc,
    const float *u_right, const uint8_t *preassigned,
    int model, const float *cam, const float *R, const float *t, const float *O,
    const float *bounds, const float *sf, int n_levels,
    const float *fp, const int32_t *ip,
    int32_t *mp_match, int32_t *mp_dist, int32_t *kp_match, int64_t *stats)
{
    const float th = fp[0], cos_lim = fp[1], cos_narrow = fp[2];
    const float r_narrow = fp[3], r_wide = fp[4], dist_lo = fp[5], dist_hi = fp[6];
    const int lv_lo = ip[0], lv_hi = ip[1], th_high = ip[2];
    const int ratio_num = ip[3], ratio_den = ip[4], same_level_only = ip[5];
    const float fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3], bf = cam[8];
    int64_t n_vis = 0, n_cand = 0, n_acc = 0;
    int64_t n_out = 0, n_near = 0, n_far = 0, n_angle = 0;   /* rejections by each visibility gate */
    int32_t *cand_k = (int32_t *)malloc(sizeof(int32_t) * (nM > 0 ? nM : 1));
    int32_t *cand_h = (int32_t *)malloc(sizeof(int32_t) * (nM > 0 ? nM : 1));
    uint8_t *alive = (uint8_t *)calloc(nM > 0 ? nM : 1, 1);

    for (int k = 0; k < nK; ++k) kp_match[k] = -1;
    for (int m = 0; m < nM; ++m) {
        mp_match[m] = -1; mp_dist[m] = -1;
        const float X = pos[3 * m], Y = pos[3 * m + 1], Z = pos[3 * m + 2];
        const float xc = ((R[0] * X + R[1] * Y) + R[2] * Z) + t[0];
        const float yc = ((R[3] * X + R[4] * Y) + R[5] * Z) + t[1];
        const float zc = ((R[6] * X + R[7] * Y) + R[8] * Z) + t[2];
        if (!(zc > 0.0f)) { ++n_out; continue; }
        float u, v;
        if (model == 0) {
            u = ((fx * xc) / zc) + cx;
            v = ((fy * yc) / zc) + cy;
        } else {
            double Pc[3] = {(double)xc, (double)yc, (double)zc}, uv[2];
            oracle_kb_project(cam, Pc, uv);
            u = (float)uv[0];
            v = (float)uv[1];
        }
        if (!(u >= bounds[0] && u <= bounds[1] && v >= bounds[2] && v <= bounds[3])) { ++n_out; continue; }
        /* scale invariance: the point must be seen from inside its distance range */
        const float pox = X - O[0], poy = Y - O[1], poz = Z - O[2];
        const float dist = sqrtf((pox * pox + poy * poy) + poz * poz);
        const float lo = dist_lo * dmin[m], hi = dist_hi * dmax[m];
        if (!(dist >= lo)) { ++n_near; continue; }
        if (!(dist <= hi)) { ++n_far; continue; }
        /* viewing angle: the ray from the camera must be close to the mean viewing direction */
        const float vcos = ((pox * normal[3 * m] + poy * normal[3 * m + 1]) + poz * normal[3 * m + 2]) / dist;
        if (!(vcos >= cos_lim)) { ++n_angle; continue; }
        const int pred = oracle_predict_level(dmax[m] / dist, sf, n_levels);
        ++n_vis;
        const float rbase = (vcos > cos_narrow ? r_narrow : r_wide) * th;
        const float Rm = rbase * sf[pred];
        float uR = 0.0f;
        if (u_right) uR = u - bf * (1.0f / zc);

        int b1 = 1000, k1 = -1, l1 = -1, b2 = 1000, l2 = -1;
        for (int k = 0; k < nK; ++k) {
            const int ok = ko[k];
            if (ok < pred - lv_lo || ok > pred + lv_hi) continue;
            if (!(fabsf(kx[k] - u) < Rm && fabsf(ky[k] - v) < Rm)) continue;
            if (preassigned && preassigned[k]) continue;
            if (u_right && u_right[k] > 0.0f && !(fabsf(uR - u_right[k]) <= Rm)) continue;
            ++n_cand;
            const int h = oracle_hamming(mdesc + 32 * (size_t)m, kdesc + 32 * (size_t)k);
            if (h < b1) { b2 = b1; l2 = l1; b1 = h; k1 = k; l1 = ok; }
            else if (h < b2) { b2 = h; l2 = ok; }
        }
        if (k1 < 0) continue;
        if (b2 == 1000) { b2 = 256; l2 = -1; }
        if (!(b1 <= th_high)) continue;
        const int fails_ratio = ratio_den * b1 > ratio_num * b2;
        if (same_level_only ? (l1 == l2 && fails_ratio) : fails_ratio) continue;
        ++n_acc;
        cand_k[m] = k1; cand_h[m] = b1; alive[m] = 1;
    }
    resolve_conflicts(nM, cand_k, cand_h, nK, alive);
    int64_t n_match = 0;
    for (int m = 0; m < nM; ++m) {
        if (!alive[m]) continue;
        mp_match[m] = cand_k[m]; mp_dist[m] = cand_h[m]; kp_match[cand_k[m]] = m;
        ++n_match;
    }
    if (stats) {
        stats[0] = n_vis; stats[1] = n_cand; stats[2] = n_acc; stats[3] = n_match;
        stats[4] = n_out; stats[5] = n_near; stats[6] = n_far; stats[7] = n_angle;
    }
    free(cand_k); free(cand_h); free(alive);
}

/* Rotation bin of a match between a last-frame keypoint (orientation a_last)
 * and a current keypoint (a_cur), degrees: the rotation plus 360 when
 * negative, rounded to one of `bins` equal bins and taken modulo `bins` (for
 * angles in [0, 360) only the bin past the last wraps, to 0). */
int oracle_rotation_bin(float a_last, float a_cur, int bins)
{
    float rot = a_last - a_cur;
    if (rot < 0.0f) rot += 360.0f;
    const float factor = (float)bins / 360.0f;
    int bin = (int)roundf(rot * factor) % bins;   /* the bin past the last is bin 0 */
    if (bin < 0) bin += bins;
    return bin;
}

/* The fullest bin, then the second and third fullest (ties to the lower bin),
 * the latter two kept only while 10 * count >= the fullest count.  kept[b] is
 * set to 1 for the kept bins and 0 for the others. */
void oracle_three_fullest(const int32_t *count, int bins, int32_t *kept)
{
    int i1 = -1, i2 = -1, i3 = -1;
    int m1 = 0, m2 = 0, m3 = 0;
    for (int b = 0; b < bins; ++b) {
        const int c = count[b];
        if (c > m1) { m3 = m2; i3 = i2; m2 = m1; i2 = i1; m1 = c; i1 = b; }
        else if (c > m2) { m3 = m2; i3 = i2; m2 = c; i2 = b; }
        else if (c > m3) { m3 = c; i3 = b; }
    }
    if (10 * m2 < m1) { i2 = -1; i3 = -1; }
    else if (10 * m3 < m1) i3 = -1;
    for (int b = 0; b < bins; ++b) kept[b] = (b == i1 || b == i2 || b == i3) ? 1 : 0;
}

void oracle_search_last_frame(
    int nL, const float *lpos, const uint8_t *ldesc, const uint8_t *lo, const float *la,
    int nK, const float *kx, const float *ky, const uint8_t *ko, const uint8_t *kdesc,
    const float *ka, const float *u_right, const uint8_t *preassigned,
    int model, const float *cam, const float *R, const float *t, const float *bounds,
    const float *sf, int n_levels, const float *fp, const int32_t *ip,
    int32_t *l_match, int32_t *l_dist, int32_t *kp_match, int64_t *stats)
{
    const float th = fp[0];
    const int th_high = ip[0], direction = ip[1], check_rot = ip[2], bins = ip[3];
    const float fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3], bf = cam[8];
    int64_t n_in = 0, n_cand = 0, n_acc = 0;
    int32_t *cand_k = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    int32_t *cand_h = (int32_t *)malloc(sizeof(int32_t) * (nL > 0 ? nL : 1));
    uint8_t *alive = (uint8_t *)calloc(nL > 0 ? nL : 1, 1);

    for (int k = 0; k < nK; ++k) kp_match[k] = -1;
    for (int i = 0; i < nL; ++i) {
        l_match[i] = -1; l_dist[i] = -1;
        const float X = lpos[3 * i], Y = lpos[3 * i + 1], Z = lpos[3 * i + 2];
        const float xc = ((R[0] * X + R[1] * Y) + R[2] * Z) + t[0];
        const float yc = ((R[3] * X + R[4] * Y) + R[5] * Z) + t[1];
        const float zc = ((R[6] * X + R[7] * Y) + R[8] * Z) + t[2];
        if (!(zc > 0.0f)) continue;
        float u, v;
        if (model == 0) {
            u = ((fx * xc) / zc) + cx;
            v = ((fy * yc) / zc) + cy;
        } else {
            double Pc[3] = {(double)xc, (double)yc, (double)zc}, uv[2];
            oracle_kb_project(cam, Pc, uv);
            u = (float)uv[0];
            v = (float)uv[1];
        }
        if (!(u >= bounds[0] && u <= bounds[1] && v >= bounds[2] && v <= bounds[3])) continue;
        ++n_in;
        const int ol = lo[i];
        const float r = th * sf[ol < n_levels ? ol : n_levels - 1];
        int lv_min, lv_max;
        if (direction > 0) { lv_min = ol; lv_max = n_levels - 1; }
        else if (direction < 0) { lv_min = 0; lv_max = ol; }
        else { lv_min = ol - 1; lv_max = ol + 1; }
        float ur_proj = 0.0f;
        if (u_right) ur_proj = u - bf * (1.0f / zc);
        int best = 1000, kbest = -1;
        for (int k = 0; k < nK; ++k) {
            if (ko[k] < lv_min || ko[k] > lv_max) continue;
            if (!(fabsf(kx[k] - u) < r && fabsf(ky[k] - v) < r)) continue;
            if (preassigned && preassigned[k]) continue;
            if (u_right && u_right[k] > 0.0f && !(fabsf(ur_proj - u_right[k]) <= r)) continue;
            ++n_cand;
            const int h = oracle_hamming(ldesc + 32 * (size_t)i, kdesc + 32 * (size_t)k);
            if (h < best) { best = h; kbest = k; }
        }
        if (kbest < 0 || !(best <= th_high)) continue;
        ++n_acc;
        cand_k[i] = kbest; cand_h[i] = best; alive[i] = 1;
    }
    resolve_conflicts(nL, cand_k, cand_h, nK, alive);
    int64_t n_conf = 0;
    for (int i = 0; i < nL; ++i) n_conf += alive[i];
    int32_t kept3[3] = {-1, -1, -1};
    if (check_rot && bins > 0) {
        int32_t *count = (int32_t *)calloc((size_t)bins, sizeof(int32_t));
        int32_t *kept = (int32_t *)calloc((size_t)bins, sizeof(int32_t));
        for (int i = 0; i < nL; ++i)
            if (alive[i]) ++count[oracle_rotation_bin(la[i], ka[cand_k[i]], bins)];
        oracle_three_fullest(count, bins, kept);
        for (int i = 0; i < nL; ++i)
            if (alive[i] && !kept[oracle_rotation_bin(la[i], ka[cand_k[i]], bins)]) alive[i] = 0;
        for (int b = 0, n = 0; b < bins && n < 3; ++b)
            if (kept[b]) kept3[n++] = b;
        free(count); free(kept);
    }
    int64_t n_match = 0;
    for (int i = 0; i < nL; ++i) {
        if (!alive[i]) continue;
        l_match[i] = cand_k[i]; l_dist[i] = cand_h[i]; kp_match[cand_k[i]] = i;
        ++n_match;
    }
    if (stats) {
        stats[0] = n_in; stats[1] = n_cand; stats[2] = n_acc; stats[3] = n_conf; stats[4] = n_match;
        stats[5] = kept3[0]; stats[6] = kept3[1]; stats[7] = kept3[2];
    }
    free(cand_k); free(cand_h); free(alive);
}

/* Copy map record `from` over record `to`. */
static void map_copy(float *pos, float *normal, float *dmin, float *dmax, uint8_t *desc, int to,
                     const float *spos, const float *snormal, const float *sdmin, const float *sdmax,
                     const uint8_t *sdesc, int from)
{
    for (int c = 0; c < 3; ++c) {
        pos[3 * to + c] = spos[3 * from + c];
        normal[3 * to + c] = snormal[3 * from + c];
    }
    dmin[to] = sdmin[from];
    dmax[to] = sdmax[from];
    memcpy(desc + 32 * (size_t)to, sdesc + 32 * (size_t)from, 32);
}

int oracle_map_update(int n, int capacity, float *pos, float *normal, float *dmin, float *dmax, uint8_t *desc,
                      int n_remove, const int32_t *remove, int n_insert, const float *ipos,
                      const float *inormal, const float *idmin, const float *idmax, const uint8_t *idesc)
{
    if (n < 0 || n_remove < 0 || n_insert < 0 || n_remove > n) return -1;
    uint8_t *gone = (uint8_t *)calloc(n > 0 ? n : 1, 1);
    for (int i = 0; i < n_remove; ++i) {
        const int r = remove[i];
        if (r < 0 || r >= n || gone[r]) { free(gone); return -1; }
        gone[r] = 1;
    }
    const int n1 = n - n_remove;
    if ((int64_t)n1 + n_insert > capacity) { free(gone); return -1; }
    /* the k-th removed slot below n1 takes the k-th surviving point at or above n1 */
    int h = 0, src = n1;
    for (;;) {
        while (h < n1 && !gone[h]) ++h;
        while (src < n && gone[src]) ++src;
        if (h >= n1 || src >= n) break;
        map_copy(pos, normal, dmin, dmax, desc, h, pos, normal, dmin, dmax, desc, src);
        ++h;
        ++src;
    }
    for (int j = 0; j < n_insert; ++j)
        map_copy(pos, normal, dmin, dmax, desc, n1 + j, ipos, inormal, idmin, idmax, idesc, j);
    free(gone);
    return n1 + n_insert;
}

/* ------------------------------------------------------------------------ */
/* ORB extraction on the image pyramid (Section II-A: keypoints extracted    */
/* on every scale and described; Section IV-B: done on the device next to    */
/* the pyramid).  The readings are stated in ft_oracle.h.                    */

/* The 16 pixels at distance 3 from a centre, in order round the circle
 * (clockwise in image coordinates, starting straight above the centre). */
static const int orb_ring_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
static const int orb_ring_dy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

/* Largest threshold at which nine consecutive ring pixels are all brighter,
 * or all darker, than the centre by more than it: over the 16 arcs of nine
 * and both signs, the largest smallest difference, minus one (-1 when no arc
 * differs positively throughout). */
static int orb_fast_score(const uint8_t *img, int w, int x, int y)
{
    const int c = img[(size_t)y * w + x];
    int best = -1;
    for (int a = 0; a < 16; ++a) {
        int lo_bright = 256, lo_dark = 256;
        for (int k = 0; k < 9; ++k) {
            const int r = (a + k) % 16;
            const int v = img[(size_t)(y + orb_ring_dy[r]) * w + (x + orb_ring_dx[r])];
            if (v - c < lo_bright) lo_bright = v - c;
            if (c - v < lo_dark) lo_dark = c - v;
        }
        if (lo_bright - 1 > best) best = lo_bright - 1;
        if (lo_dark - 1 > best) best = lo_dark - 1;
    }
    return best;
}

void oracle_fast_score_map(const uint8_t *img, int w, int h, int t, int edge, uint8_t *out)
{
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int v = 0;
            if (x >= edge && x < w - edge && y >= edge && y < h - edge) {
                const int s = orb_fast_score(img, w, x, y);
                if (s >= t) v = s;
            }
            out[(size_t)y * w + x] = (uint8_t)v;
        }
}

int64_t oracle_orb_detect(const uint8_t *pyr, const int64_t *off, const int32_t *w, const int32_t *h,
                          int n_levels, const float *sf, int t, int edge, int64_t cap, int16_t *lx,
                          int16_t *ly, uint8_t *oct, uint8_t *score, float *x, float *y)
{
    int64_t n = 0;
    for (int l = 0; l < n_levels; ++l) {
        const int W = w[l], H = h[l];
        uint8_t *s = (uint8_t *)calloc((size_t)W * H + 1, 1);
        oracle_fast_score_map(pyr + off[l], W, H, t, edge, s);
        for (int yy = 0; yy < H; ++yy)
            for (int xx = 0; xx < W; ++xx) {
                const int v = s[(size_t)yy * W + xx];
                if (v == 0) continue;
                int keep = 1;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        const int nx = xx + dx, ny = yy + dy;
                        const int nb = (nx >= 0 && nx < W && ny >= 0 && ny < H) ? s[(size_t)ny * W + nx] : 0;
                        if (v <= nb) keep = 0;
                    }
                if (!keep) continue;
                if (n < cap) {
                    lx[n] = (int16_t)xx;
                    ly[n] = (int16_t)yy;
                    oct[n] = (uint8_t)l;
                    score[n] = (uint8_t)v;
                    x[n] = (float)xx * sf[l];
                    y[n] = (float)yy * sf[l];
                }
                ++n;
            }
        free(s);
    }
    return n;
}

/* 7-tap binomial weights of the descriptor's smoothing. */
static const int orb_blur_k[7] = {1, 6, 15, 20, 15, 6, 1};

void oracle_orb_blur(const uint8_t *img, int w, int h, uint8_t *out)
{
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * ((size_t)w * h + 1));
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int32_t acc = 0;
            for (int i = 0; i < 7; ++i) {
                int xs = x + i - 3;
                xs = xs < 0 ? 0 : (xs > w - 1 ? w - 1 : xs);
                acc += orb_blur_k[i] * img[(size_t)y * w + xs];
            }
            rows[(size_t)y * w + x] = acc;
        }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int32_t acc = 0;
            for (int j = 0; j < 7; ++j) {
                int ys = y + j - 3;
                ys = ys < 0 ? 0 : (ys > h - 1 ? h - 1 : ys);
                acc += orb_blur_k[j] * rows[(size_t)ys * w + x];
            }
            out[(size_t)y * w + x] = (uint8_t)((acc + 2048) >> 12);
        }
    free(rows);
}

/* The integer nearest to num / sqrt(m2), halves away from zero, decided
 * exactly: the largest k >= 0 with k = 0 or (2k - 1)^2 m2 <= 4 num^2, given
 * the sign of num. */
static int orb_round_ratio(int64_t num, int64_t m2)
{
    const int64_t a = num < 0 ? -num : num;
    int k = 0;
    for (;;) {
        const int64_t odd = 2 * (int64_t)(k + 1) - 1;
        if (odd * odd * m2 > 4 * a * a) break;
        ++k;
    }
    return num < 0 ? -k : k;
}

void oracle_orb_describe(const uint8_t *pyr, const uint8_t *blurred, const int64_t *off, const int32_t *w,
                         int n, const int16_t *lx, const int16_t *ly, const uint8_t *oct,
                         const int8_t *pattern, float *angle, uint8_t *desc)
{
    for (int i = 0; i < n; ++i) {
        const int l = oct[i], W = w[l], u = lx[i], v = ly[i];
        const uint8_t *img = pyr + off[l];
        const uint8_t *B = blurred + off[l];
        int64_t m10 = 0, m01 = 0;
        for (int dy = -15; dy <= 15; ++dy)
            for (int dx = -15; dx <= 15; ++dx) {
                if (dx * dx + dy * dy > 225) continue;
                const int I = img[(size_t)(v + dy) * W + (u + dx)];
                m10 += (int64_t)dx * I;
                m01 += (int64_t)dy * I;
            }
        double a = atan2((double)m01, (double)m10) * (180.0 / 3.14159265358979323846);
        if (a < 0.0) a += 360.0;
        angle[i] = (float)a;
        const int64_t m2 = m10 * m10 + m01 * m01;
        uint8_t *d = desc + 32 * (size_t)i;
        memset(d, 0, 32);
        for (int t = 0; t < 256; ++t) {
            const int x1 = pattern[4 * t], y1 = pattern[4 * t + 1];
            const int x2 = pattern[4 * t + 2], y2 = pattern[4 * t + 3];
            int c1 = x1, r1 = y1, c2 = x2, r2 = y2;
            if (m2 > 0) {   /* the pattern turned by the intensity-centroid angle */
                c1 = orb_round_ratio((int64_t)x1 * m10 - (int64_t)y1 * m01, m2);
                r1 = orb_round_ratio((int64_t)x1 * m01 + (int64_t)y1 * m10, m2);
                c2 = orb_round_ratio((int64_t)x2 * m10 - (int64_t)y2 * m01, m2);
                r2 = orb_round_ratio((int64_t)x2 * m01 + (int64_t)y2 * m10, m2);
            }
            if (B[(size_t)(v + r1) * W + (u + c1)] < B[(size_t)(v + r2) * W + (u + c2)])
                d[t / 8] |= (uint8_t)(1u << (t % 8));
        }
    }
}
