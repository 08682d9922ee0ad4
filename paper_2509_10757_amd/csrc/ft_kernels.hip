// HIP kernels of the tracking correspondence search for gfx950 (MI355X).
//
// Every kernel runs 256-thread workgroups (four 64-wide waves) and is written
// as phase functions over one frame job, so the single-frame calls and the
// batched submissions execute the very same code.  Build flags:
// -ffp-contract=off (no fused multiply-add: every float expression rounds
// exactly as written) with correctly rounded fp32 divide and sqrt.
//
// Phases per frame (Section IV-C and IV-E of the paper):
//   setup      row index of right keypoints (pinhole) | overlap lists (fisheye)
//              + per-view keypoint grids; clears claim tables and counters
//   stereo_a   pinhole best match per left keypoint (row band, xor+popcount)
//              | fisheye all-pairs top-2 on the matrix cores (int8 +-1 MFMA)
//   stereo_b   pinhole SAD refinement, one wave per match
//              | fisheye ratio + triangulation check (float64)
//   stereo_c   pinhole duplicate resolution + median filter + outputs
//              | fisheye duplicate resolution + outputs
//   search     projection + windowed best/second search, thread per map point
//   search_fin duplicate resolution + outputs

#include <hip/hip_runtime.h>

#include "ft_internal.h"

namespace ft {

typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ helpers
struct Desc {
    uint4 a, b;
};

__device__ __forceinline__ Desc load_desc(const uint8_t *base, int idx)
{
    const uint4 *p = reinterpret_cast<const uint4 *>(base + 32 * (size_t)idx);
    Desc d;
    d.a = p[0];
    d.b = p[1];
    return d;
}

__device__ __forceinline__ int hamming(const Desc &u, const Desc &v)
{
    return __popc(u.a.x ^ v.a.x) + __popc(u.a.y ^ v.a.y) + __popc(u.a.z ^ v.a.z) +
           __popc(u.a.w ^ v.a.w) + __popc(u.b.x ^ v.b.x) + __popc(u.b.y ^ v.b.y) +
           __popc(u.b.z ^ v.b.z) + __popc(u.b.w ^ v.b.w);
}

// Pyramid level of a keypoint as a table index (levels are 0..7 by contract;
// the clamp only keeps a malformed octave byte inside the tables).
__device__ __forceinline__ int lvl(uint8_t o) { return o < kLevels ? (int)o : kLevels - 1; }

// Workgroup-wide exclusive scan of a[0..n) in LDS; returns the total.
__device__ int wg_exclusive_scan(int *a, int n, int *tmp)
{
    const int tid = threadIdx.x;
    const int per = (n + kWG - 1) / kWG;
    const int beg = min(tid * per, n), end = min(beg + per, n);
    int s = 0;
    for (int i = beg; i < end; ++i) s += a[i];
    tmp[tid] = s;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        const int v = tid >= off ? tmp[tid - off] : 0;
        __syncthreads();
        tmp[tid] += v;
        __syncthreads();
    }
    int run = tmp[tid] - s;
    const int total = tmp[kWG - 1];
    for (int i = beg; i < end; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// Rows [lo, hi] of the row index covered by a right keypoint; false if none.
__device__ __forceinline__ bool band_rows(const DevJob &J, int j, int &lo, int &hi)
{
    const float y = J.R.y[j];
    const float r = J.band * J.sf[lvl(J.R.oct[j])];
    const float flo = floorf(y - r);
    const float fhi = ceilf(y + r);
    if (!(fhi >= 0.0f) || !(flo <= (float)(J.rows - 1))) return false;
    lo = flo < 0.0f ? 0 : (int)flo;
    hi = fhi > (float)(J.rows - 1) ? J.rows - 1 : (int)fhi;
    return lo <= hi;
}

__device__ __forceinline__ int cell_coord(float v, float lo, float inv, int n)
{
    const float f = (v - lo) * inv;
    if (!(f >= 0.0f)) return 0;           // negative or NaN
    if (!(f < (float)n)) return n - 1;
    return (int)f;
}

// ------------------------------------------------ setup: row index (pinhole)
__device__ void ph_rowband(const DevJob &J, int *cnt, int *tmp)
{
    const int tid = threadIdx.x;
    const int rows = J.rows, nR = J.R.n;
    for (int r = tid; r < rows; r += kWG) cnt[r] = 0;
    for (int j = tid; j < nR; j += kWG) J.claimR[j] = 0xFFFFFFFFu;
    __syncthreads();
    for (int j = tid; j < nR; j += kWG) {
        int lo, hi;
        if (!band_rows(J, j, lo, hi)) continue;
        for (int r = lo; r <= hi; ++r) atomicAdd(&cnt[r], 1);
    }
    __syncthreads();
    const int total = wg_exclusive_scan(cnt, rows, tmp);
    for (int r = tid; r < rows; r += kWG) J.row_off[r] = cnt[r];
    if (tid == 0) J.row_off[rows] = min(total, J.row_items_cap);
    __syncthreads();
    for (int j = tid; j < nR; j += kWG) {
        int lo, hi;
        if (!band_rows(J, j, lo, hi)) continue;
        for (int r = lo; r <= hi; ++r) {
            const int pos = atomicAdd(&cnt[r], 1);
            if (pos < J.row_items_cap) J.row_items[pos] = j;
        }
    }
}

// ------------------------------------------- setup: overlap lists (fisheye)
__device__ int compact_range(const float *x, int n, float a, float b, int32_t *out, int *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int base = 0;
    for (int s = 0; s < n; s += kWG) {
        const int i = s + tid;
        const bool p = i < n && x[i] >= a && x[i] <= b;
        const unsigned long long m = __ballot(p);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (p) out[off + rank] = i;
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
        base += tot;
    }
    return base;
}

__device__ void ph_overlap(const DevJob &J, int *wsum)
{
    const int tid = threadIdx.x;
    for (int j = tid; j < J.R.n; j += kWG) J.claimR[j] = 0xFFFFFFFFu;
    for (int i = tid; i < J.L.n; i += kWG) J.flag[i] = 0;
    const int nQ = compact_range(J.L.x, J.L.n, J.ovl[0], J.ovl[1], J.qlist, wsum);
    const int nT = compact_range(J.R.x, J.R.n, J.ovr[0], J.ovr[1], J.tlist, wsum);
    if (tid == 0) {
        J.counts[0] = nQ;
        J.counts[1] = nT;
        *J.o_nmatch = 0;
    }
}

// ------------------------------------------------ setup: keypoint grid
__device__ void ph_grid(const DevView &V, const DevKps &K, int *cnt, int *tmp)
{
    const int tid = threadIdx.x;
    const int cells = V.cols * V.rows;
    for (int c = tid; c < cells; c += kWG) cnt[c] = 0;
    for (int k = tid; k < K.n; k += kWG) V.claim[k] = 0xFFFFFFFFu;
    if (tid == 0) *V.n_matches = 0;
    __syncthreads();
    for (int k = tid; k < K.n; k += kWG) {
        const int cx = cell_coord(K.x[k], V.min_x, V.inv_cw, V.cols);
        const int cy = cell_coord(K.y[k], V.min_y, V.inv_ch, V.rows);
        atomicAdd(&cnt[cy * V.cols + cx], 1);
    }
    __syncthreads();
    const int total = wg_exclusive_scan(cnt, cells, tmp);
    for (int c = tid; c < cells; c += kWG) V.cell_off[c] = cnt[c];
    if (tid == 0) V.cell_off[cells] = total;
    __syncthreads();
    for (int k = tid; k < K.n; k += kWG) {
        const int cx = cell_coord(K.x[k], V.min_x, V.inv_cw, V.cols);
        const int cy = cell_coord(K.y[k], V.min_y, V.inv_ch, V.rows);
        const int pos = atomicAdd(&cnt[cy * V.cols + cx], 1);
        V.cell_items[pos] = k;
    }
}

// ------------------------------------- stereo_a (pinhole): row-band best match
__device__ void ph_best(const DevJob &J, int tile)
{
    const int i = tile * kWG + threadIdx.x;
    if (i >= J.L.n) return;
    int bj = -1, bh = 1 << 20;
    const float y = J.L.y[i];
    const float x = J.L.x[i];
    const float minU = x - J.maxD;
    const float maxU = x - 0.0f;
    if (y > -1.0f && y < (float)J.rows && !(maxU < 0.0f)) {
        const int row = (int)y;
        const int oi = J.L.oct[i];
        const Desc di = load_desc(J.L.desc, i);
        const int e = min(J.row_off[row + 1], J.row_items_cap);
        for (int idx = J.row_off[row]; idx < e; ++idx) {
            const int j = J.row_items[idx];
            const int oj = J.R.oct[j];
            if (oj < oi - J.level_window || oj > oi + J.level_window) continue;
            const float xj = J.R.x[j];
            if (!(xj >= minU && xj <= maxU)) continue;
            const int h = hamming(di, load_desc(J.R.desc, j));
            if (h < bh || (h == bh && j < bj)) {
                bh = h;
                bj = j;
            }
        }
    }
    const bool ok = bj >= 0 && bh < J.th_orb;
    J.best_j[i] = ok ? bj : -1;
    J.best_h[i] = ok ? bh : -1;
}

// ----------------------------- stereo_a (fisheye): all-pairs top-2 on MFMA
// Expand one descriptor byte to eight signed bytes: bit t -> byte t, 1 -> +1,
// 0 -> -1.  Then H(a, b) = (256 - <a, b>) / 2 exactly for the +-1 vectors.
__device__ __forceinline__ uint64_t pm1_bytes(uint32_t b)
{
    uint64_t x = (uint64_t)(b & 0xFFu) * 0x0101010101010101ull;
    x &= 0x8040201008040201ull;
    x = ((x + 0x7F7F7F7F7F7F7F7Full) >> 7) & 0x0101010101010101ull;
    return ~(x * 0xFEull);
}

// Operand of K-step s for lane group g: descriptor bytes 8s + 2g and 8s + 2g + 1.
// Any assignment of descriptor bits to (lane group, byte) works as long as the
// A and B operands use the same one, because the dot product sums over K.
__device__ __forceinline__ v4i pm1_operand(const Desc &d, int s, int g)
{
    const uint32_t w[8] = {d.a.x, d.a.y, d.a.z, d.a.w, d.b.x, d.b.y, d.b.z, d.b.w};
    const int byte0 = 8 * s + 2 * g;
    const uint32_t word = w[byte0 >> 2];
    const int sh = (byte0 & 3) * 8;
    const uint64_t lo = pm1_bytes(word >> sh);
    const uint64_t hi = pm1_bytes(word >> (sh + 8));
    v4i r;
    r.x = (int)(uint32_t)lo;
    r.y = (int)(uint32_t)(lo >> 32);
    r.z = (int)(uint32_t)hi;
    r.w = (int)(uint32_t)(hi >> 32);
    return r;
}

__device__ __forceinline__ void top2_insert(uint32_t key, uint32_t &k1, uint32_t &k2)
{
    if (key < k1) {
        k2 = k1;
        k1 = key;
    } else if (key < k2) {
        k2 = key;
    }
}

__device__ void ph_knn(const DevJob &J, int tile)
{
    const int nQ = J.counts[0], nT = J.counts[1];
    const int q0 = tile * kKnnQueriesPerWG + (threadIdx.x >> 6) * 16;
    if (q0 >= nQ || nT < 2) return;
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int qa = q0 + c;
    v4i A[4];
    if (qa < nQ) {
        const Desc dq = load_desc(J.L.desc, J.qlist[qa]);
        for (int s = 0; s < 4; ++s) A[s] = pm1_operand(dq, s, g);
    } else {
        for (int s = 0; s < 4; ++s) A[s] = v4i{0, 0, 0, 0};
    }
    uint32_t k1[4], k2[4];
    for (int r = 0; r < 4; ++r) k1[r] = k2[r] = 0xFFFFFFFFu;
    for (int t0 = 0; t0 < nT; t0 += 16) {
        const int tj = t0 + c;
        const bool tv = tj < nT;
        const int j = tv ? J.tlist[tj] : 0;
        v4i B[4];
        if (tv) {
            const Desc dt = load_desc(J.R.desc, j);
            for (int s = 0; s < 4; ++s) B[s] = pm1_operand(dt, s, g);
        } else {
            for (int s = 0; s < 4; ++s) B[s] = v4i{0, 0, 0, 0};
        }
        v4i acc = {0, 0, 0, 0};
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[s], B[s], acc, 0, 0, 0);
        // acc[r] = dot(query row 4g + r, target column c)
        if (tv) {
            for (int r = 0; r < 4; ++r) {
                const uint32_t h = (uint32_t)((256 - acc[r]) >> 1);
                top2_insert((h << 16) | (uint32_t)j, k1[r], k2[r]);
            }
        }
    }
    for (int r = 0; r < 4; ++r) {
        for (int m = 1; m < 16; m <<= 1) {
            const uint32_t o1 = __shfl_xor(k1[r], m);
            const uint32_t o2 = __shfl_xor(k2[r], m);
            const uint32_t lo = min(k1[r], o1), hi = max(k1[r], o1);
            k2[r] = min(hi, min(k2[r], o2));
            k1[r] = lo;
        }
    }
    if (c == 0) {
        for (int r = 0; r < 4; ++r) {
            const int q = q0 + 4 * g + r;
            if (q >= nQ) continue;
            const int i = J.qlist[q];
            J.best_j[i] = (int)(k1[r] & 0xFFFFu);
            J.best_h[i] = (int)(k1[r] >> 16);
            J.h2[i] = (int)(k2[r] >> 16);
        }
    }
}

// ------------------------------------- stereo_b (pinhole): SAD refinement
__device__ void ph_refine(const DevJob &J, int tile)
{
    const int lane = threadIdx.x & 63;
    const int i = tile * kRefinePerWG + (threadIdx.x >> 6);
    if (i >= J.L.n) return;
    const int j = J.best_j[i];
    if (j < 0) {
        if (lane == 0) J.flag[i] = 0;
        return;
    }
    const int w = J.half_win, L = J.half_range;
    const int l = lvl(J.L.oct[i]);
    const float s = J.inv_sf[l];
    const int su = (int)roundf(J.L.x[i] * s);
    const int sv = (int)roundf(J.L.y[i] * s);
    const int su0 = (int)roundf(J.R.x[j] * s);
    const int Wl = J.lv_w[l], Hl = J.lv_h[l];
    if (su - w < 0 || su + w >= Wl || sv - w < 0 || sv + w >= Hl || su0 - L - w < 0 ||
        su0 + L + w >= Wl) {
        if (lane == 0) J.flag[i] = 0;
        return;
    }
    const uint8_t *IL = J.pyrL + J.lv_off[l];
    const uint8_t *IR = J.pyrR + J.lv_off[l];
    const int nS = 2 * L + 1;          // shifts
    const int parts = 64 / nS;         // lanes per shift
    const int side = 2 * w + 1;
    const int k_idx = lane / parts, part = lane - k_idx * parts;
    int acc = 0;
    if (k_idx < nS) {
        const int k = k_idx - L;
        const int cL = IL[(size_t)sv * Wl + su];
        const int cR = IR[(size_t)sv * Wl + su0 + k];
        for (int dyi = part; dyi < side; dyi += parts) {
            const uint8_t *pl = IL + (size_t)(sv + dyi - w) * Wl + su - w;
            const uint8_t *pr = IR + (size_t)(sv + dyi - w) * Wl + su0 + k - w;
            for (int dx = 0; dx < side; ++dx) acc += abs(((int)pl[dx] - cL) - ((int)pr[dx] - cR));
        }
    }
    // sum the `parts` partial sums of each shift into the first lane of its group
    int tot = acc;
    for (int p = 1; p < parts; ++p) tot += __shfl(acc, min(lane + p, 63));
    // gather the profile in every lane (all lanes take part in the shuffles);
    // ties go to the smaller shift; lane 0 then decides
    int best = 0x7FFFFFFF, kb = -L;
    for (int kk = 0; kk < nS; ++kk) {
        const int v = __shfl(tot, kk * parts);
        if (v < best) {
            best = v;
            kb = kk - L;
        }
    }
    const int a = __shfl(tot, max(kb + L - 1, 0) * parts);
    const int e = __shfl(tot, min(kb + L + 1, nS - 1) * parts);
    const int c = best;
    if (lane != 0) return;
    if (kb == -L || kb == L) {
        J.flag[i] = 0;
        return;
    }
    const float num = (float)(a - e);
    const float den = (float)(2 * (a + e - 2 * c));
    const float delta = num / den;
    if (delta < -1.0f || delta > 1.0f) {
        J.flag[i] = 0;
        return;
    }
    const float xi = J.L.x[i];
    float uR = J.sf[l] * (((float)su0 + (float)kb) + delta);
    float disp = xi - uR;
    if (!(disp >= 0.0f && disp < J.maxD)) {
        J.flag[i] = 0;
        return;
    }
    if (disp <= 0.0f) {
        disp = 0.01f;
        uR = (float)((double)xi - 0.01);
    }
    J.sad[i] = c;
    J.uR[i] = uR;
    J.depth[i] = J.bf / disp;
    J.flag[i] = 1;
    atomicMin(&J.claimR[j], ((uint32_t)J.best_h[i] << 23) | (uint32_t)i);
}

// ------------------------------- stereo_b (fisheye): ratio + triangulation
__device__ double kb_distort(const float *kb, double th)
{
    const double k1 = kb[4], k2 = kb[5], k3 = kb[6], k4 = kb[7];
    const double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    return th * ((((1.0 + k1 * t2) + k2 * t4) + k3 * t6) + k4 * t8);
}

__device__ void kb_project(const float *kb, const double X[3], double uv[2])
{
    const double fx = kb[0], fy = kb[1], cx = kb[2], cy = kb[3];
    const double rho = sqrt(X[0] * X[0] + X[1] * X[1]);
    if (rho == 0.0) {
        uv[0] = cx;
        uv[1] = cy;
        return;
    }
    const double th = atan2(rho, X[2]);
    const double thd = kb_distort(kb, th);
    uv[0] = fx * ((thd * X[0]) / rho) + cx;
    uv[1] = fy * ((thd * X[1]) / rho) + cy;
}

__device__ bool kb_unproject(const float *kb, float u, float v, int iters, double tol,
                             double max_theta, double ray[3])
{
    const double fx = kb[0], fy = kb[1], cx = kb[2], cy = kb[3];
    const double k1 = kb[4], k2 = kb[5], k3 = kb[6], k4 = kb[7];
    const double xp = ((double)u - cx) / fx;
    const double yp = ((double)v - cy) / fy;
    double thd = sqrt(xp * xp + yp * yp);
    const double half_pi = 1.5707963267948966;
    if (thd > half_pi) thd = half_pi;
    if (!(thd > 1e-8)) {
        ray[0] = xp;
        ray[1] = yp;
        ray[2] = 1.0;
        return true;
    }
    double th = thd;
    for (int it = 0; it < iters; ++it) {
        const double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
        const double f = th * ((((1.0 + k1 * t2) + k2 * t4) + k3 * t6) + k4 * t8) - thd;
        const double fp = (((1.0 + 3.0 * k1 * t2) + 5.0 * k2 * t4) + 7.0 * k3 * t6) + 9.0 * k4 * t8;
        const double step = f / fp;
        th = th - step;
        if (fabs(step) < tol) break;
    }
    if (!(th < max_theta)) return false;
    const double scale = tan(th) / thd;
    ray[0] = xp * scale;
    ray[1] = yp * scale;
    ray[2] = 1.0;
    return true;
}

__device__ double det3(const double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// Linear least-squares triangulation with the homogeneous coordinate fixed to
// one; 3x3 normal equations solved by Cramer's rule (float64).
__device__ bool triangulate(const double r1[3], const double r2[3], const float *R_lr,
                            const float *t_lr, double X[3])
{
    double Rrl[3][3], trl[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rrl[r][c] = (double)R_lr[3 * c + r];
    for (int r = 0; r < 3; ++r)
        trl[r] = -(((Rrl[r][0] * (double)t_lr[0]) + Rrl[r][1] * (double)t_lr[1]) +
                   Rrl[r][2] * (double)t_lr[2]);
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
    if (D == 0.0 || !isfinite(D)) return false;
    for (int c = 0; c < 3; ++c) {
        double Mc[3][3];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) Mc[r][q] = q == c ? v[r] : M[r][q];
        X[c] = det3(Mc) / D;
    }
    return true;
}

__device__ void ph_tri(const DevJob &J, int tile)
{
    const int nQ = J.counts[0], nT = J.counts[1];
    const int q = tile * kWG + threadIdx.x;
    if (q >= nQ || nT < 2) return;
    const int i = J.qlist[q];
    const int j1 = J.best_j[i], h1 = J.best_h[i], h2 = J.h2[i];
    if (!(J.ratio_den * h1 < J.ratio_num * h2)) return;
    double r1[3], r2[3];
    if (!kb_unproject(J.kbL, J.L.x[i], J.L.y[i], J.newton_iters, J.newton_tol, J.max_theta, r1)) return;
    if (!kb_unproject(J.kbR, J.R.x[j1], J.R.y[j1], J.newton_iters, J.newton_tol, J.max_theta, r2)) return;
    double r21[3];
    for (int r = 0; r < 3; ++r)
        r21[r] = (((double)J.R_lr[3 * r] * r2[0]) + (double)J.R_lr[3 * r + 1] * r2[1]) +
                 (double)J.R_lr[3 * r + 2] * r2[2];
    const double n1 = sqrt((r1[0] * r1[0] + r1[1] * r1[1]) + r1[2] * r1[2]);
    const double n2 = sqrt((r21[0] * r21[0] + r21[1] * r21[1]) + r21[2] * r21[2]);
    const double cosp = ((r1[0] * r21[0] + r1[1] * r21[1]) + r1[2] * r21[2]) / (n1 * n2);
    if (!(cosp <= J.cos_max)) return;
    double X[3];
    if (!triangulate(r1, r2, J.R_lr, J.t_lr, X)) return;
    if (!(X[2] > 0.0)) return;
    double X2[3];
    for (int r = 0; r < 3; ++r)
        X2[r] = (((double)J.R_lr[r] * (X[0] - (double)J.t_lr[0])) +
                 (double)J.R_lr[3 + r] * (X[1] - (double)J.t_lr[1])) +
                (double)J.R_lr[6 + r] * (X[2] - (double)J.t_lr[2]);
    if (!(X2[2] > 0.0)) return;
    double uv[2];
    kb_project(J.kbL, X, uv);
    double ex = uv[0] - (double)J.L.x[i], ey = uv[1] - (double)J.L.y[i];
    if (!(ex * ex + ey * ey <= J.chi2 * (double)J.sigma2[lvl(J.L.oct[i])])) return;
    kb_project(J.kbR, X2, uv);
    ex = uv[0] - (double)J.R.x[j1];
    ey = uv[1] - (double)J.R.y[j1];
    if (!(ex * ex + ey * ey <= J.chi2 * (double)J.sigma2[lvl(J.R.oct[j1])])) return;
    J.depth[i] = (float)X[2];
    J.xyz[3 * i] = (float)X[0];
    J.xyz[3 * i + 1] = (float)X[1];
    J.xyz[3 * i + 2] = (float)X[2];
    J.flag[i] = 1;
    atomicMin(&J.claimR[j1], ((uint32_t)h1 << 23) | (uint32_t)i);
}

// ---------------------- stereo_c (pinhole): conflicts + median + outputs
__device__ __forceinline__ bool pinhole_survivor(const DevJob &J, int i)
{
    if (!J.flag[i]) return false;
    const int j = J.best_j[i];
    return J.claimR[j] == (((uint32_t)J.best_h[i] << 23) | (uint32_t)i);
}

// Value at rank `target` (0-based, ascending) of the 16-bit SAD of survivors,
// by a two-pass 8-bit radix select in LDS.
__device__ void ph_median(const DevJob &J, int *hist, int *sh)
{
    const int tid = threadIdx.x, nL = J.L.n;
    if (tid < 256) hist[tid] = 0;
    if (tid == 0) sh[0] = 0;
    __syncthreads();
    for (int i = tid; i < nL; i += kWG) {
        if (pinhole_survivor(J, i)) {
            atomicAdd(&sh[0], 1);
            atomicAdd(&hist[(J.sad[i] >> 8) & 0xFF], 1);
        }
    }
    __syncthreads();
    const int n = sh[0];
    if (tid == 0) {
        int target = n / 2, acc = 0, bin = 0;
        for (; bin < 256; ++bin) {
            if (acc + hist[bin] > target) break;
            acc += hist[bin];
        }
        sh[1] = bin;
        sh[2] = target - acc;
    }
    __syncthreads();
    const int hb = sh[1];
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    for (int i = tid; i < nL; i += kWG)
        if (pinhole_survivor(J, i) && ((J.sad[i] >> 8) & 0xFF) == hb) atomicAdd(&hist[J.sad[i] & 0xFF], 1);
    __syncthreads();
    if (tid == 0) {
        int target = sh[2], acc = 0, bin = 0;
        for (; bin < 256; ++bin) {
            if (acc + hist[bin] > target) break;
            acc += hist[bin];
        }
        sh[3] = (hb << 8) | bin;
        sh[4] = 0;
    }
    __syncthreads();
    const long long m = sh[3];
    int kept = 0;
    for (int i = tid; i < nL; i += kWG) {
        const bool keep = n > 0 && pinhole_survivor(J, i) &&
                          (long long)J.med_den * J.sad[i] < (long long)J.med_num * m;
        if (keep) {
            J.o_right_idx[i] = J.best_j[i];
            J.o_dist[i] = J.best_h[i];
            J.o_uR[i] = J.uR[i];
            J.o_depth[i] = J.depth[i];
            J.o_sad[i] = J.sad[i];
            ++kept;
        } else {
            J.o_right_idx[i] = -1;
            J.o_dist[i] = -1;
            J.o_uR[i] = -1.0f;
            J.o_depth[i] = -1.0f;
            J.o_sad[i] = -1;
        }
    }
    atomicAdd(&sh[4], kept);
    __syncthreads();
    if (tid == 0) *J.o_nmatch = sh[4];
}

// ---------------------- stereo_c (fisheye): conflicts + outputs
__device__ void ph_fish_final(const DevJob &J, int tile)
{
    const int i = tile * kWG + threadIdx.x;
    bool keep = false;
    if (i < J.L.n) {
        keep = J.flag[i] &&
               J.claimR[J.best_j[i]] == (((uint32_t)J.best_h[i] << 23) | (uint32_t)i);
        if (keep) {
            J.o_right_idx[i] = J.best_j[i];
            J.o_dist[i] = J.best_h[i];
            J.o_depth[i] = J.depth[i];
            J.o_xyz[3 * i] = J.xyz[3 * i];
            J.o_xyz[3 * i + 1] = J.xyz[3 * i + 1];
            J.o_xyz[3 * i + 2] = J.xyz[3 * i + 2];
        } else {
            J.o_right_idx[i] = -1;
            J.o_dist[i] = -1;
            J.o_depth[i] = -1.0f;
            J.o_xyz[3 * i] = 0.0f;
            J.o_xyz[3 * i + 1] = 0.0f;
            J.o_xyz[3 * i + 2] = 0.0f;
        }
    }
    const unsigned long long m = __ballot(keep);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(J.o_nmatch, (int)__popcll(m));
}

// ------------------------------------------------ search by projection
__device__ void ph_search(const DevJob &J, const DevView &V, const DevKps &K, int tile)
{
    const int m = tile * kWG + threadIdx.x;
    if (m >= J.nM) return;
    int k1 = -1;
    int b1 = 1 << 20;
    const float X = J.pos[3 * m], Y = J.pos[3 * m + 1], Z = J.pos[3 * m + 2];
    const float xc = ((V.R[0] * X + V.R[1] * Y) + V.R[2] * Z) + V.t[0];
    const float yc = ((V.R[3] * X + V.R[4] * Y) + V.R[5] * Z) + V.t[1];
    const float zc = ((V.R[6] * X + V.R[7] * Y) + V.R[8] * Z) + V.t[2];
    do {
        if (!(zc > 0.0f)) break;
        float u, v;
        if (V.model == FT_CAMERA_PINHOLE) {
            u = ((V.fx * xc) / zc) + V.cx;
            v = ((V.fy * yc) / zc) + V.cy;
        } else {
            const float kb[8] = {V.fx, V.fy, V.cx, V.cy, V.k[0], V.k[1], V.k[2], V.k[3]};
            const double Pc[3] = {(double)xc, (double)yc, (double)zc};
            double uv[2];
            kb_project(kb, Pc, uv);
            u = (float)uv[0];
            v = (float)uv[1];
        }
        if (!(u >= V.min_x && u <= V.max_x && v >= V.min_y && v <= V.max_y)) break;
        const float pox = X - V.O[0], poy = Y - V.O[1], poz = Z - V.O[2];
        const float dist = sqrtf((pox * pox + poy * poy) + poz * poz);
        const float dmin = J.dmin[m], dmax = J.dmax[m];
        const float lo = J.dist_lo * dmin, hi = J.dist_hi * dmax;
        if (!(dist >= lo && dist <= hi)) break;
        const float vcos =
            ((pox * J.normal[3 * m] + poy * J.normal[3 * m + 1]) + poz * J.normal[3 * m + 2]) / dist;
        if (!(vcos >= J.cos_lim)) break;
        const float ratio = dmax / dist;
        int pred = kLevels - 1;
        for (int l = 0; l < kLevels; ++l)
            if (J.sf[l] >= ratio) {
                pred = l;
                break;
            }
        const float rbase = (vcos > J.cos_narrow ? J.r_narrow : J.r_wide) * J.th;
        const float Rm = rbase * J.sf[pred];
        float uR = 0.0f;
        if (V.u_right) uR = u - V.bf * (1.0f / zc);
        // cells covering the window, one cell of margin on each side for rounding
        const int cx0 = max(cell_coord(u - Rm, V.min_x, V.inv_cw, V.cols) - 1, 0);
        const int cx1 = min(cell_coord(u + Rm, V.min_x, V.inv_cw, V.cols) + 1, V.cols - 1);
        const int cy0 = max(cell_coord(v - Rm, V.min_y, V.inv_ch, V.rows) - 1, 0);
        const int cy1 = min(cell_coord(v + Rm, V.min_y, V.inv_ch, V.rows) + 1, V.rows - 1);
        const Desc dm = load_desc(J.mdesc, m);
        int kk2 = -1, b2 = 1 << 20, l1 = -1, l2 = -1;
        const int plo = pred - J.lv_lo, phi = pred + J.lv_hi;
        for (int cy = cy0; cy <= cy1; ++cy) {
            const int c0 = V.cell_off[cy * V.cols + cx0];
            const int c1 = V.cell_off[cy * V.cols + cx1 + 1];
            for (int idx = c0; idx < c1; ++idx) {
                const int k = V.cell_items[idx];
                const int ok = K.oct[k];
                if (ok < plo || ok > phi) continue;
                if (!(fabsf(K.x[k] - u) < Rm && fabsf(K.y[k] - v) < Rm)) continue;
                if (V.preassigned && V.preassigned[k]) continue;
                if (V.u_right) {
                    const float ur = V.u_right[k];
                    if (ur > 0.0f && !(fabsf(uR - ur) <= Rm)) continue;
                }
                const int h = hamming(dm, load_desc(K.desc, k));
                if (h < b1 || (h == b1 && k < k1)) {
                    b2 = b1; kk2 = k1; l2 = l1;
                    b1 = h; k1 = k; l1 = ok;
                } else if (h < b2 || (h == b2 && k < kk2)) {
                    b2 = h; kk2 = k; l2 = ok;
                }
            }
        }
        if (k1 < 0) break;
        if (kk2 < 0) {
            b2 = 256;
            l2 = -1;
        }
        if (!(b1 <= J.th_high)) {
            k1 = -1;
            break;
        }
        const bool fails = J.s_ratio_den * b1 > J.s_ratio_num * b2;
        if (J.same_level_only ? (l1 == l2 && fails) : fails) {
            k1 = -1;
            break;
        }
    } while (false);
    V.mp_k[m] = k1;
    V.mp_h[m] = k1 >= 0 ? b1 : -1;
    if (k1 >= 0) atomicMin(&V.claim[k1], ((uint32_t)b1 << 23) | (uint32_t)m);
}

__device__ void ph_search_final(const DevJob &J, const DevView &V, const DevKps &K, int tile)
{
    const int idx = tile * kWG + threadIdx.x;
    if (idx < J.nM) {
        const int k = V.mp_k[idx];
        const bool keep = k >= 0 && V.claim[k] == (((uint32_t)V.mp_h[idx] << 23) | (uint32_t)idx);
        V.mp_match[idx] = keep ? k : -1;
        V.mp_dist[idx] = keep ? V.mp_h[idx] : -1;
    }
    bool has = false;
    if (idx < K.n) {
        const uint32_t c = V.claim[idx];
        has = c != 0xFFFFFFFFu;
        V.kp_match[idx] = has ? (int)(c & 0x7FFFFFu) : -1;
    }
    const unsigned long long m = __ballot(has);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(V.n_matches, (int)__popcll(m));
}

// ------------------------------------------------------------------ kernels
struct OneJob {
    DevJob j;
    __device__ __forceinline__ const DevJob &operator()(int) const { return j; }
};
struct JobTable {
    const DevJob *p;
    __device__ __forceinline__ const DevJob &operator()(int i) const { return p[i]; }
};

__device__ __forceinline__ const DevKps &view_kps(const DevJob &J, int v)
{
    return J.view[v].side ? J.R : J.L;
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_setup(Src src, int do_stereo, int do_search)
{
    __shared__ int lds[kMaxCells + 8];
    __shared__ int tmp[kWG];
    const DevJob &J = src(blockIdx.y);
    const int part = blockIdx.x;
    if (part == 0) {
        if (!do_stereo) return;
        if (J.flags & JOB_STEREO_PINHOLE) ph_rowband(J, lds, tmp);
        else if (J.flags & JOB_STEREO_FISHEYE) ph_overlap(J, tmp);
    } else {
        const int v = part - 1;
        if (!do_search || !(J.flags & (JOB_SEARCH0 << v))) return;
        ph_grid(J.view[v], view_kps(J, v), lds, tmp);
    }
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_stereo_a(Src src)
{
    const DevJob &J = src(blockIdx.y);
    if (J.flags & JOB_STEREO_PINHOLE) ph_best(J, blockIdx.x);
    else if (J.flags & JOB_STEREO_FISHEYE) ph_knn(J, blockIdx.x);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_stereo_b(Src src)
{
    const DevJob &J = src(blockIdx.y);
    if (J.flags & JOB_STEREO_PINHOLE) ph_refine(J, blockIdx.x);
    else if (J.flags & JOB_STEREO_FISHEYE) ph_tri(J, blockIdx.x);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_stereo_c(Src src)
{
    __shared__ int hist[256];
    __shared__ int sh[8];
    const DevJob &J = src(blockIdx.y);
    if (J.flags & JOB_STEREO_PINHOLE) {
        if (blockIdx.x == 0) ph_median(J, hist, sh);
    } else if (J.flags & JOB_STEREO_FISHEYE) {
        ph_fish_final(J, blockIdx.x);
    }
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_search(Src src)
{
    const DevJob &J = src(blockIdx.y);
    const int v = blockIdx.z;
    if (!(J.flags & (JOB_SEARCH0 << v))) return;
    ph_search(J, J.view[v], view_kps(J, v), blockIdx.x);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_search_final(Src src)
{
    const DevJob &J = src(blockIdx.y);
    const int v = blockIdx.z;
    if (!(J.flags & (JOB_SEARCH0 << v))) return;
    ph_search_final(J, J.view[v], view_kps(J, v), blockIdx.x);
}

template <class Src>
static hipError_t run(Src src, const LaunchDims &d, hipStream_t s, bool do_stereo, bool do_search,
                      hipEvent_t *ev)
{
    const dim3 blk(kWG);
    const int nj = d.n_jobs;
    auto mark = [&](int p) {
        if (ev) (void)hipEventRecord(ev[p], s);
    };
    mark(0);
    hipLaunchKernelGGL(k_setup<Src>, dim3(d.setup_x, nj), blk, 0, s, src, (int)do_stereo, (int)do_search);
    mark(1);
    if (do_stereo) {
        hipLaunchKernelGGL(k_stereo_a<Src>, dim3(max(d.tiles_stereo_a, 1), nj), blk, 0, s, src);
        mark(2);
        hipLaunchKernelGGL(k_stereo_b<Src>, dim3(max(d.tiles_stereo_b, 1), nj), blk, 0, s, src);
        mark(3);
        hipLaunchKernelGGL(k_stereo_c<Src>, dim3(max(d.tiles_stereo_c, 1), nj), blk, 0, s, src);
        mark(4);
    } else {
        mark(2); mark(3); mark(4);
    }
    if (do_search) {
        hipLaunchKernelGGL(k_search<Src>, dim3(max(d.tiles_search, 1), nj, 2), blk, 0, s, src);
        mark(5);
        hipLaunchKernelGGL(k_search_final<Src>, dim3(max(d.tiles_search_fin, 1), nj, 2), blk, 0, s, src);
        mark(6);
    } else {
        mark(5); mark(6);
    }
    return hipGetLastError();
}

hipError_t launch_pipeline(const DevJob *table, const DevJob &one, const LaunchDims &d,
                           hipStream_t stream, bool do_stereo, bool do_search, hipEvent_t *ev)
{
    if (table) return run(JobTable{table}, d, stream, do_stereo, do_search, ev);
    return run(OneJob{one}, d, stream, do_stereo, do_search, ev);
}

}  // namespace ft
