// HIP kernels of the tracking correspondence search for gfx950 (MI355X).
//
// Every kernel runs 256-thread workgroups (four 64-wide waves) and is written
// as phase functions over one frame job, so the single-frame calls and the
// batched submissions execute the very same code.  Build flags:
// -ffp-contract=off (no fused multiply-add: every float expression rounds
// exactly as written) with correctly rounded fp32 divide and sqrt.
//
// Phases per frame (Section IV-C and IV-E of the paper):
//   setup      counting sort of right keypoints by row (pinhole) | overlap
//              lists + packed target descriptors (fisheye); counting sort of
//              each view's keypoints by grid cell into packed records; clears
//              claim tables and counters
//   stereo_a   pinhole best match: G lanes per left keypoint stream the
//              row-sorted records of the rows that can hold a match
//              | fisheye all-pairs top-2 on the matrix cores (int8 +-1 MFMA)
//   refine     pinhole SAD refinement, one wave per match, patches in LDS
//   tri        fisheye ratio + triangulation check (float64; its own kernel
//              so that its register demand does not cap the refinement's
//              occupancy)
//   stereo_c   pinhole duplicate resolution + median filter + outputs
//              | fisheye duplicate resolution + outputs
//   search     projection + window search: G lanes per map point stream the
//              cell-sorted keypoint records of the window's cells
//   search_fin duplicate resolution + outputs
//
// Batched submissions flatten every phase's tiles over the jobs; the flat
// block index is first remapped so that consecutive tiles (one frame's data)
// land on the same XCD and share its L2.

#include <hip/hip_runtime.h>

#include <algorithm>

#define FT_KERNELS 1
#include "ft_internal.h"

namespace ft {

typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ helpers
struct Desc {
    uint4 a, b;
};

// 16-byte vector for copying descriptor halves through registers (a native
// vector type: arrays of it stay in registers, unlike arrays of uint4).
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Keypoints per thread whose loads are issued together in the setup sorts and
// the median pass (a strided loop body unrolled; surplus entries masked).
constexpr int kSortUnroll = 4;

// Candidates of a scan whose descriptors are read in one round.
constexpr int kCandBatch = 3;

// Candidates whose loads are issued together in the best-match and search scans.
constexpr int kBestUnroll = 2;
constexpr int kSearchUnroll = 2;

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

__host__ __device__ inline int div_up(int n, int d) { return (n + d - 1) / d; }

// The refinement runs four matches per wave for the 11x11 window and +-5 shifts.
__host__ __device__ inline bool refine_quarter(const DevJob &J) { return J.half_win == 5 && J.half_range == 5; }

__host__ __device__ inline int view_kp(const DevJob &J, int v) { return J.view[v].side ? J.R.n : J.L.n; }
// Entry l of a per-level table, selected from values loaded for every level
// (the loads do not wait for l; a select chain instead of a dependent load).
template <class T>
__device__ __forceinline__ T pick_level(const T (&t)[kLevels], int l)
{
    T v[kLevels];
    _Pragma("unroll") for (int k = 0; k < kLevels; ++k) v[k] = t[k];
    T r = v[0];
    _Pragma("unroll") for (int k = 1; k < kLevels; ++k) r = l == k ? v[k] : r;
    return r;
}

// Pyramid level of a keypoint as a table index (levels are 0..7 by contract;
// the clamp only keeps a malformed octave byte inside the tables).
__device__ __forceinline__ int lvl(uint32_t o) { return o < (uint32_t)kLevels ? (int)o : kLevels - 1; }

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// The two smallest keys seen so far (by value, so they stay in registers).
template <class T>
struct Top2 {
    T a, b;
};

template <class T>
__device__ __forceinline__ Top2<T> top2_insert(Top2<T> t, T key)
{
    const bool lt1 = key < t.a, lt2 = key < t.b;
    Top2<T> r;
    r.b = lt1 ? t.a : (lt2 ? key : t.b);
    r.a = lt1 ? key : t.a;
    return r;
}

template <class T>
__device__ __forceinline__ Top2<T> top2_merge(Top2<T> t, T o1, T o2)
{
    Top2<T> r;
    const T hi = t.a < o1 ? o1 : t.a;
    const T m2 = t.b < o2 ? t.b : o2;
    r.a = t.a < o1 ? t.a : o1;
    r.b = hi < m2 ? hi : m2;
    return r;
}

// Inclusive prefix across the 64 lanes of a wave (every lane active) with DPP
// lane moves: shifts by 1, 2, 4 and 8 inside each row of 16 lanes (lanes whose
// source lies in another row read 0), then lane 15 of rows 0 and 2 into rows
// 1 and 3, then lane 31 into rows 2 and 3.  Six VALU steps, no LDS traffic;
// 0 is the identity of both operations used (sum, and max of values >= 0).
template <bool kMax>
__device__ __forceinline__ int wave_inclusive_dpp(int v)
{
    auto op = [](int a, int b) { return kMax ? max(a, b) : a + b; };
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false));   // row_shr:8
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return v;
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) { return wave_inclusive_dpp<false>(v); }

// Inclusive prefix maximum of non-negative values across the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_max(int v) { return wave_inclusive_dpp<true>(v); }

// Value of lane 63 (the total of an inclusive scan), wave-uniform.
__device__ __forceinline__ int wave_last(int v) { return __builtin_amdgcn_readlane(v, 63); }

// Workgroup-wide exclusive scan of a[0..n) in LDS; returns the total.  Each
// thread owns a contiguous run of a[], the runs' sums are scanned inside each
// wave with lane shuffles, and the waves' totals (tmp[0..NT/64)) are combined
// after one barrier.
template <int NT>
__device__ __forceinline__ int wg_exclusive_scan(int *a, int n, int *tmp)
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + NT - 1) / NT;
    const int beg = min(tid * per, n), end = min(beg + per, n);
    int s = 0;
    for (int i = beg; i < end; ++i) s += a[i];
    const int inc = wave_inclusive_scan(s);
    if (lane == 63) tmp[wave] = inc;
    __syncthreads();
    int run = inc - s, total = 0;
    _Pragma("unroll") for (int w = 0; w < NW; ++w)
    {
        const int t = tmp[w];
        run += w < wave ? t : 0;
        total += t;
    }
    for (int i = beg; i < end; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ int cell_coord(float v, float lo, float inv, int n)
{
    const float f = (v - lo) * inv;
    if (!(f >= 0.0f)) return 0;           // negative or NaN
    if (!(f < (float)n)) return n - 1;
    return (int)f;
}

// ------------------------------------------------------ image pyramid
// Level l of a pyramid is a bilinear resample of level 0 (Section IV-B: the
// pyramid is built on the device and kept for stereo; every level is computed
// from the image at once, so one launch builds them all).  Output index x of a
// level n_out wide samples s = ((2x + 1) * n_in - n_out) / (2 * n_out) of the
// level-0 axis n_in long: source pixel floor(s) and weight floor(256 * frac(s)),
// clamped to the first and last pixel.  Returns pixel | weight << 16.
//
// floor(num / den) by a reciprocal estimate and one correction step each way
// (num < 2^28 and den < 2^15, so the estimate is off by at most one).
__device__ __forceinline__ int div_floor_small(int num, int den, int &rem)
{
    int q = (int)floorf((float)num * __builtin_amdgcn_rcpf((float)den));
    int r = num - q * den;
    if (r < 0) {
        --q;
        r += den;
    } else if (r >= den) {
        ++q;
        r -= den;
    }
    rem = r;
    return q;
}

__device__ __forceinline__ uint32_t pyr_tap(int x, int n_in, int n_out)
{
    const int num = (2 * x + 1) * n_in - n_out;
    if (num <= 0) return 0u;
    const int den = 2 * n_out;
    int r;
    int q = div_floor_small(num, den, r);
    int r2;
    int wq = div_floor_small(256 * r, den, r2);
    if (q >= n_in - 1) {
        q = n_in - 1;
        wq = 0;
    }
    return (uint32_t)q | ((uint32_t)wq << 16);
}

// LDS of one pyramid tile: kPyrRows + 1 staged level-0 rows, then per level
// the first output row, the row count and the row taps of the tile's rows.
constexpr int kPyrStage = (kPyrRows + 1) * kMaxPyrW;
constexpr int kPyrRowTaps = kPyrRows + 2;                   // output rows of one level in a tile (bound)
constexpr int kPyrMeta = kPyrStage;                         // int [kLevels][2]: first row, count
constexpr int kPyrRowTab = kPyrMeta + 2 * kLevels * 4;      // uint32 [kLevels][kPyrRowTaps]
constexpr int kPyrLds = kPyrRowTab + kLevels * kPyrRowTaps * 4;
static_assert((kLevels - 1) * kPyrRowTaps <= kWG, "one thread per row tap of levels 1..7");

// First output row y of a level h rows tall whose top tap row is at least Y
// (0 <= Y < H): the tap is floor(((2y + 1) H - h) / (2h)), and its clamp to
// H - 1 never takes it below Y, so y is the smallest with
// (2y + 1) H - h >= 2hY: ceil((2hY + h - H) / (2H)), and at least 0.
__device__ __forceinline__ int pyr_first_row(int Y, int H, int h)
{
    const int num = 2 * h * Y + h - H;
    if (num <= 0) return 0;
    return (num + 2 * H - 1) / (2 * H);
}

// One tile: image `side` (0 left, 1 right) of the frame, level-0 rows
// [Y0, Y0 + kPyrRows).  Stages those rows and the next in LDS, copies them to
// level 0 and writes every output row of levels 1..7 whose top tap row is
// among them: each source row is read from memory once and each output byte
// written once.  A thread owns output columns (of all levels in turn), takes
// the column's tap once and walks the tile's rows of that level; neighbouring
// threads write neighbouring bytes of a row.
__device__ __forceinline__ void ph_pyramid(const DevJob &J, int tile, unsigned char *smem)
{
    const int W = J.img_w, H = J.img_h, pitch = J.img_pitch;
    const int per = div_up(H, kPyrRows);
    const int side = tile / per;
    const FT_G uint8_t *src = side ? J.imgR : J.imgL;
    FT_G uint8_t *dst = side ? J.pyr_outR : J.pyr_outL;
    if (!src) return;
    const int Y0 = (tile - side * per) * kPyrRows;
    const int Y1 = min(Y0 + kPyrRows, H);
    const int ys = min(Y1 + 1, H);           // staged rows [Y0, ys)
    const int stride = (W + 3) & ~3;
    uint8_t *stage = smem;
    int *meta = reinterpret_cast<int *>(smem + kPyrMeta);          // first row | row count per level
    uint32_t *rtab = reinterpret_cast<uint32_t *>(smem + kPyrRowTab);
    const int tid = threadIdx.x;
    // one thread per (level, row) tap of the tile
    if (tid < (kLevels - 1) * kPyrRowTaps) {
        const int l = 1 + tid / kPyrRowTaps, r = tid - (l - 1) * kPyrRowTaps;
        const int hl = J.lv_h[l];
        const int ylo = pyr_first_row(Y0, H, hl);
        const int yhi = Y1 >= H ? hl : pyr_first_row(Y1, H, hl);
        const int n = min(yhi - ylo, kPyrRowTaps);   // at most ceil(kPyrRows * hl / H) + 1 rows
        if (r == 0) {
            meta[2 * l] = ylo;
            meta[2 * l + 1] = n;
        }
        if (r < n) rtab[l * kPyrRowTaps + r] = pyr_tap(ylo + r, H, hl);
    }
    // Stage the level-0 rows (4-byte loads when rows and base are aligned).
    // Element e of a row-major walk is row e / w, column e % w: one division
    // for the thread's first element, then steps of kWG elements.
    auto walk = [&](int w, int &r, int &c, int &dr, int &dc) {
        r = tid / w;
        c = tid - r * w;
        dr = kWG / w;
        dc = kWG - dr * w;
    };
    auto step = [&](int w, int &r, int &c, int dr, int dc) {
        r += dr;
        c += dc;
        if (c >= w) {
            c -= w;
            ++r;
        }
    };
    const bool al4 = ((reinterpret_cast<uintptr_t>(src) | (uintptr_t)pitch | (uintptr_t)W) & 3u) == 0;
    if (al4) {
        const int wq = W >> 2;
        int r, c, dr, dc;
        walk(wq, r, c, dr, dc);
        for (; r < ys - Y0; step(wq, r, c, dr, dc)) {
            const uint32_t v = *reinterpret_cast<const FT_G uint32_t *>(src + (size_t)(Y0 + r) * pitch + 4 * c);
            *reinterpret_cast<uint32_t *>(stage + r * stride + 4 * c) = v;
        }
    } else {
        int r, c, dr, dc;
        walk(W, r, c, dr, dc);
        for (; r < ys - Y0; step(W, r, c, dr, dc)) stage[r * stride + c] = src[(size_t)(Y0 + r) * pitch + c];
    }
    __syncthreads();
    // level 0: the staged rows [Y0, Y1)
    {
        FT_G uint8_t *d0 = dst + (size_t)Y0 * W;
        if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(dst) & 3u) == 0) {
            const int wq = W >> 2;
            int r, c, dr, dc;
            walk(wq, r, c, dr, dc);
            for (; r < Y1 - Y0; step(wq, r, c, dr, dc))
                *reinterpret_cast<FT_G uint32_t *>(d0 + (size_t)r * W + 4 * c) =
                    *reinterpret_cast<const uint32_t *>(stage + r * stride + 4 * c);
        } else {
            int r, c, dr, dc;
            walk(W, r, c, dr, dc);
            for (; r < Y1 - Y0; step(W, r, c, dr, dc)) d0[(size_t)r * W + c] = stage[r * stride + c];
        }
    }
    // levels 1..7: columns of the levels laid end to end, dealt over the threads
    int wsum[kLevels];
    int total = 0;
    _Pragma("unroll") for (int l = 1; l < kLevels; ++l)
    {
        wsum[l] = total;
        total += J.lv_w[l];
    }
    for (int e = tid; e < total; e += kWG) {
        int l = 1;
        _Pragma("unroll") for (int k = 2; k < kLevels; ++k) l = e >= wsum[k] ? k : l;
        const int x = e - wsum[l];
        const int wl = J.lv_w[l];
        const uint32_t c = pyr_tap(x, W, wl);
        // column x0 + 1 is read even where the tap is clamped to the last
        // column: its weight a is 0 there, and the byte read lies in LDS
        const int x0 = (int)(c & 0xFFFFu), a = (int)(c >> 16);
        const int ylo = meta[2 * l], n = meta[2 * l + 1];
        FT_G uint8_t *dcol = dst + J.lv_off[l] + (size_t)ylo * wl + x;
        const uint32_t *rt = rtab + l * kPyrRowTaps;
        for (int r = 0; r < n; ++r) {
            const uint32_t t = rt[r];
            const int y0 = (int)(t & 0xFFFFu), b = (int)(t >> 16);
            const uint8_t *r0 = stage + (y0 - Y0) * stride + x0;
            const uint8_t *r1 = stage + (min(y0 + 1, H - 1) - Y0) * stride + x0;
            // (256 - w) p + w q = 256 p + w (q - p), exactly
            const int p00 = r0[0], p10 = r1[0];
            const int top = (p00 << 8) + a * ((int)r0[1] - p00);
            const int bot = (p10 << 8) + a * ((int)r1[1] - p10);
            const int v = (top << 8) + b * (bot - top);
            dcol[(size_t)r * wl] = (uint8_t)((v + 32768) >> 16);
        }
    }
}

// ------------------------------------------------ setup: rows (pinhole)
// Row bin of a right keypoint (clamped; non-finite rows go to bin 0).
__device__ __forceinline__ int row_bin(float y, int rows)
{
    if (!(y >= 0.0f)) return 0;
    if (!(y < (float)rows)) return rows - 1;
    return (int)y;
}

// Packed rows [lo, hi] of the epipolar band of a right keypoint, or an empty
// range (lo > hi).
__device__ __forceinline__ uint32_t band_rows(const DevJob &J, float y, int oct)
{
    const float r = J.band * J.sf[lvl(oct)];
    const float flo = floorf(y - r);
    const float fhi = ceilf(y + r);
    if (!(fhi >= 0.0f) || !(flo <= (float)(J.rows - 1))) return 0xFFFFu;  // lo = 65535 > hi = 0
    const int lo = flo < 0.0f ? 0 : (int)flo;
    const int hi = fhi > (float)(J.rows - 1) ? J.rows - 1 : (int)fhi;
    return (uint32_t)lo | ((uint32_t)hi << 16);
}

template <int NT>
__device__ __forceinline__ void ph_rowsort(const DevJob &J, int *cnt, int *tmp)
{
    const int tid = threadIdx.x;
    const int rows = J.rows, nR = J.R.n, nb = J.n_lb * rows;
    const bool per_level = J.n_lb > 1;
    for (int r = tid; r < nb; r += NT) cnt[r] = 0;
    for (int j = tid; j < nR; j += NT) J.claimR[j] = 0xFFFFFFFFu;
    for (int i = tid; i < J.L.n; i += NT) J.flag[i] = 0;   // the refinement flags matches only
    if (tid == 0) J.counts[2] = 0;                          // length of the match list
    __syncthreads();
    // A chunk of kSortUnroll right keypoints per thread; the first chunk stays
    // in registers from the counting pass to the scatter.
    auto load = [&](int j0, float *x, float *y, int *oc) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int j = min(j0 + e * NT, nR - 1);
            x[e] = J.R.x[j];
            y[e] = J.R.y[j];
            oc[e] = J.R.oct[j];
        }
    };
    auto bin_of = [&](float y, int oc) { return (per_level ? lvl(oc) * rows : 0) + row_bin(y, rows); };
    auto count = [&](int j0, const float *y, const int *oc) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
            if (j0 + e * NT < nR) atomicAdd(&cnt[bin_of(y[e], oc[e])], 1);
    };
    auto scatter = [&](int j0, const float *x, const float *y, const int *oc) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int j = j0 + e * NT;
            if (j < nR) {
                const int pos = atomicAdd(&cnt[bin_of(y[e], oc[e])], 1);
                RowRec rec;
                rec.x = x[e];
                rec.band = band_rows(J, y[e], oc[e]);
                rec.meta = (uint32_t)oc[e] | ((uint32_t)j << 16);
                rec.pad = 0;
                J.rrec[pos] = rec;
            }
        }
    };
    float x0[kSortUnroll], y0[kSortUnroll];
    int oc0[kSortUnroll];
    if (tid < nR) {
        load(tid, x0, y0, oc0);
        count(tid, y0, oc0);
    }
    for (int j0 = tid + kSortUnroll * NT; j0 < nR; j0 += kSortUnroll * NT) {
        float x[kSortUnroll], y[kSortUnroll];
        int oc[kSortUnroll];
        load(j0, x, y, oc);
        count(j0, y, oc);
    }
    __syncthreads();
    const int total = wg_exclusive_scan<NT>(cnt, nb, tmp);
    // row_start[lb][r] = first record of (lb, r); row_start[lb][rows] = end of level bin lb
    for (int e = tid; e < J.n_lb * (rows + 1); e += NT) {
        const int lb = e / (rows + 1), r = e - lb * (rows + 1);
        const int bin = lb * rows + r;
        J.row_start[e] = bin < nb ? cnt[bin] : total;
    }
    __syncthreads();
    if (tid < nR) scatter(tid, x0, y0, oc0);
    for (int j0 = tid + kSortUnroll * NT; j0 < nR; j0 += kSortUnroll * NT) {
        float x[kSortUnroll], y[kSortUnroll];
        int oc[kSortUnroll];
        load(j0, x, y, oc);
        scatter(j0, x, y, oc);
    }
}

// ------------------------------------------- setup: overlap lists (fisheye)
template <int NT>
__device__ __forceinline__ int compact_range(const float *x, int n, float a, float b, int32_t *out, int *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int base = 0;
    for (int s = 0; s < n; s += NT) {
        const int i = s + tid;
        const bool p = i < n && x[i] >= a && x[i] <= b;
        const unsigned long long m = __ballot(p);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (p) out[off + rank] = i;
        int tot = 0;
        for (int w = 0; w < NT / 64; ++w) tot += wsum[w];
        __syncthreads();
        base += tot;
    }
    return base;
}

template <int NT>
__device__ __forceinline__ void ph_overlap(const DevJob &J, int *wsum)
{
    const int tid = threadIdx.x;
    for (int j = tid; j < J.R.n; j += NT) J.claimR[j] = 0xFFFFFFFFu;
    for (int i = tid; i < J.L.n; i += NT) J.flag[i] = 0;
    const int nQ = compact_range<NT>(J.L.x, J.L.n, J.ovl[0], J.ovl[1], J.qlist, wsum);
    const int nT = compact_range<NT>(J.R.x, J.R.n, J.ovr[0], J.ovr[1], J.tlist, wsum);
    // targets' descriptors in overlap order: one 16-byte half per thread step
    const uint4 *src = reinterpret_cast<const uint4 *>(J.R.desc);
    uint4 *dst = reinterpret_cast<uint4 *>(J.tdesc);
    for (int h = tid; h < 2 * nT; h += NT) dst[h] = src[2 * J.tlist[h >> 1] + (h & 1)];
    if (tid == 0) {
        J.counts[0] = nQ;
        J.counts[1] = nT;
        *J.o_nmatch = 0;
    }
}

// ------------------------------------------------ setup: keypoint grid
// Level bins of the cell index that hold a keypoint of octave o: the bins p
// whose octave window p - lv_lo .. p + lv_hi contains o, i.e. the predicted
// levels of the map points that may match it; one bin when the index is not
// binned.
__device__ __forceinline__ void cell_bins(const DevView &V, int o, int lv_lo, int lv_hi, int &p0, int &p1)
{
    if (V.n_pb == 1) {
        p0 = p1 = 0;
        return;
    }
    p0 = max(o - lv_hi, 0);
    p1 = min(o + lv_lo, kLevels - 1);
}

// Counting sort of the view's keypoints by (level bin, row, column) into
// 16-byte records; a keypoint is copied into every bin that holds its octave.
template <int NT>
__device__ __forceinline__ void ph_cellsort(const DevView &V, const DevKps &K, int lv_lo, int lv_hi, int *cnt,
                                            int *tmp)
{
    const int tid = threadIdx.x;
    const int cells = V.cols * V.rows;
    const int nb = V.n_pb * cells;
    for (int c = tid; c < nb; c += NT) cnt[c] = 0;
    for (int k = tid; k < K.n; k += NT) V.claim[k] = 0xFFFFFFFFu;
    for (int b = tid; b < kRotBinsMax; b += NT) V.hist[b] = 0;
    if (tid == 0) *V.n_matches = 0;
    __syncthreads();
    // A chunk of kSortUnroll keypoints per thread: the cell, position and
    // record meta of each (load), its counts (count) and its records (scatter).
    // The first chunk stays in registers from the counting pass to the scatter,
    // so a view of up to kSortUnroll * NT keypoints is read once.
    auto load = [&](int k0, int *cell, float *x, float *y, uint32_t *meta) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int k = min(k0 + e * NT, K.n - 1);
            x[e] = K.x[k];
            y[e] = K.y[k];
            const uint32_t pre = (V.preassigned && V.preassigned[k]) ? 1u : 0u;
            meta[e] = (uint32_t)K.oct[k] | (pre << 8) | ((uint32_t)k << 16);
        }
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int cx = cell_coord(x[e], V.min_x, V.inv_cw, V.cols);
            const int cy = cell_coord(y[e], V.min_y, V.inv_ch, V.rows);
            cell[e] = cy * V.cols + cx;
        }
    };
    auto count = [&](int k0, const int *cell, const uint32_t *meta) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            if (k0 + e * NT < K.n) {
                int p0, p1;
                cell_bins(V, (int)(meta[e] & 0xFFu), lv_lo, lv_hi, p0, p1);
                for (int p = p0; p <= p1; ++p) atomicAdd(&cnt[p * cells + cell[e]], 1);
            }
        }
    };
    auto scatter = [&](int k0, const int *cell, const float *x, const float *y, const uint32_t *meta) {
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            if (k0 + e * NT < K.n) {
                CellRec rec;
                rec.x = x[e];
                rec.y = y[e];
                rec.meta = meta[e];
                rec.pad = 0;
                int p0, p1;
                cell_bins(V, (int)(meta[e] & 0xFFu), lv_lo, lv_hi, p0, p1);
                for (int p = p0; p <= p1; ++p) V.crec[atomicAdd(&cnt[p * cells + cell[e]], 1)] = rec;
            }
        }
    };
    int cell0[kSortUnroll];
    float x0[kSortUnroll], y0[kSortUnroll];
    uint32_t meta0[kSortUnroll];
    if (tid < K.n) {
        load(tid, cell0, x0, y0, meta0);
        count(tid, cell0, meta0);
    }
    for (int k0 = tid + kSortUnroll * NT; k0 < K.n; k0 += kSortUnroll * NT) {
        int cell[kSortUnroll];
        float x[kSortUnroll], y[kSortUnroll];
        uint32_t meta[kSortUnroll];
        load(k0, cell, x, y, meta);
        count(k0, cell, meta);
    }
    __syncthreads();
    const int total = wg_exclusive_scan<NT>(cnt, nb, tmp);
    for (int c = tid; c < nb; c += NT) V.cell_off[c] = cnt[c];
    if (tid == 0) V.cell_off[nb] = total;
    __syncthreads();
    if (tid < K.n) scatter(tid, cell0, x0, y0, meta0);
    for (int k0 = tid + kSortUnroll * NT; k0 < K.n; k0 += kSortUnroll * NT) {
        int cell[kSortUnroll];
        float x[kSortUnroll], y[kSortUnroll];
        uint32_t meta[kSortUnroll];
        load(k0, cell, x, y, meta);
        scatter(k0, cell, x, y, meta);
    }
}

// ------------------------------------- stereo_a (pinhole): row-band best match
// Level bins of the row index a left keypoint of octave oi scans: the bins of
// octaves oi - level_window .. oi + level_window (clamped into the table;
// octaves above the last level share its bin), or the one bin of all levels.
__device__ __forceinline__ void level_bins(const DevJob &J, int oi, int &lb0, int &lb1)
{
    if (J.n_lb == 1) {
        lb0 = lb1 = 0;
        return;
    }
    lb0 = min(max(oi - J.level_window, 0), kLevels - 1);
    lb1 = min(max(oi + J.level_window, 0), kLevels - 1);
}

// G lanes per left keypoint.  The candidates of row r are the right keypoints
// whose band covers r; their integer rows lie within J.row_reach of r, so the
// lanes stream the row-sorted records of those bins and test the band exactly.
// Appends the wave's accepted pinhole matches to the frame's match list, one
// counter update per wave; the list order does not matter (the refinement
// writes by left keypoint).  Every lane of the wave calls it.
__device__ __forceinline__ void append_match(const DevJob &J, bool take, const MatchRec &r)
{
    const unsigned long long bal = __ballot(take);
    if (bal == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)bal) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&J.counts[2], (int)__popcll(bal));
    base = __shfl(base, leader);
    if (take) J.mrec[base + (int)__popcll(bal & ((1ull << lane) - 1ull))] = r;
}

__device__ __forceinline__ MatchRec match_rec(int i, uint32_t best, float bx, float x, float y, int oi)
{
    MatchRec r;
    r.i = i;
    r.j = (int)(best & 0xFFFFu);
    r.h = (int)(best >> 16);
    r.bx = bx;
    r.x = x;
    r.y = y;
    r.oct = oi;
    r.pad = 0;
    return r;
}

// Records [s, s + n) of level bin lb whose integer rows lie within that bin's
// reach of row.
__device__ __forceinline__ void bin_range(const DevJob &J, int lb, int row, int &s, int &n)
{
    const int reach = pick_level(J.lv_reach, lb);
    const FT_G int32_t *rs = J.row_start + lb * (J.rows + 1);
    s = rs[max(row - reach, 0)];
    n = rs[min(row + reach, J.rows - 1) + 1] - s;
}

template <int G>
__device__ __forceinline__ void ph_best(const DevJob &J, int tile)
{
    const int sub = threadIdx.x % G;
    const int i = tile * (kWG / G) + threadIdx.x / G;
    uint32_t best = 0xFFFFFFFFu;   // Hamming << 16 | right index
    float bx = 0.0f;               // x of that right keypoint (for the refinement)
    float x = 0.0f, y = 0.0f;
    int oi = 0;
    if (i < J.L.n) {
        y = J.L.y[i];
        x = J.L.x[i];
        oi = J.L.oct[i];
        const float minU = x - J.maxD;
        const float maxU = x - 0.0f;
        if (y > -1.0f && y < (float)J.rows && !(maxU < 0.0f)) {
            const int row = (int)y;
            const Desc di = load_desc(J.L.desc, i);
            int lb0, lb1;
            level_bins(J, oi, lb0, lb1);
            auto test = [&](const RowRec &rec) {
                const int lo = (int)(rec.band & 0xFFFFu), hi = (int)(rec.band >> 16);
                const int oj = (int)(rec.meta & 0xFFu);
                return row >= lo && row <= hi && oj >= oi - J.level_window && oj <= oi + J.level_window &&
                       rec.x >= minU && rec.x <= maxU;
            };
            auto push = [&](const RowRec &rec, const Desc &d) {
                const uint32_t key = ((uint32_t)hamming(di, d) << 16) | (rec.meta >> 16);
                if (key < best) {
                    best = key;
                    bx = rec.x;
                }
            };
            if (lb1 - lb0 < 3) {
                // Up to three bins: their ranges are read together, positions
                // 0 .. total - 1 run over them in order, lane `sub` taking every
                // G-th, kBestUnroll per step; a step's descriptors load together
                // with the next step's records.  (The minimum over distinct
                // keys does not depend on the order.)
                int s0, n0, s1 = 0, n1 = 0, s2 = 0, n2 = 0;
                bin_range(J, lb0, row, s0, n0);
                if (lb0 + 1 <= lb1) bin_range(J, lb0 + 1, row, s1, n1);
                if (lb0 + 2 <= lb1) bin_range(J, lb0 + 2, row, s2, n2);
                const int n01 = n0 + n1, total = n01 + n2;
                auto at = [&](int p) {
                    p = min(p, total - 1);   // past the end: a record loaded and never used
                    return J.rrec[p < n0 ? s0 + p : p < n01 ? s1 + (p - n0) : s2 + (p - n01)];
                };
                RowRec rec[kBestUnroll];
                if (total > 0) {
                    _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) rec[u] = at(sub + u * G);
                }
                for (int p0 = sub; p0 < total; p0 += kBestUnroll * G) {
                    bool cand[kBestUnroll];
                    Desc d[kBestUnroll];
                    _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u)
                    {
                        cand[u] = p0 + u * G < total && test(rec[u]);
                        if (cand[u]) d[u] = load_desc(J.R.desc, (int)(rec[u].meta >> 16));
                    }
                    RowRec nx[kBestUnroll];
                    _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) nx[u] = at(p0 + (kBestUnroll + u) * G);
                    _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) if (cand[u]) push(rec[u], d[u]);
                    _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) rec[u] = nx[u];
                }
            } else {
                // any number of bins, one after another
                for (int lb = lb0; lb <= lb1; ++lb) {
                    int s, n;
                    bin_range(J, lb, row, s, n);
                    const int p1 = s + n;
                    // kBestUnroll records per step are loaded together (indices
                    // clamped into the range, surplus entries masked); then the
                    // descriptors of the candidates among them.
                    for (int p0 = s + sub; p0 < p1; p0 += kBestUnroll * G) {
                        RowRec rec[kBestUnroll];
                        bool cand[kBestUnroll];
                        Desc d[kBestUnroll];
                        _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) rec[u] = J.rrec[min(p0 + u * G, p1 - 1)];
                        _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u)
                        {
                            cand[u] = p0 + u * G < p1 && test(rec[u]);
                            if (cand[u]) d[u] = load_desc(J.R.desc, (int)(rec[u].meta >> 16));
                        }
                        _Pragma("unroll") for (int u = 0; u < kBestUnroll; ++u) if (cand[u]) push(rec[u], d[u]);
                    }
                }
            }
        }
    }
    for (int m = 1; m < G; m <<= 1) {
        const uint32_t o = __shfl_xor(best, m);
        const float ox = __shfl_xor(bx, m);
        if (o < best) {
            best = o;
            bx = ox;
        }
    }
    const int h = (int)(best >> 16);
    const bool ok = best != 0xFFFFFFFFu && h < J.th_orb;
    if (sub == 0 && i < J.L.n) {
        J.best_j[i] = ok ? (int)(best & 0xFFFFu) : -1;
        J.best_h[i] = ok ? h : -1;
    }
    append_match(J, sub == 0 && i < J.L.n && ok, match_rec(i, best, bx, x, y, oi));
}

// Row-band scan of one pinhole left keypoint over staged (LDS) or global row
// records: lane `sub` of G takes every G-th record of the bins row +- reach;
// the candidates are collected first (kCandBatch at a time) and their
// row-ordered descriptors then read together (as in the wide search).
template <int G>
__device__ __forceinline__ void best_scan(const DevJob &J, const int *rs, const RowRec *rr, int row, int oi,
                                          float minU, float maxU, const Desc &di, int sub, uint32_t &best,
                                          float &bx)
{
    int lb0, lb1;
    level_bins(J, oi, lb0, lb1);
    int done = 0;
    for (;;) {
        int n = 0, seen = 0;
        int cp[kCandBatch];
        _Pragma("unroll") for (int e = 0; e < kCandBatch; ++e) cp[e] = 0;
        for (int lb = lb0; lb <= lb1; ++lb) {
        const int reach = pick_level(J.lv_reach, lb);
        const int *rsl = rs + lb * (J.rows + 1);
        const int b0 = max(row - reach, 0);
        const int b1 = min(row + reach, J.rows - 1);
        const int p1 = rsl[b1 + 1];
        for (int p = rsl[b0] + sub; p < p1; p += G) {
            const RowRec rec = rr[p];
            const int lo = (int)(rec.band & 0xFFFFu), hi = (int)(rec.band >> 16);
            const int oj = (int)(rec.meta & 0xFFu);
            if (row < lo || row > hi || oj < oi - J.level_window || oj > oi + J.level_window ||
                !(rec.x >= minU && rec.x <= maxU))
                continue;
            if (seen >= done && n < kCandBatch) {
                _Pragma("unroll") for (int e = 0; e < kCandBatch; ++e) if (n == e) cp[e] = p;
                ++n;
            }
            ++seen;
        }
        }
        Desc d[kCandBatch];
        _Pragma("unroll") for (int e = 0; e < kCandBatch; ++e)
        {
            if (e < n) d[e] = load_desc(J.R.desc, (int)(rr[cp[e]].meta >> 16));
        }
        _Pragma("unroll") for (int e = 0; e < kCandBatch; ++e)
        {
            if (e < n) {
                const RowRec rec = rr[cp[e]];
                const uint32_t key = ((uint32_t)hamming(di, d[e]) << 16) | (rec.meta >> 16);
                if (key < best) {
                    best = key;
                    bx = rec.x;
                }
            }
        }
        done += n;
        if (done >= seen) break;
    }
}

// ----------------------------- stereo_a (fisheye): all-pairs top-2 on MFMA
// H(a, b) = (256 - <a, b>) / 2 for the +-1 expansions of two descriptors.
// A workgroup owns 16 queries (one MFMA row block); its four waves take every
// fourth 16-target tile; partial top-2 lists are merged in LDS.  Each lane
// group g (lanes 16g..16g+15) supplies descriptor bytes 8g..8g+7 over the four
// K-steps of v_mfma_i32_16x16x64_i8 (two bytes = sixteen int8 per step); the A
// and B operands use the same byte-to-K assignment, so the dot product is the
// full 256-term sum whatever order the hardware sums K in.
// NT threads = NT / 256 independent subgroups of four waves; subgroup k of
// tile t owns queries (t * NT / 256 + k) * 16 ... + 15.  `part` holds 128
// words per subgroup.  Every thread reaches both barriers.
// Top-2 of 32-bit keys by value (keys are distinct: they carry the target
// index).  a <= b always holds, so the new second is the median of a, b and
// the key, one v_med3_u32; the new best is min(a, key).
__device__ __forceinline__ void top2_push(uint32_t &a, uint32_t &b, uint32_t key)
{
    uint32_t m;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(m) : "v"(a), "v"(b), "v"(key));
    b = m;
    a = min(a, key);
}

// +-1 bytes of 16 descriptor bits (two table entries per byte pair).
__device__ __forceinline__ v4i expand16(const uint64_t *tab, uint32_t word, int half)
{
    const uint64_t lo = tab[(word >> (16 * half)) & 0xFF];
    const uint64_t hi = tab[(word >> (16 * half + 8)) & 0xFF];
    return v4i{(int)(uint32_t)lo, (int)(uint32_t)(lo >> 32), (int)(uint32_t)hi, (int)(uint32_t)(hi >> 32)};
}

// Fisheye all-pairs top-2 on the matrix cores.  A workgroup subgroup (256
// threads) owns kKnnQueriesPerWG queries; its four waves split the target
// tiles.  Each wave holds the +-1 expansion of all its queries (QB blocks of
// 16) and expands every 16-target tile once for all QB blocks.
template <int NT>
__device__ __forceinline__ void ph_knn(const DevJob &J, int tile, uint64_t *tab, uint32_t *part)
{
    constexpr int QB = kKnnQueriesPerWG / 16;
    const int tid = threadIdx.x, ltid = tid & 255, sg = tid >> 8;
    // +-1 expansion of every byte value: bit t -> byte t, 1 -> +1, 0 -> -1
    if (tid < 256) {
        uint64_t e = 0;
        for (int t = 0; t < 8; ++t) e |= (uint64_t)(((tid >> t) & 1) ? 0x01u : 0xFFu) << (8 * t);
        tab[tid] = e;
    }
    __syncthreads();
    const int nQ = J.counts[0], nT = J.counts[1];
    const int q0 = (tile * (NT / 256) + sg) * kKnnQueriesPerWG;
    part += sg * (4 * kKnnQueriesPerWG * 2);
    const bool active = q0 < nQ && nT >= 2;   // uniform over the subgroup
    const int lane = ltid & 63, wave = ltid >> 6, g = lane >> 4, c = lane & 15;
    if (active) {
    v4i A[QB][4];
    _Pragma("unroll") for (int qb = 0; qb < QB; ++qb)
    {
        const int qa = q0 + 16 * qb + c;
        uint2 w = make_uint2(0, 0);
        if (qa < nQ) w = *reinterpret_cast<const uint2 *>(J.L.desc + 32 * (size_t)J.qlist[qa] + 8 * g);
        _Pragma("unroll") for (int s = 0; s < 4; ++s)
        {
            // the queries' signs are flipped (x ^ 0xFE negates a +-1 byte), so
            // the MFMA accumulates -dot
            const v4i e = expand16(tab, s < 2 ? w.x : w.y, s & 1);
            const int f = (int)0xFEFEFEFE;
            A[qb][s] = qa < nQ ? v4i{e[0] ^ f, e[1] ^ f, e[2] ^ f, e[3] ^ f} : v4i{0, 0, 0, 0};
        }
    }
    uint32_t ta[QB][4], tb[QB][4];
    _Pragma("unroll") for (int qb = 0; qb < QB; ++qb)
        _Pragma("unroll") for (int r = 0; r < 4; ++r) ta[qb][r] = tb[qb][r] = 0xFFFFFFFFu;
    // (wave-uniform, so that the loop below branches on scalars)
    const int n_tiles = __builtin_amdgcn_readfirstlane((nT + 15) >> 4);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // A ring of kKnnTilesInFlight target tiles' descriptor bytes per wave: the
    // loop is unrolled over the ring, and a slot is reloaded with the tile
    // kKnnTilesInFlight steps ahead as soon as its bytes are expanded, so that
    // several loads are in flight while the matrix cores work.
    constexpr int D = kKnnTilesInFlight;
    const uint8_t *tdesc = J.tdesc + 8 * g;
    uint2 ring[D];
    _Pragma("unroll") for (int d = 0; d < D; ++d)
    {
        const int tj = min(((wv + 4 * d) << 4) + c, nT - 1);
        ring[d] = *reinterpret_cast<const uint2 *>(tdesc + 32 * (size_t)tj);
    }
    // one tile: expand its bytes from ring slot d (then refill the slot with
    // the tile D steps ahead), run the MFMAs, push the column's keys
    auto step = [&](uint2 &slot, int t, bool refill) {
        const int tj = (t << 4) + c;
        const bool tv = tj < nT;
        // (a column past the end holds the last target's bytes: its sums are
        // computed and never pushed)
        v4i B[4];
        _Pragma("unroll") for (int s = 0; s < 4; ++s) B[s] = expand16(tab, s < 2 ? slot.x : slot.y, s & 1);
        if (refill) slot = *reinterpret_cast<const uint2 *>(tdesc + 32 * (size_t)min(tj + 64 * D, nT - 1));
        // acc[r] = -dot(query row 4g + r of block qb, target column c); the key
        // (256 - dot) << 15 | index = Hamming << 16 | index (dot = 256 - 2 H) is
        // kbase + (acc << 15), one shift-add.  The blocks' MFMA chains are
        // interleaved so that each hides the other's latency.
        const uint32_t kbase = (256u << 15) | (uint32_t)tj;
        v4i acc[QB];
        _Pragma("unroll") for (int qb = 0; qb < QB; ++qb) acc[qb] = v4i{0, 0, 0, 0};
        _Pragma("unroll") for (int s = 0; s < 4; ++s)
            _Pragma("unroll") for (int qb = 0; qb < QB; ++qb)
                acc[qb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qb][s], B[s], acc[qb], 0, 0, 0);
        if (tv) {
            _Pragma("unroll") for (int qb = 0; qb < QB; ++qb)
                _Pragma("unroll") for (int r = 0; r < 4; ++r)
                    top2_push(ta[qb][r], tb[qb][r], kbase + ((uint32_t)acc[qb][r] << 15));
        }
    };
    // whole turns of the ring (no exit inside, so the loads' waits stay
    // counted), then the last tiles with no refill
    int t0 = wv;
    for (; t0 + 4 * (D - 1) < n_tiles; t0 += 4 * D)
        _Pragma("unroll") for (int d = 0; d < D; ++d) step(ring[d], t0 + 4 * d, true);
    _Pragma("unroll") for (int d = 0; d < D - 1; ++d)
        if (t0 + 4 * d < n_tiles) step(ring[d], t0 + 4 * d, false);
    _Pragma("unroll") for (int qb = 0; qb < QB; ++qb)
    {
        _Pragma("unroll") for (int r = 0; r < 4; ++r)
        {
            Top2<uint32_t> t = {ta[qb][r], tb[qb][r]};
            _Pragma("unroll") for (int m = 1; m < 16; m <<= 1) t = top2_merge(t, __shfl_xor(t.a, m), __shfl_xor(t.b, m));
            if (c == 0) {
                uint32_t *pw = part + (wave * kKnnQueriesPerWG + 16 * qb + 4 * g + r) * 2;
                pw[0] = t.a;
                pw[1] = t.b;
            }
        }
    }
    }
    __syncthreads();
    if (active && ltid < kKnnQueriesPerWG && q0 + ltid < nQ) {
        Top2<uint32_t> t = {part[ltid * 2], part[ltid * 2 + 1]};
        for (int w = 1; w < 4; ++w)
            t = top2_merge(t, part[(w * kKnnQueriesPerWG + ltid) * 2], part[(w * kKnnQueriesPerWG + ltid) * 2 + 1]);
        const int i = J.qlist[q0 + ltid];
        J.best_j[i] = J.tlist[t.a & 0xFFFFu];
        J.best_h[i] = (int)(t.a >> 16);
        J.h2[i] = (int)(t.b >> 16);
    }
}

// ------------------------------------- stereo_b (pinhole): SAD refinement
// One wave per match.  The wave stages the left patch and the right strip of
// the left keypoint's level in LDS, then 64 lanes split the (shift, row) sums.
// General window sizes: one wave per match, lanes split the (shift, row) sums.
__device__ __forceinline__ void ph_refine_wave(const DevJob &J, int tile, uint8_t *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int idx = tile * kRefinePerWG + wave;   // position in the frame's match list
    const bool has = idx < J.counts[2];
    const MatchRec mr = J.mrec[min(idx, max(J.L.n - 1, 0))];   // loaded with the list length
    const int i = mr.i;
    const int w = J.half_win, L = J.half_range;
    const int side = 2 * w + 1, strip = 2 * (L + w) + 1, nS = 2 * L + 1;
    int j = -1, l = 0, su = 0, sv = 0, su0 = 0, Wl = 0, bh = 0;
    float xi = 0.0f, sfl = 0.0f;
    int64_t off = 0;
    bool act = false;
    if (has) {
        // everything the match needs is in its list record: one round of loads
        j = mr.j;
        bh = mr.h;
        const float xj = mr.bx;
        xi = mr.x;
        const float yi = mr.y;
        l = lvl(mr.oct);
        const float s = pick_level(J.inv_sf, l);
        sfl = pick_level(J.sf, l);
        su = (int)roundf(xi * s);
        sv = (int)roundf(yi * s);
        su0 = (int)roundf(xj * s);
        Wl = pick_level(J.lv_w, l);
        const int Hl = pick_level(J.lv_h, l);
        off = pick_level(J.lv_off, l);
        act = su - w >= 0 && su + w < Wl && sv - w >= 0 && sv + w < Hl && su0 - L - w >= 0 &&
              su0 + L + w < Wl;
    }
    uint8_t *P = lds + wave * kRefineLds;          // left patch [side][side]
    uint8_t *S = P + side * side;                  // right strip [side][strip]
    if (act) {
        const uint8_t *IL = J.pyrL + off;
        const uint8_t *IR = J.pyrR + off;
        const int nP = side * side, n = nP + side * strip;
        for (int e = lane; e < n; e += 64) {
            if (e < nP) {
                const int r = e / side, c = e - r * side;
                P[e] = IL[(size_t)(sv - w + r) * Wl + su - w + c];
            } else {
                const int e2 = e - nP, r = e2 / strip, c = e2 - r * strip;
                P[e] = IR[(size_t)(sv - w + r) * Wl + su0 - L - w + c];
            }
        }
    }
    __syncthreads();
    const int parts = 64 / nS;
    const int k_idx = lane / parts, part = lane - k_idx * parts;
    int acc = 0;
    if (act && k_idx < nS) {
        const int cL = P[w * side + w];
        const int cR = S[w * strip + k_idx + w];
        for (int r = part; r < side; r += parts) {
            const uint8_t *pl = P + r * side;
            const uint8_t *pr = S + r * strip + k_idx;
            for (int dx = 0; dx < side; ++dx) acc += abs(((int)pl[dx] - cL) - ((int)pr[dx] - cR));
        }
    }
    int tot = acc;
    for (int p = 1; p < parts; ++p) tot += __shfl(acc, min(lane + p, 63));
    // every lane takes part in the shuffles; ties go to the smaller shift
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
    if (lane != 0 || !has) return;
    if (!act || kb == -L || kb == L) {
        J.flag[i] = 0;
        return;
    }
    const int c = best;
    const float num = (float)(a - e);
    const float den = (float)(2 * (a + e - 2 * c));
    const float delta = num / den;
    if (delta < -1.0f || delta > 1.0f) {
        J.flag[i] = 0;
        return;
    }
    float uR = sfl * (((float)su0 + (float)kb) + delta);
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
    atomicMin(&J.claimR[j], ((uint32_t)bh << 23) | (uint32_t)i);
}

// The usual 11x11 window and +-5 shifts: four matches per wave, sixteen lanes
// each; lane k of a match stages its share of the windows and computes SAD of
// shift k - 5 alone, so the argmin is a 16-lane shuffle reduction.  A quarter
// of the waves of the general path, the same dependent round trips.
__device__ __forceinline__ void ph_refine_quarter(const DevJob &J, int tile, uint8_t *lds)
{
    constexpr int w = 5, L = 5, side = 2 * w + 1, strip = 2 * (L + w) + 1, nS = 2 * L + 1;
    static_assert(side == 11 && strip == 21, "the row staging reads 11-byte patch and 21-byte strip rows");
    static_assert((side * 12 + side * 24) * 2 <= kRefineQLds, "refine windows");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ql = lane & 15, slot = wave * 4 + (lane >> 4);
    const int idx = tile * kRefineQPerWG + slot;   // position in the frame's match list
    const bool has = idx < J.counts[2];
    const MatchRec mr = J.mrec[min(idx, max(J.L.n - 1, 0))];   // loaded with the list length
    const int i = mr.i;
    int j = -1, l = 0, su = 0, sv = 0, su0 = 0, Wl = 0, bh = 0;
    float xi = 0.0f, sfl = 0.0f;
    int64_t off = 0;
    bool act = false;
    if (has) {
        // everything the match needs is in its list record: one round of loads
        j = mr.j;
        bh = mr.h;
        const float xj = mr.bx;
        xi = mr.x;
        const float yi = mr.y;
        l = lvl(mr.oct);
        const float s = pick_level(J.inv_sf, l);
        sfl = pick_level(J.sf, l);
        su = (int)roundf(xi * s);
        sv = (int)roundf(yi * s);
        su0 = (int)roundf(xj * s);
        Wl = pick_level(J.lv_w, l);
        const int Hl = pick_level(J.lv_h, l);
        off = pick_level(J.lv_off, l);
        act = su - w >= 0 && su + w < Wl && sv - w >= 0 && sv + w < Hl && su0 - L - w >= 0 &&
              su0 + L + w < Wl;
    }
    // Windows in LDS as 16-bit values, rows padded to whole dwords: the left
    // patch holds P + 255, the right strip holds S.  For shift k (lane k) the
    // centre-subtracted difference |(P - cL) - (S - cR)| equals
    // |(P + 255) - (S + off)| with off = cL - cR + 255 in [0, 510]; both
    // terms lie in [0, 765], so v_sad_u16 sums two pixels per instruction.
    constexpr int pS = 12, sS = 24;   // row strides (u16) of patch and strip
    uint16_t *P = reinterpret_cast<uint16_t *>(lds + slot * kRefineQLds);
    uint16_t *S = P + side * pS;
    if (act) {
        // 22 row jobs per match (the patch's 11 rows, then the strip's), two
        // per lane: each row read whole (unaligned dword loads covering exactly
        // its 11 or 21 bytes) and widened to 16-bit pairs by byte permutes
        const uint8_t *IL = J.pyrL + off;
        const uint8_t *IR = J.pyrR + off;
        constexpr uint32_t kLo = 0x0C010C00u, kHi = 0x0C030C02u;   // bytes 0,1 / 2,3 -> u16 pair
        _Pragma("unroll") for (int h = 0; h < 2; ++h)
        {
            const int jb = ql + 16 * h;
            if (jb < side) {
                const uint8_t *src = IL + (size_t)(sv - w + jb) * Wl + su - w;
                uint32_t d0, d1;
                uint16_t d2;
                __builtin_memcpy(&d0, src, 4);
                __builtin_memcpy(&d1, src + 4, 4);
                __builtin_memcpy(&d2, src + 8, 2);
                const uint32_t d3 = src[10];
                uint32_t *row = reinterpret_cast<uint32_t *>(P + jb * pS);
                constexpr uint32_t k255 = 0x00FF00FFu;
                row[0] = __builtin_amdgcn_perm(0u, d0, kLo) + k255;
                row[1] = __builtin_amdgcn_perm(0u, d0, kHi) + k255;
                row[2] = __builtin_amdgcn_perm(0u, d1, kLo) + k255;
                row[3] = __builtin_amdgcn_perm(0u, d1, kHi) + k255;
                row[4] = __builtin_amdgcn_perm(0u, (uint32_t)d2, kLo) + k255;
                row[5] = d3 + 255u;   // column 11 is padding
            } else if (jb < 2 * side) {
                const int r = jb - side;
                const uint8_t *src = IR + (size_t)(sv - w + r) * Wl + su0 - L - w;
                uint32_t d[5];
                _Pragma("unroll") for (int k = 0; k < 5; ++k) __builtin_memcpy(&d[k], src + 4 * k, 4);
                const uint32_t d5 = src[20];
                uint32_t *row = reinterpret_cast<uint32_t *>(S + r * sS);
                _Pragma("unroll") for (int k = 0; k < 5; ++k)
                {
                    row[2 * k] = __builtin_amdgcn_perm(0u, d[k], kLo);
                    row[2 * k + 1] = __builtin_amdgcn_perm(0u, d[k], kHi);
                }
                row[10] = d5;
            }
        }
    }
    __syncthreads();
    int sad = 0;
    uint32_t key = 0xFFFFFFFFu;   // SAD << 4 | lane: ties go to the smaller shift
    if (act && ql < nS) {
        const int cL = (int)P[w * pS + w] - 255;
        const int cR = S[w * sS + ql + w];
        const uint32_t off1 = (uint32_t)(cL - cR + 255);
        const uint32_t off2 = off1 | (off1 << 16);
        const int b0 = ql & ~1;                   // first u16 of the strip pairs read
        const uint32_t sh = (uint32_t)(ql & 1) * 2;   // byte shift realigning them to pixel ql
        uint32_t acc = 0;
        _Pragma("unroll 1") for (int r = 0; r < side; ++r)
        {
            const uint32_t *pa = reinterpret_cast<const uint32_t *>(P + r * pS);
            const uint32_t *pb = reinterpret_cast<const uint32_t *>(S + r * sS + b0);
            uint32_t db[6];
            _Pragma("unroll") for (int t = 0; t < 6; ++t) db[t] = pb[t];
            _Pragma("unroll") for (int t = 0; t < 5; ++t)
                acc = __builtin_amdgcn_sad_u16(pa[t], __builtin_amdgcn_alignbyte(db[t + 1], db[t], sh) + off2, acc);
            const int d10 = (int)P[r * pS + 10] - ((int)S[r * sS + ql + 10] + (int)off1);
            acc += (uint32_t)abs(d10);
        }
        sad = (int)acc;
        key = ((uint32_t)sad << 4) | (uint32_t)ql;
    }
    for (int m = 8; m >= 1; m >>= 1) {
        const uint32_t o = __shfl_xor(key, m);
        key = o < key ? o : key;
    }
    const int kb = (int)(key & 15u) - L;
    const int base = lane & ~15;
    const int a = __shfl(sad, base + max(kb + L - 1, 0));
    const int e = __shfl(sad, base + min(kb + L + 1, nS - 1));
    if (ql != 0 || !has) return;
    if (!act || kb == -L || kb == L) {
        J.flag[i] = 0;
        return;
    }
    const int c = (int)(key >> 4);
    const float num = (float)(a - e);
    const float den = (float)(2 * (a + e - 2 * c));
    const float delta = num / den;
    if (delta < -1.0f || delta > 1.0f) {
        J.flag[i] = 0;
        return;
    }
    float uR = sfl * (((float)su0 + (float)kb) + delta);
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
    atomicMin(&J.claimR[j], ((uint32_t)bh << 23) | (uint32_t)i);
}

__device__ __forceinline__ void ph_refine(const DevJob &J, int tile, uint8_t *lds)
{
    if (refine_quarter(J)) ph_refine_quarter(J, tile, lds);
    else ph_refine_wave(J, tile, lds);
}

// ------------------------------- stereo_b (fisheye): ratio + triangulation
__device__ __forceinline__ double kb_distort(const float *kb, double th)
{
    const double k1 = kb[4], k2 = kb[5], k3 = kb[6], k4 = kb[7];
    const double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
    return th * ((((1.0 + k1 * t2) + k2 * t4) + k3 * t6) + k4 * t8);
}

__device__ __forceinline__ void kb_project(const float *kb, const double X[3], double uv[2])
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

__device__ __forceinline__ bool kb_unproject(const float *kb, float u, float v, int iters, double tol,
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

__device__ __forceinline__ double det3(const double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// Linear least-squares triangulation with the homogeneous coordinate fixed to
// one; 3x3 normal equations solved by Cramer's rule (float64).
__device__ __forceinline__ bool triangulate(const double r1[3], const double r2[3], const float *R_lr,
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

__device__ __forceinline__ void ph_tri(const DevJob &J, int tile)
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
// The median is the value at rank n/2 of the survivors' 16-bit SADs, found by
// a two-pass 8-bit radix select with a parallel prefix over the 256 bins.
template <int NT>
__device__ __forceinline__ int select_bin(int *hist, int *tmp, int target, int *out_rank, int *found)
{
    const int tid = threadIdx.x;
    const int h = tid < 256 ? hist[tid] : 0;
    wg_exclusive_scan<NT>(hist, 256, tmp);   // hist now holds exclusive prefixes
    if (tid < 256 && h > 0 && hist[tid] <= target && target < hist[tid] + h) {
        found[0] = tid;
        found[1] = target - hist[tid];
    }
    __syncthreads();
    *out_rank = found[1];
    const int b = found[0];
    __syncthreads();
    return b;
}

__device__ __forceinline__ bool bit(const uint32_t *b, int i) { return (b[i >> 5] >> (i & 31)) & 1u; }

template <int NT>
__device__ __forceinline__ void ph_median(const DevJob &J, int *hist, int *tmp, uint32_t *surv, int *sh)
{
    const int tid = threadIdx.x, nL = J.L.n;
    // Up to kSortUnroll * NT keypoints, every field a thread needs stays in
    // its registers from the first pass to the outputs; larger frames re-read.
    const bool held = nL <= kSortUnroll * NT;
    if (tid < 256) hist[tid] = 0;
    if (tid == 0) sh[0] = 0;
    for (int w = tid; w < (nL + 31) / 32; w += NT) surv[w] = 0;
    __syncthreads();
    int my_n = 0;
    int bj[kSortUnroll], bh[kSortUnroll], sd[kSortUnroll];
    float ur[kSortUnroll], dp[kSortUnroll];
    bool sv[kSortUnroll] = {};
    for (int i0 = tid; i0 < nL; i0 += kSortUnroll * NT) {
        int fl[kSortUnroll];
        uint32_t cl[kSortUnroll];
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int i = min(i0 + e * NT, nL - 1);
            fl[e] = J.flag[i];
            bj[e] = J.best_j[i];
            bh[e] = J.best_h[i];
            sd[e] = J.sad[i];
            ur[e] = J.uR[i];
            dp[e] = J.depth[i];
        }
        // a flagged keypoint has a valid right index; others read index 0
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e) cl[e] = J.claimR[fl[e] ? bj[e] : 0];
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int i = i0 + e * NT;
            sv[e] = i < nL && fl[e] && cl[e] == (((uint32_t)bh[e] << 23) | (uint32_t)i);
            if (sv[e]) {
                atomicOr(&surv[i >> 5], 1u << (i & 31));
                ++my_n;
                atomicAdd(&hist[(sd[e] >> 8) & 0xFF], 1);
            }
        }
    }
    atomicAdd(&sh[0], my_n);
    __syncthreads();
    const int n = sh[0];
    int m = 0;
    if (n > 0) {
        int rank;
        const int hb = select_bin<NT>(hist, tmp, n / 2, &rank, sh + 2);
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
        if (held) {
            _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
                if (tid + e * NT < nL && sv[e] && ((sd[e] >> 8) & 0xFF) == hb) atomicAdd(&hist[sd[e] & 0xFF], 1);
        } else {
            for (int i = tid; i < nL; i += NT)
                if (bit(surv, i) && ((J.sad[i] >> 8) & 0xFF) == hb) atomicAdd(&hist[J.sad[i] & 0xFF], 1);
        }
        __syncthreads();
        int rank2;
        const int lb = select_bin<NT>(hist, tmp, rank, &rank2, sh + 2);
        m = (hb << 8) | lb;
    }
    if (tid == 0) sh[1] = 0;
    __syncthreads();
    int kept = 0;
    for (int i0 = tid; i0 < nL; i0 += kSortUnroll * NT) {
        if (!held) {
            _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
            {
                const int i = min(i0 + e * NT, nL - 1);
                bj[e] = J.best_j[i];
                bh[e] = J.best_h[i];
                sd[e] = J.sad[i];
                ur[e] = J.uR[i];
                dp[e] = J.depth[i];
                sv[e] = bit(surv, i);
            }
        }
        _Pragma("unroll") for (int e = 0; e < kSortUnroll; ++e)
        {
            const int i = i0 + e * NT;
            if (i >= nL) continue;
            const bool keep = sv[e] && (long long)J.med_den * sd[e] < (long long)J.med_num * m;
            J.o_right_idx[i] = keep ? bj[e] : -1;
            J.o_dist[i] = keep ? bh[e] : -1;
            J.o_uR[i] = keep ? ur[e] : -1.0f;
            J.o_depth[i] = keep ? dp[e] : -1.0f;
            J.o_sad[i] = keep ? sd[e] : -1;
            kept += keep ? 1 : 0;
        }
    }
    atomicAdd(&sh[1], kept);
    __syncthreads();
    if (tid == 0) *J.o_nmatch = sh[1];
}

// ---------------------- stereo_c (fisheye): conflicts + outputs
template <int NT>
__device__ __forceinline__ void ph_fish_final(const DevJob &J, int tile)
{
    const int i = tile * NT + threadIdx.x;
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
// G lanes per map point.  Every lane of the group evaluates the projection and
// the visibility tests (identical results), then the group streams the
// cell-sorted records of the window's cells (one cell of margin on each side
// covers the rounding of the cell arithmetic) and merges its top-2 lists.
// Keys order candidates by (distance, keypoint index): distance << 40 |
// index << 8 | level.
// What one map point looks for in one view: its projection, the search
// window (radius, levels, cells) and its descriptor.
struct Query {
    bool vis;
    bool gate;          // stereo right-coordinate gate applies
    float u, v, Rm, uR;
    int cx0, cx1, cy0, cy1, plo, phi;
    int cb;             // first cell offset of the level bin of the predicted level
    Desc dm;
};

__device__ __forceinline__ Query make_query(const DevJob &J, const DevView &V, int m)
{
    Query q;
    // every field of the map point record is issued up front (one round trip)
    const float X = J.pos[3 * m], Y = J.pos[3 * m + 1], Z = J.pos[3 * m + 2];
    const float nx = J.normal[3 * m], ny = J.normal[3 * m + 1], nz = J.normal[3 * m + 2];
    const float dmin = J.dmin[m], dmax = J.dmax[m];
    q.dm = load_desc(J.mdesc, m);
    const float xc = ((V.R[0] * X + V.R[1] * Y) + V.R[2] * Z) + V.t[0];
    const float yc = ((V.R[3] * X + V.R[4] * Y) + V.R[5] * Z) + V.t[1];
    const float zc = ((V.R[6] * X + V.R[7] * Y) + V.R[8] * Z) + V.t[2];
    float u = 0.0f, v = 0.0f;
    bool vis = false;
    if (zc > 0.0f) {
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
        vis = u >= V.min_x && u <= V.max_x && v >= V.min_y && v <= V.max_y;
    }
    const float pox = X - V.O[0], poy = Y - V.O[1], poz = Z - V.O[2];
    const float dist = sqrtf((pox * pox + poy * poy) + poz * poz);
    vis = vis && dist >= J.dist_lo * dmin && dist <= J.dist_hi * dmax;
    const float vcos = ((pox * nx + poy * ny) + poz * nz) / dist;
    q.vis = vis && vcos >= J.cos_lim;
    q.u = u;
    q.v = v;
    if (!q.vis) return q;
    const float ratio = dmax / dist;
    int pred = kLevels - 1;
    for (int l = 0; l < kLevels; ++l)
        if (J.sf[l] >= ratio) {
            pred = l;
            break;
        }
    const float rbase = (vcos > J.cos_narrow ? J.r_narrow : J.r_wide) * J.th;
    q.Rm = rbase * J.sf[pred];
    q.gate = V.u_right != nullptr;
    q.uR = q.gate ? u - V.bf * (1.0f / zc) : 0.0f;
    // A candidate has |x - u| < Rm up to one rounding of the subtraction, so x
    // lies within Rm + 0.01 px of u; cell_coord is monotone, so the cells of
    // u -+ (Rm + 0.01) bracket the cells of every candidate.
    const float Rc = q.Rm + 0.01f;
    q.cx0 = cell_coord(u - Rc, V.min_x, V.inv_cw, V.cols);
    q.cx1 = cell_coord(u + Rc, V.min_x, V.inv_cw, V.cols);
    q.cy0 = cell_coord(v - Rc, V.min_y, V.inv_ch, V.rows);
    q.cy1 = cell_coord(v + Rc, V.min_y, V.inv_ch, V.rows);
    q.plo = pred - J.lv_lo;
    q.phi = pred + J.lv_hi;
    q.cb = (V.n_pb > 1 ? pred : 0) * (V.cols * V.rows);
    return q;
}

// A keypoint record (level, position) is a candidate of the query, before the
// stereo gate.
__device__ __forceinline__ bool in_window(const Query &q, float x, float y, uint32_t meta)
{
    const int ok = (int)(meta & 0xFFu);
    return ok >= q.plo && ok <= q.phi && fabsf(x - q.u) < q.Rm && fabsf(y - q.v) < q.Rm && !(meta & 0x100u);
}

__device__ __forceinline__ bool gate_rejects(const Query &q, float ur)
{
    return q.gate && ur > 0.0f && !(fabsf(q.uR - ur) <= q.Rm);
}

__device__ __forceinline__ uint64_t cand_key(int h, uint32_t meta)
{
    return ((uint64_t)h << 40) | ((uint64_t)(meta >> 16) << 8) | (uint64_t)(meta & 0xFFu);
}

// Scan of the window over the sorted records in global memory; lane `sub` of
// G takes every G-th record.  One record range per window row; the next row's
// bounds are loaded before the current row is scanned, and kSearchUnroll
// records are loaded together (indices clamped into the range, surplus
// entries masked), then the descriptors of the candidates among them.
template <int G>
__device__ __forceinline__ Top2<uint64_t> scan_global(const DevView &V, const Query &q, int sub)
{
    Top2<uint64_t> top = {~0ull, ~0ull};
    const FT_G int32_t *off = V.cell_off + q.cb;
    int c0 = off[q.cy0 * V.cols + q.cx0];
    int c1 = off[q.cy0 * V.cols + q.cx1 + 1];
    for (int cy = q.cy0; cy <= q.cy1; ++cy) {
        int n0 = 0, n1 = 0;
        if (cy < q.cy1) {
            n0 = off[(cy + 1) * V.cols + q.cx0];
            n1 = off[(cy + 1) * V.cols + q.cx1 + 1];
        }
        for (int p0 = c0 + sub; p0 < c1; p0 += kSearchUnroll * G) {
            CellRec rec[kSearchUnroll];
            bool cand[kSearchUnroll];
            Desc d[kSearchUnroll];
            float ur[kSearchUnroll];
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e) rec[e] = V.crec[min(p0 + e * G, c1 - 1)];
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e)
            {
                cand[e] = p0 + e * G < c1 && in_window(q, rec[e].x, rec[e].y, rec[e].meta);
                ur[e] = 0.0f;
                if (cand[e]) {
                    d[e] = load_desc(V.kdesc, (int)(rec[e].meta >> 16));
                    if (q.gate) ur[e] = V.u_right[rec[e].meta >> 16];
                }
            }
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e)
            {
                if (cand[e] && !gate_rejects(q, ur[e]))
                    top = top2_insert(top, cand_key(hamming(q.dm, d[e]), rec[e].meta));
            }
        }
        c0 = n0;
        c1 = n1;
    }
    return top;
}

// Merge of the G lanes' lists, acceptance, outputs and the claim on the
// matched keypoint.  Every lane of the wave calls it (shuffles).
template <int G>
__device__ __forceinline__ void finish_query(const DevJob &J, const DevView &V, int m, int sub,
                                             Top2<uint64_t> top)
{
    for (int o = 1; o < G; o <<= 1) top = top2_merge(top, shfl_xor64(top.a, o), shfl_xor64(top.b, o));
    if (sub != 0 || m >= J.nM) return;
    const uint64_t k1 = top.a, k2 = top.b;
    int kk1 = -1, b1 = -1;
    if (k1 != ~0ull) {
        const int h1 = (int)(k1 >> 40), l1 = (int)(k1 & 0xFFu);
        const int h2 = k2 != ~0ull ? (int)(k2 >> 40) : 256;
        const int l2 = k2 != ~0ull ? (int)(k2 & 0xFFu) : -1;
        const bool fails = J.s_ratio_den * h1 > J.s_ratio_num * h2;
        if (h1 <= J.th_high && !(J.same_level_only ? (l1 == l2 && fails) : fails)) {
            kk1 = (int)((k1 >> 8) & 0xFFFFu);
            b1 = h1;
        }
    }
    V.mp_k[m] = kk1;
    V.mp_h[m] = b1;
    if (kk1 >= 0) atomicMin(&V.claim[kk1], ((uint32_t)b1 << 23) | (uint32_t)m);
}

// Candidate keys of the record-dealt search are 32 bits: distance (9 bits),
// keypoint (16), level (4; octaves are 0..7 by contract), in the same order as
// cand_key; each map point's best two keys are kept in LDS by atomic minima: a
// key goes to the best slot, and whichever of it and the displaced best is
// larger goes to the second slot, which leaves the two smallest distinct keys.
__device__ __forceinline__ uint64_t key32_to_64(uint32_t k)
{
    if (k == 0xFFFFFFFFu) return ~0ull;
    return ((uint64_t)(k >> 20) << 40) | ((uint64_t)((k >> 4) & 0xFFFFu) << 8) | (uint64_t)(k & 15u);
}

// Orders one wave's LDS accesses (its lanes read what other lanes wrote); the
// record-dealt search syncs only within a wave, whose chunk and round counts
// are wave-uniform but may differ between the waves of a workgroup.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Record-dealt search (one lane per map point).  Every lane projects its map
// point and loads the record ranges of up to kDealRows window rows at once;
// the wave then lays the records of all 64 windows end to end and deals them
// out in rounds of 64 * kDealRecs positions, lane d taking positions d, d + 64,
// d + 128, ..., so every lane issues all its record loads together whatever
// the window sizes and each load instruction reads 64 consecutive positions.
// Records that pass the window test become candidates in one wave-wide list,
// which is again dealt evenly for the descriptor reads; each map point's best
// two keys are kept in LDS by 32-bit atomic minima.
constexpr int kDealRows = 4;    // window rows per lane and chunk
constexpr int kDealRecs = 4;    // records per lane and round
constexpr int kDealFlush = 1;   // candidates per lane and descriptor batch
constexpr int kDealQp = 0;                                // float4 u, v, Rm, level window [64]
constexpr int kDealUr = kDealQp + 64 * 16;                // float uR [64]
constexpr int kDealQd = kDealUr + 64 * 4;                 // Desc [64]
constexpr int kDealTb = kDealQd + 64 * 32;                // best [64], second [64]
constexpr int kDealSeg = kDealTb + 128 * 4;               // record offset of each segment [64][kDealRows]
constexpr int kDealCands = kDealSeg + 64 * kDealRows * 4;  // candidate list [64 * kDealRecs], or the round's marks
constexpr int kDealLdsPerWave = kDealCands + 64 * kDealRecs * 4;

// The wave takes map points m0 .. m0 + 63 of the view; `base` is its LDS.
__device__ __forceinline__ void ph_search_deal(const DevJob &J, const DevView &V, int m0, unsigned char *base)
{
    const int lane = threadIdx.x & 63;
    const int m = m0 + lane;
    float4 *qp = reinterpret_cast<float4 *>(base + kDealQp);
    float *quR = reinterpret_cast<float *>(base + kDealUr);
    Desc *qd = reinterpret_cast<Desc *>(base + kDealQd);
    uint32_t *tb = reinterpret_cast<uint32_t *>(base + kDealTb);
    uint32_t *seg = reinterpret_cast<uint32_t *>(base + kDealSeg);
    uint32_t *cl = reinterpret_cast<uint32_t *>(base + kDealCands);
    uint32_t *mark = cl;

    Query q;
    q.vis = false;
    if (m < J.nM) q = make_query(J, V, m);
    const int cx0 = q.vis ? q.cx0 : 0, cx1 = q.vis ? q.cx1 : 0;
    const int cy0 = q.vis ? q.cy0 : 0, cy1 = q.vis ? q.cy1 : -1;
    const FT_G int32_t *off = V.cell_off + (q.vis ? q.cb : 0);
    const int lv = q.vis ? ((q.plo + 16) | ((q.phi + 16) << 8)) : (16 | (15 << 8));
    qp[lane] = make_float4(q.u, q.v, q.vis ? q.Rm : 0.0f, __int_as_float(lv));
    quR[lane] = q.vis ? q.uR : 0.0f;
    qd[lane] = q.dm;
    tb[lane] = 0xFFFFFFFFu;
    tb[64 + lane] = 0xFFFFFFFFu;
    const bool gate = V.u_right != nullptr;
    const int chunks = wave_last(wave_inclusive_max((cy1 - cy0 + kDealRows) / kDealRows));
    for (int ch = 0; ch < chunks; ++ch) {
        // record ranges of this lane's rows of the chunk: one round of loads
        const int r0 = cy0 + ch * kDealRows;
        int sa[kDealRows], sn[kDealRows];
        int mine = 0;
        _Pragma("unroll") for (int e = 0; e < kDealRows; ++e)
        {
            const bool in = r0 + e <= cy1;
            const int row = in ? r0 + e : 0;
            sa[e] = off[row * V.cols + cx0];
            const int b = off[row * V.cols + cx1 + 1];
            sn[e] = in ? b - sa[e] : 0;
            mine += sn[e];
        }
        const int incl = wave_inclusive_scan(mine);
        const int total = wave_last(incl);
        // the records of all segments (lane, row) end to end: a segment's first
        // position in the chunk, and the offset from a position to its record
        int st[kDealRows];
        st[0] = incl - mine;
        _Pragma("unroll") for (int e = 1; e < kDealRows; ++e) st[e] = st[e - 1] + sn[e - 1];
        wave_lds_sync();   // the previous chunk's readers are done with seg
        _Pragma("unroll") for (int e = 0; e < kDealRows; ++e) seg[lane * kDealRows + e] = (uint32_t)(sa[e] - st[e]);
        for (int g_lo = 0; g_lo < total; g_lo += 64 * kDealRecs) {
            const int cnt = min(total - g_lo, 64 * kDealRecs);
            // Position g_lo + 64k + d of the chunk goes to lane d.  Each
            // non-empty segment writes its id + 1 at its first position of the
            // round (position 0 for the one begun in an earlier round); no two
            // segments share a position and ids grow with positions, so the
            // prefix maximum over positions names every position's segment.
            // The marks use the candidate list's memory.
            *reinterpret_cast<uint4 *>(mark + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
            wave_lds_sync();
            _Pragma("unroll") for (int e = 0; e < kDealRows; ++e)
            {
                const int A = st[e] - g_lo;
                if (sn[e] > 0 && A < cnt && A + sn[e] > 0) mark[max(A, 0)] = (uint32_t)(lane * kDealRows + e + 1);
            }
            wave_lds_sync();
            int own[kDealRecs];
            int carry = 0;
            _Pragma("unroll") for (int k = 0; k < kDealRecs; ++k)
            {
                own[k] = max(wave_inclusive_max((int)mark[k * 64 + lane]), carry) - 1;
                carry = wave_last(own[k]) + 1;
            }
            // the records: position + its segment's offset, 64 consecutive
            // positions per load instruction
            CellRec rec[kDealRecs];
            _Pragma("unroll") for (int k = 0; k < kDealRecs; ++k)
            {
                const int p = k * 64 + lane;
                if (p < cnt) rec[k] = V.crec[g_lo + p + (int)seg[max(own[k], 0)]];
            }
            // window test; candidates as keypoint | level << 16 | map lane << 20
            uint32_t cand[kDealRecs];
            int nc = 0;
            _Pragma("unroll") for (int k = 0; k < kDealRecs; ++k)
            {
                cand[k] = 0xFFFFFFFFu;
                if (k * 64 + lane < cnt) {
                    const int ml = max(own[k], 0) / kDealRows;
                    const float4 qq = qp[ml];
                    const int l = __float_as_int(qq.w);
                    Query iq;
                    iq.u = qq.x;
                    iq.v = qq.y;
                    iq.Rm = qq.z;
                    iq.plo = (l & 0xFF) - 16;
                    iq.phi = ((l >> 8) & 0xFF) - 16;
                    if (in_window(iq, rec[k].x, rec[k].y, rec[k].meta)) {
                        cand[k] = (rec[k].meta >> 16) | ((rec[k].meta & 15u) << 16) | ((uint32_t)ml << 20);
                        ++nc;
                    }
                }
            }
            const int cincl = wave_inclusive_scan(nc);
            const int ctot = wave_last(cincl);
            int cw = cincl - nc;
            _Pragma("unroll") for (int k = 0; k < kDealRecs; ++k) if (cand[k] != 0xFFFFFFFFu) cl[cw++] = cand[k];
            wave_lds_sync();
            // candidates dealt evenly: descriptor (and right coordinate) reads together
            for (int c0 = 0; c0 < ctot; c0 += 64 * kDealFlush) {
                uint32_t cc[kDealFlush];
                Desc d[kDealFlush];
                float ur[kDealFlush];
                _Pragma("unroll") for (int t = 0; t < kDealFlush; ++t)
                {
                    const int ci = c0 + t * 64 + lane;
                    cc[t] = ci < ctot ? cl[ci] : 0xFFFFFFFFu;
                    if (cc[t] != 0xFFFFFFFFu) d[t] = load_desc(V.kdesc, (int)(cc[t] & 0xFFFFu));
                    ur[t] = 0.0f;
                    if (cc[t] != 0xFFFFFFFFu && gate) ur[t] = V.u_right[cc[t] & 0xFFFFu];
                }
                _Pragma("unroll") for (int t = 0; t < kDealFlush; ++t)
                {
                    if (cc[t] == 0xFFFFFFFFu) continue;
                    const int ml = (int)(cc[t] >> 20);
                    const bool rej = gate && ur[t] > 0.0f && !(fabsf(quR[ml] - ur[t]) <= qp[ml].z);
                    if (!rej) {
                        const uint32_t key32 = ((uint32_t)hamming(qd[ml], d[t]) << 20) | ((cc[t] & 0xFFFFu) << 4) |
                                               ((cc[t] >> 16) & 15u);
                        const uint32_t old = atomicMin(&tb[ml], key32);
                        atomicMin(&tb[64 + ml], key32 < old ? old : key32);
                    }
                }
            }
            wave_lds_sync();   // the list is free for the next round
        }
    }
    wave_lds_sync();
    Top2<uint64_t> top = {key32_to_64(tb[lane]), key32_to_64(tb[64 + lane])};
    finish_query<1>(J, V, m, 0, top);
}

// Search by projection, kWG-thread tiles, G lanes per map point, records read
// from global memory.
template <int G>
__device__ __forceinline__ void ph_search(const DevJob &J, const DevView &V, int tile)
{
    const int sub = threadIdx.x % G;
    const int m = tile * (kWG / G) + threadIdx.x / G;
    Top2<uint64_t> top = {~0ull, ~0ull};
    if (m < J.nM) {
        const Query q = make_query(J, V, m);
        if (q.vis) top = scan_global<G>(V, q, sub);
    }
    finish_query<G>(J, V, m, sub, top);
}

__device__ __forceinline__ void ph_search_final(const DevJob &J, const DevView &V, int nK, int tile)
{
    const int idx = tile * kWG + threadIdx.x;
    if (idx < J.nM) {
        const int k = V.mp_k[idx];
        const bool keep = k >= 0 && V.claim[k] == (((uint32_t)V.mp_h[idx] << 23) | (uint32_t)idx);
        V.mp_match[idx] = keep ? k : -1;
        V.mp_dist[idx] = keep ? V.mp_h[idx] : -1;
    }
    bool has = false;
    if (idx < nK) {
        const uint32_t c = V.claim[idx];
        has = c != 0xFFFFFFFFu;
        V.kp_match[idx] = has ? (int)(c & 0x7FFFFFu) : -1;
    }
    const unsigned long long mk = __ballot(has);
    if ((threadIdx.x & 63) == 0 && mk) atomicAdd(V.n_matches, (int)__popcll(mk));
}

// --------------------------------- last-frame search by projection
// Initial Pose Estimation projects the last frame's matched map points into
// the current frame and searches its keypoints (Section II-C); the same
// search by projection as the local-map search (Section IV-E), with the
// window taken from the last-frame keypoint (radius th * sf[octave], levels
// by the direction of motion) instead of the predicted level, no ratio test,
// and a rotation-consistency check over the frame's matches.
//
// Camera projection of a world point into view V (pinhole binary32, KB
// binary64 rounded to binary32); false when the point is behind the camera
// or outside the image bounds.
__device__ __forceinline__ bool project_point(const DevView &V, float X, float Y, float Z, float &u, float &v,
                                              float &zc)
{
    const float xc = ((V.R[0] * X + V.R[1] * Y) + V.R[2] * Z) + V.t[0];
    const float yc = ((V.R[3] * X + V.R[4] * Y) + V.R[5] * Z) + V.t[1];
    zc = ((V.R[6] * X + V.R[7] * Y) + V.R[8] * Z) + V.t[2];
    u = 0.0f;
    v = 0.0f;
    if (!(zc > 0.0f)) return false;
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
    return u >= V.min_x && u <= V.max_x && v >= V.min_y && v <= V.max_y;
}

struct LastQuery {
    bool in;            // projected inside the image
    bool gate;          // stereo right-coordinate gate applies
    float u, v, r, uR;
    int lmin, lmax;     // keypoint levels searched
    int cx0, cx1, cy0, cy1;
    Desc d;
};

__device__ __forceinline__ LastQuery make_last_query(const DevJob &J, const DevView &V, int i)
{
    LastQuery q;
    const float X = J.pos[3 * i], Y = J.pos[3 * i + 1], Z = J.pos[3 * i + 2];
    const int ol = lvl(J.l_oct[i]);
    q.d = load_desc(J.mdesc, i);
    float zc;
    q.in = project_point(V, X, Y, Z, q.u, q.v, zc);
    if (!q.in) return q;
    q.r = J.th * J.sf[ol];
    if (J.direction > 0) {
        q.lmin = ol;
        q.lmax = kLevels - 1;
    } else if (J.direction < 0) {
        q.lmin = 0;
        q.lmax = ol;
    } else {
        q.lmin = ol - 1;
        q.lmax = ol + 1;
    }
    q.gate = V.u_right != nullptr;
    q.uR = q.gate ? q.u - V.bf * (1.0f / zc) : 0.0f;
    // cells of u -+ (r + 0.01) bracket every candidate (as in the local search)
    const float Rc = q.r + 0.01f;
    q.cx0 = cell_coord(q.u - Rc, V.min_x, V.inv_cw, V.cols);
    q.cx1 = cell_coord(q.u + Rc, V.min_x, V.inv_cw, V.cols);
    q.cy0 = cell_coord(q.v - Rc, V.min_y, V.inv_ch, V.rows);
    q.cy1 = cell_coord(q.v + Rc, V.min_y, V.inv_ch, V.rows);
    return q;
}

// Best candidate key (distance << 40 | keypoint << 8 | level) of one point
// over the window's cells of the one-bin index; lane `sub` of G takes every
// G-th record of each window row.
template <int G>
__device__ __forceinline__ uint64_t scan_last(const DevView &V, const LastQuery &q, int sub)
{
    uint64_t best = ~0ull;
    const FT_G int32_t *off = V.cell_off;
    for (int cy = q.cy0; cy <= q.cy1; ++cy) {
        const int c0 = off[cy * V.cols + q.cx0], c1 = off[cy * V.cols + q.cx1 + 1];
        for (int p0 = c0 + sub; p0 < c1; p0 += kSearchUnroll * G) {
            CellRec rec[kSearchUnroll];
            bool cand[kSearchUnroll];
            Desc d[kSearchUnroll];
            float ur[kSearchUnroll];
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e) rec[e] = V.crec[min(p0 + e * G, c1 - 1)];
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e)
            {
                const int ok = (int)(rec[e].meta & 0xFFu);
                cand[e] = p0 + e * G < c1 && ok >= q.lmin && ok <= q.lmax && fabsf(rec[e].x - q.u) < q.r &&
                          fabsf(rec[e].y - q.v) < q.r && !(rec[e].meta & 0x100u);
                ur[e] = 0.0f;
                if (cand[e]) {
                    d[e] = load_desc(V.kdesc, (int)(rec[e].meta >> 16));
                    if (q.gate) ur[e] = V.u_right[rec[e].meta >> 16];
                }
            }
            _Pragma("unroll") for (int e = 0; e < kSearchUnroll; ++e)
            {
                const bool rej = q.gate && ur[e] > 0.0f && !(fabsf(q.uR - ur[e]) <= q.r);
                if (cand[e] && !rej) best = min(best, cand_key(hamming(q.d, d[e]), rec[e].meta));
            }
        }
    }
    return best;
}

// G lanes per last-frame point: best candidate, acceptance, claim.
template <int G>
__device__ __forceinline__ void ph_last_search(const DevJob &J, const DevView &V, int tile)
{
    const int sub = threadIdx.x % G;
    const int i = tile * (kWG / G) + threadIdx.x / G;
    uint64_t best = ~0ull;
    if (i < J.nM) {
        const LastQuery q = make_last_query(J, V, i);
        if (q.in) best = scan_last<G>(V, q, sub);
    }
    for (int o = 1; o < G; o <<= 1) {
        const uint64_t other = shfl_xor64(best, o);
        best = other < best ? other : best;
    }
    if (sub != 0 || i >= J.nM) return;
    int k = -1, h = -1;
    if (best != ~0ull && (int)(best >> 40) <= J.th_high) {
        h = (int)(best >> 40);
        k = (int)((best >> 8) & 0xFFFFu);
    }
    V.mp_k[i] = k;
    V.mp_h[i] = h;
    if (k >= 0) atomicMin(&V.claim[k], ((uint32_t)h << 23) | (uint32_t)i);
}

// Rotation bin of a match: last minus current orientation, plus 360 when
// negative, rounded to one of `bins` equal bins, taken modulo `bins` (the one
// past the last is bin 0).
__device__ __forceinline__ int rotation_bin(float a_last, float a_cur, int bins)
{
    float rot = a_last - a_cur;
    if (rot < 0.0f) rot += 360.0f;
    const float factor = (float)bins / 360.0f;
    int bin = (int)roundf(rot * factor) % bins;   // the bin past the last is bin 0
    if (bin < 0) bin += bins;                      // (angles outside [0, 360) stay in range)
    return bin;
}

// Thread per point: the claim winners keep their keypoint (mp_k, distance |
// bin << 16 in mp_h; losers get -1) and count their rotation bin.
__device__ __forceinline__ void ph_last_resolve(const DevJob &J, const DevView &V, int tile)
{
    const int i = tile * kWG + threadIdx.x;
    if (i >= J.nM) return;
    const int k = V.mp_k[i];
    const int h = V.mp_h[i];
    const bool keep = k >= 0 && V.claim[k] == (((uint32_t)h << 23) | (uint32_t)i);
    int bin = 0;
    if (keep && J.check_rot) {
        bin = rotation_bin(J.l_ang[i], J.k_ang[k], J.rot_bins);
        atomicAdd(&V.hist[bin], 1);
    }
    V.mp_k[i] = keep ? k : -1;
    V.mp_h[i] = keep ? (h | (bin << 16)) : -1;
}

// Bins kept by the rotation check (bit b set): the fullest bin and, while
// holding a tenth of it, the second and third fullest; ties to the lower bin.
__device__ __forceinline__ uint64_t kept_bins(const DevView &V, int bins)
{
    int i1 = -1, i2 = -1, i3 = -1, m1 = 0, m2 = 0, m3 = 0;
    for (int b = 0; b < bins; ++b) {
        const int c = V.hist[b];
        if (c > m1) {
            m3 = m2;
            i3 = i2;
            m2 = m1;
            i2 = i1;
            m1 = c;
            i1 = b;
        } else if (c > m2) {
            m3 = m2;
            i3 = i2;
            m2 = c;
            i2 = b;
        } else if (c > m3) {
            m3 = c;
            i3 = b;
        }
    }
    if (10 * m2 < m1) {
        i2 = -1;
        i3 = -1;
    } else if (10 * m3 < m1) {
        i3 = -1;
    }
    uint64_t kept = 0;
    if (i1 >= 0) kept |= 1ull << i1;
    if (i2 >= 0) kept |= 1ull << i2;
    if (i3 >= 0) kept |= 1ull << i3;
    return kept;
}

// Thread per point / keypoint: the rotation check and the outputs.
__device__ __forceinline__ void ph_last_final(const DevJob &J, const DevView &V, int nK, int tile)
{
    const uint64_t kept = J.check_rot ? kept_bins(V, J.rot_bins) : ~0ull;
    auto alive = [&](int i) {
        return V.mp_k[i] >= 0 && ((kept >> ((V.mp_h[i] >> 16) & 63)) & 1ull);
    };
    const int idx = tile * kWG + threadIdx.x;
    if (idx < J.nM) {
        const bool a = alive(idx);
        V.mp_match[idx] = a ? V.mp_k[idx] : -1;
        V.mp_dist[idx] = a ? (V.mp_h[idx] & 0xFFFF) : -1;
    }
    bool has = false;
    if (idx < nK) {
        const uint32_t c = V.claim[idx];
        has = c != 0xFFFFFFFFu && alive((int)(c & 0x7FFFFFu));
        V.kp_match[idx] = has ? (int)(c & 0x7FFFFFu) : -1;
    }
    const unsigned long long mk = __ballot(has);
    if ((threadIdx.x & 63) == 0 && mk) atomicAdd(V.n_matches, (int)__popcll(mk));
}

// ------------------------------------------------------- tile bookkeeping

// Search tiles of a view: one wave of 64 map points for the record-dealt
// search (one lane per map point), else kWG / lanes map points.
__host__ __device__ inline int search_tiles_per_view(const DevJob &J, int lanes)
{
    return div_up(J.nM, lanes == 1 ? 64 : kWG / lanes);
}


__host__ __device__ inline int final_tiles_view(const DevJob &J, int v)
{
    const int nK = view_kp(J, v);
    return div_up(J.nM > nK ? J.nM : nK, kWG);
}

void job_tiles(const DevJob &J, const Shapes &s, bool do_stereo, bool do_search, int32_t out[PH_COUNT])
{
    for (int p = 0; p < PH_COUNT; ++p) out[p] = 0;
    if (do_stereo && J.imgL) out[PH_PYRAMID] = (J.imgR ? 2 : 1) * div_up(J.img_h, kPyrRows);
    const int nL = J.L.n;
    const bool pin = do_stereo && (J.flags & JOB_STEREO_PINHOLE);
    const bool fish = do_stereo && (J.flags & JOB_STEREO_FISHEYE);
    const int nv = do_search ? J.n_views : 0;
    out[PH_SETUP] = (pin || fish ? 1 : 0) + nv;
    if (pin) {
        out[PH_STEREO_A] = div_up(nL, kWG / s.best_lanes);
        out[PH_REFINE] = div_up(nL, refine_quarter(J) ? kRefineQPerWG : kRefinePerWG);
        out[PH_STEREO_C] = 1;
    } else if (fish) {
        out[PH_STEREO_A] = div_up(nL, kKnnQueriesPerWG);
        out[PH_TRI] = div_up(nL, kWG);
        out[PH_STEREO_C] = div_up(nL, s.aux_block);
    }
    for (int v = 0; v < nv; ++v) {
        out[PH_SEARCH] += search_tiles_per_view(J, s.search_lanes);
        out[PH_SEARCH_FIN] += final_tiles_view(J, v);
    }
}

// ------------------------------------------------------------------ kernels
// Consecutive logical tiles on one XCD: workgroups are dealt round-robin over
// the 8 XCDs, so block b runs on XCD b % 8; map it to a contiguous chunk.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int per = n >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

struct OneJob {
    DevJob j;
    __device__ __forceinline__ const DevJob &operator()(int) const { return j; }
    __device__ __forceinline__ bool locate(int, int &job, int &tile) const
    {
        job = 0;
        tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
        return true;
    }
};

struct JobTable : BatchArgs {
    __device__ __forceinline__ const DevJob &operator()(int i) const { return p[i]; }
    __device__ __forceinline__ bool locate(int ph, int &job, int &tile) const
    {
        const int32_t *pre = map.prefix + ph * (map.n_jobs + 1);
        const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
        int lo = 0, hi = map.n_jobs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= b) lo = mid;
            else hi = mid;
        }
        job = lo;
        tile = b - pre[lo];
        return tile < pre[lo + 1] - pre[lo];
    }
};
static_assert(sizeof(JobTable) == sizeof(BatchArgs), "graph nodes pass a BatchArgs as the JobTable argument");

// ------------------------------------------------------------ phase tasks
// One task = one tile of one phase of one frame, run by a whole workgroup.
// `smem` is the workgroup's LDS scratch (kTaskLds bytes, 16-byte aligned).
constexpr int kTaskLds = (kMaxCells + 8 + kWG) * 4;

template <int NT>
__device__ __forceinline__ void task_setup(const DevJob &J, int tile, unsigned char *smem)
{
    int *lds = reinterpret_cast<int *>(smem);
    int *tmp = lds + kMaxCells + 8;
    const bool stereo = J.flags & (JOB_STEREO_PINHOLE | JOB_STEREO_FISHEYE);
    if (stereo && tile == 0) {
        if (J.flags & JOB_STEREO_PINHOLE) ph_rowsort<NT>(J, lds, tmp);
        else ph_overlap<NT>(J, tmp);
        return;
    }
    const int v = tile - (stereo ? 1 : 0);
    const DevView &V = J.view[v];
    ph_cellsort<NT>(V, V.side ? J.R : J.L, J.lv_lo, J.lv_hi, lds, tmp);
}

template <int G>
__device__ __forceinline__ void task_stereo_a(const DevJob &J, int tile, unsigned char *smem)
{
    uint64_t *tab = reinterpret_cast<uint64_t *>(smem);
    uint32_t *part = reinterpret_cast<uint32_t *>(smem + 256 * sizeof(uint64_t));
    if (J.flags & JOB_STEREO_PINHOLE) ph_best<G>(J, tile);
    else ph_knn<kWG>(J, tile, tab, part);
}

template <int NT>
__device__ __forceinline__ void task_stereo_c(const DevJob &J, int tile, unsigned char *smem)
{
    int *hist = reinterpret_cast<int *>(smem);
    int *tmp = hist + 256;
    int *sh = tmp + NT;
    uint32_t *surv = reinterpret_cast<uint32_t *>(sh + 8);
    if (J.flags & JOB_STEREO_PINHOLE) ph_median<NT>(J, hist, tmp, surv, sh);
    else ph_fish_final<NT>(J, tile);
}

template <int G>
__device__ __forceinline__ void task_search(const DevJob &J, int tile, unsigned char *smem)
{
    const int tpv = search_tiles_per_view(J, G);
    const int v = tile / tpv;
    if (v >= J.n_views) return;
    if constexpr (G == 1) ph_search_deal(J, J.view[v], (tile - v * tpv) * 64, smem);
    else ph_search<G>(J, J.view[v], tile - v * tpv);
}

__device__ __forceinline__ void task_search_final(const DevJob &J, int tile)
{
    const int t0 = final_tiles_view(J, 0);
    const int v = tile < t0 ? 0 : 1;
    if (v >= J.n_views) return;
    ph_search_final(J, J.view[v], view_kp(J, v), tile - (v ? t0 : 0));
}

static_assert(256 * 8 + 4 * kKnnQueriesPerWG * 2 * 4 <= kTaskLds, "stereo_a LDS");
static_assert(kRefinePerWG * kRefineLds <= kTaskLds, "refine LDS");
static_assert(kRefineQPerWG * kRefineQLds <= kTaskLds, "refine LDS (quarter waves)");
static_assert(kDealLdsPerWave <= kTaskLds, "record-dealt search LDS");
static_assert((256 + kWG + 8) * 4 + (kMaxKp + 32) / 32 * 4 <= kTaskLds, "median LDS");

// ------------------------------------------------------- per-phase kernels
template <class Src>
__global__ __launch_bounds__(kWG) void k_pyramid(Src src)
{
    __shared__ __align__(16) unsigned char smem[kPyrLds];
    int job, tile;
    if (!src.locate(PH_PYRAMID, job, tile)) return;
    ph_pyramid(src(job), tile, smem);
}

template <class Src, int NT>
__global__ __launch_bounds__(NT) void k_setup(Src src)
{
    __shared__ __align__(16) unsigned char smem[(kMaxCells + 8 + NT) * 4];
    int job, tile;
    if (!src.locate(PH_SETUP, job, tile)) return;
    task_setup<NT>(src(job), tile, smem);
}

template <class Src, int G>
__global__ __launch_bounds__(kWG) void k_stereo_a(Src src)
{
    __shared__ __align__(16) unsigned char smem[256 * 8 + 4 * kKnnQueriesPerWG * 2 * 4];
    int job, tile;
    if (!src.locate(PH_STEREO_A, job, tile)) return;
    task_stereo_a<G>(src(job), tile, smem);
}

template <class Src>
// 7 waves per SIMD (at most 72 registers) instead of the 6 its 73 registers
// would give: more window loads in flight.  The batch kernel fits without a
// spill; the single-frame one spills two values.
__global__ __launch_bounds__(kWG, 7) void k_refine(Src src)
{
    __shared__ __align__(16) unsigned char smem[kRefineQPerWG * kRefineQLds > kRefinePerWG * kRefineLds
                                                    ? kRefineQPerWG * kRefineQLds
                                                    : kRefinePerWG * kRefineLds];
    int job, tile;
    if (!src.locate(PH_REFINE, job, tile)) return;
    ph_refine(src(job), tile, smem);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_tri(Src src)
{
    int job, tile;
    if (!src.locate(PH_TRI, job, tile)) return;
    ph_tri(src(job), tile);
}

template <class Src, int NT>
__global__ __launch_bounds__(NT) void k_stereo_c(Src src)
{
    __shared__ __align__(16) unsigned char smem[(256 + NT + 8) * 4 + (kMaxKp + 32) / 32 * 4];
    int job, tile;
    if (!src.locate(PH_STEREO_C, job, tile)) return;
    task_stereo_c<NT>(src(job), tile, smem);
}

template <class Src, int G>
__global__ __launch_bounds__(kWG) void k_search(Src src)
{
    int job, tile;
    if (!src.locate(PH_SEARCH, job, tile)) return;
    task_search<G>(src(job), tile, nullptr);
}

// Record-dealt search in one-wave workgroups: a wave's LDS and registers are
// released as soon as it ends (waves of one workgroup would hold theirs until
// the slowest ends), and single-wave workgroups take no barrier slot, so LDS
// alone bounds the waves per CU.  Registers are capped at seven waves per SIMD.
template <class Src>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_search_deal(Src src)
{
    __shared__ __align__(16) unsigned char smem[kDealLdsPerWave];
    int job, tile;
    if (!src.locate(PH_SEARCH, job, tile)) return;
    task_search<1>(src(job), tile, smem);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_search_final(Src src)
{
    int job, tile;
    if (!src.locate(PH_SEARCH_FIN, job, tile)) return;
    task_search_final(src(job), tile);
}

// Last-frame search (one view of one job): search, claim resolution with the
// rotation histogram, rotation check and outputs.
template <class Src, int G>
__global__ __launch_bounds__(kWG) void k_last_search(Src src)
{
    int job, tile;
    if (!src.locate(PH_SEARCH, job, tile)) return;
    const DevJob &J = src(job);
    ph_last_search<G>(J, J.view[0], tile);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_last_resolve(Src src)
{
    int job, tile;
    if (!src.locate(PH_SEARCH_FIN, job, tile)) return;
    const DevJob &J = src(job);
    ph_last_resolve(J, J.view[0], tile);
}

template <class Src>
__global__ __launch_bounds__(kWG) void k_last_final(Src src)
{
    int job, tile;
    if (!src.locate(PH_SEARCH_FIN, job, tile)) return;
    const DevJob &J = src(job);
    ph_last_final(J, J.view[0], view_kp(J, 0), tile);
}

hipError_t launch_last_frame(const DevJob &J, int lanes, hipStream_t s)
{
    OneJob src{J};
    void *args[] = {&src};
    const int nK = view_kp(J, 0);
    // setup: the view's one-bin cell index, claims cleared, histogram and
    // match count zeroed
    hipError_t e = hipLaunchKernel(reinterpret_cast<void *>(&k_setup<OneJob, kWG>), dim3(1), dim3(kWG), args, 0, s);
    if (e != hipSuccess) return e;
    if (J.nM > 0) {
        void *fn;
        switch (lanes) {
        case 1: fn = reinterpret_cast<void *>(&k_last_search<OneJob, 1>); break;
        case 2: fn = reinterpret_cast<void *>(&k_last_search<OneJob, 2>); break;
        case 8: fn = reinterpret_cast<void *>(&k_last_search<OneJob, 8>); break;
        default: fn = reinterpret_cast<void *>(&k_last_search<OneJob, 4>); lanes = 4; break;
        }
        if ((e = hipLaunchKernel(fn, dim3(div_up(J.nM, kWG / lanes)), dim3(kWG), args, 0, s)) != hipSuccess) return e;
        if ((e = hipLaunchKernel(reinterpret_cast<void *>(&k_last_resolve<OneJob>), dim3(div_up(J.nM, kWG)),
                                 dim3(kWG), args, 0, s)) != hipSuccess)
            return e;
    }
    const int n = J.nM > nK ? J.nM : nK;
    if (n > 0 && (e = hipLaunchKernel(reinterpret_cast<void *>(&k_last_final<OneJob>), dim3(div_up(n, kWG)),
                                      dim3(kWG), args, 0, s)) != hipSuccess)
        return e;
    return hipGetLastError();
}

// ---------------------------------------------------- local-map edit
// A thread per moved or appended point copies its 64-byte record (position,
// normal, distance bounds, descriptor).
__device__ __forceinline__ void map_copy_rec(const MapEditArgs &a, int to, const FT_G float *pos,
                                             const FT_G float *normal, const FT_G float *dmin,
                                             const FT_G float *dmax, const FT_G uint8_t *desc, int from)
{
    float p[3], nr[3];
    _Pragma("unroll") for (int c = 0; c < 3; ++c)
    {
        p[c] = pos[3 * from + c];
        nr[c] = normal[3 * from + c];
    }
    const float d0 = dmin[from], d1 = dmax[from];
    const uint4 q0 = reinterpret_cast<const FT_G uint4 *>(desc + 32 * (size_t)from)[0];
    const uint4 q1 = reinterpret_cast<const FT_G uint4 *>(desc + 32 * (size_t)from)[1];
    _Pragma("unroll") for (int c = 0; c < 3; ++c)
    {
        a.pos[3 * to + c] = p[c];
        a.normal[3 * to + c] = nr[c];
    }
    a.dmin[to] = d0;
    a.dmax[to] = d1;
    reinterpret_cast<FT_G uint4 *>(a.desc + 32 * (size_t)to)[0] = q0;
    reinterpret_cast<FT_G uint4 *>(a.desc + 32 * (size_t)to)[1] = q1;
}

__global__ __launch_bounds__(kWG) void k_map_move(MapEditArgs a)
{
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i >= a.n_pairs) return;
    const int hole = a.pairs[2 * i], src = a.pairs[2 * i + 1];
    map_copy_rec(a, hole, a.pos, a.normal, a.dmin, a.dmax, a.desc, src);
}

__global__ __launch_bounds__(kWG) void k_map_append(MapEditArgs a)
{
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= a.n_insert) return;
    map_copy_rec(a, a.n1 + j, a.ipos, a.inormal, a.idmin, a.idmax, a.idesc, j);
}

hipError_t launch_map_edit(const MapEditArgs &a, hipStream_t s)
{
    if (a.n_pairs > 0) hipLaunchKernelGGL(k_map_move, dim3(div_up(a.n_pairs, kWG)), dim3(kWG), 0, s, a);
    if (a.n_insert > 0) hipLaunchKernelGGL(k_map_append, dim3(div_up(a.n_insert, kWG)), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

// Kernel of phase p for these shapes, and its workgroup size.
template <class Src>
static void *phase_kernel(const Shapes &sh, int p, int *block)
{
    *block = kWG;
    switch (p) {
    case PH_PYRAMID: return reinterpret_cast<void *>(&k_pyramid<Src>);
    case PH_SETUP:
        if (sh.aux_block == kAuxWG) {
            *block = kAuxWG;
            return reinterpret_cast<void *>(&k_setup<Src, kAuxWG>);
        }
        return reinterpret_cast<void *>(&k_setup<Src, kWG>);
    case PH_STEREO_A:
        switch (sh.best_lanes) {
        case 1: return reinterpret_cast<void *>(&k_stereo_a<Src, 1>);
        case 2: return reinterpret_cast<void *>(&k_stereo_a<Src, 2>);
        case 4: return reinterpret_cast<void *>(&k_stereo_a<Src, 4>);
        case 16: return reinterpret_cast<void *>(&k_stereo_a<Src, 16>);
        default: return reinterpret_cast<void *>(&k_stereo_a<Src, 8>);
        }
    case PH_REFINE: return reinterpret_cast<void *>(&k_refine<Src>);
    case PH_TRI: return reinterpret_cast<void *>(&k_tri<Src>);
    case PH_STEREO_C:
        if (sh.aux_block == kAuxWG) {
            *block = kAuxWG;
            return reinterpret_cast<void *>(&k_stereo_c<Src, kAuxWG>);
        }
        return reinterpret_cast<void *>(&k_stereo_c<Src, kWG>);
    case PH_SEARCH:
        switch (sh.search_lanes) {
        case 1: *block = 64; return reinterpret_cast<void *>(&k_search_deal<Src>);
        case 2: return reinterpret_cast<void *>(&k_search<Src, 2>);
        case 8: return reinterpret_cast<void *>(&k_search<Src, 8>);
        case 16: return reinterpret_cast<void *>(&k_search<Src, 16>);
        default: return reinterpret_cast<void *>(&k_search<Src, 4>);
        }
    default: return reinterpret_cast<void *>(&k_search_final<Src>);
    }
}

void batch_kernels(const Shapes &shapes, void *fn[PH_COUNT], int block[PH_COUNT])
{
    for (int p = 0; p < PH_COUNT; ++p) fn[p] = phase_kernel<JobTable>(shapes, p, &block[p]);
}

template <class Src>
static hipError_t run(Src src, const int32_t *tot, const Shapes &sh, hipStream_t s, hipEvent_t *ev)
{
    void *args[] = {&src};
    for (int p = 0; p < PH_COUNT; ++p) {
        if (ev) (void)hipEventRecord(ev[p], s);
        if (tot[p] <= 0) continue;   // planned by job_tiles for the phases asked for
        int block = kWG;
        void *fn = phase_kernel<Src>(sh, p, &block);
        const hipError_t e = hipLaunchKernel(fn, dim3(tot[p]), dim3(block), args, 0, s);
        if (e != hipSuccess) return e;
    }
    if (ev) (void)hipEventRecord(ev[PH_COUNT], s);
    return hipGetLastError();
}

hipError_t launch_pipeline(const DevJob *table, const TileMap &map, const int32_t totals[PH_COUNT],
                           const DevJob &one, const Shapes &shapes, hipStream_t stream, hipEvent_t *ev)
{
    if (table) return run(JobTable{{table, map}}, totals, shapes, stream, ev);
    return run(OneJob{one}, totals, shapes, stream, ev);
}

}  // namespace ft
