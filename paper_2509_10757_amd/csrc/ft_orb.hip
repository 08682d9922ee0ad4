// ORB extraction on the device-resident image pyramid (Section II-A: keypoints
// are extracted on every scale and described; Section IV-B: the extraction
// runs next to the pyramid on the device).
//
//  * k_orb_detect: one 1024-thread workgroup per tile of kOrbRows rows of one
//    level.  The tile's level rows and kOrbHalo rows above and below are
//    staged in LDS; FAST-9 scores (a compass-point quick test first) fill a
//    score band one row larger on each side; strict 3x3 suppression collects
//    the tile's corners in (row, column) order in LDS; the tile's first output
//    index comes from a decoupled look-back over the counts of the tiles
//    before it (tiles are in (level, row) order and taken by ticket), and the
//    corners are written contiguously; the descriptor's binomial smoothing of
//    the tile's rows is written from the same staged rows.
//  * k_orb_describe: one wave per keypoint: the intensity-centroid moments
//    over the radius-15 disc (lanes stride the disc, one wave reduction), then
//    four tests per lane on the smoothed level with the pattern turned exactly
//    by the moments (integer rounding decisions), and one ballot per 64 tests
//    gives 8 descriptor bytes.
#include <hip/hip_runtime.h>

#define FT_KERNELS 1
#include "ft_internal.h"

namespace ft {

namespace {

constexpr int kThreads = 256;      // description: one wave per keypoint, 4 waves per workgroup
constexpr int kDetThreads = 1024;  // detection: one tile per workgroup, 4 waves per SIMD
constexpr int kStaged = kOrbRows + 2 * kOrbHalo;   // level rows staged per tile
constexpr int kScoreRows = kOrbRows + 2;           // score rows: the tile and one row each side
static_assert(kOrbRows % 2 == 0 && kOrbRows <= 8 && kMaxPyrW < 2048, "emitted corners pack column, row, score");

// The 16 ring pixels at distance 3 (clockwise from straight above).
__constant__ int8_t kRingDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t kRingDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

__device__ __forceinline__ int level_of_tile(const OrbDetectArgs &a, int tile)
{
    int l = 0;
    while (l + 1 < kLevels && tile >= a.tile0[l + 1]) ++l;
    return l;
}

// FAST-9 score of the staged pixel (x, staged row sr), 0 unless it reaches t.
__device__ __forceinline__ int fast_score(const unsigned char *px, int S, int sr, int x, int t)
{
    const unsigned char *p = px + sr * S + x;
    const int c = p[0];
    const int hi = c + t, lo = c - t;
    const int n0 = p[-3 * S], n4 = p[3], n8 = p[3 * S], n12 = p[-3];
    // nine consecutive ring pixels always include two neighbouring compass points
    const bool b0 = n0 > hi, b4 = n4 > hi, b8 = n8 > hi, b12 = n12 > hi;
    const bool d0 = n0 < lo, d4 = n4 < lo, d8 = n8 < lo, d12 = n12 < lo;
    const bool maybe = (b0 && b4) || (b4 && b8) || (b8 && b12) || (b12 && b0) || (d0 && d4) || (d4 && d8) ||
                       (d8 && d12) || (d12 && d0);
    if (!maybe) return 0;
    int e[16];
    _Pragma("unroll") for (int k = 0; k < 16; ++k) e[k] = (int)p[kRingDy[k] * S + kRingDx[k]] - c;
    // sliding minimum (bright side), then maximum (dark side), over nine
    // consecutive ring pixels by doubling; one side at a time keeps the live
    // set small
    int bright = -256, dark = 256;   // best arc minimum; smallest arc maximum
    {
        int a2[16], a4[16];
        _Pragma("unroll") for (int k = 0; k < 16; ++k) a2[k] = min(e[k], e[(k + 1) & 15]);
        _Pragma("unroll") for (int k = 0; k < 16; ++k) a4[k] = min(a2[k], a2[(k + 2) & 15]);
        _Pragma("unroll") for (int k = 0; k < 16; ++k)
            bright = max(bright, min(min(a4[k], a4[(k + 4) & 15]), e[(k + 8) & 15]));
    }
    {
        int a2[16], a4[16];
        _Pragma("unroll") for (int k = 0; k < 16; ++k) a2[k] = max(e[k], e[(k + 1) & 15]);
        _Pragma("unroll") for (int k = 0; k < 16; ++k) a4[k] = max(a2[k], a2[(k + 2) & 15]);
        _Pragma("unroll") for (int k = 0; k < 16; ++k)
            dark = min(dark, max(max(a4[k], a4[(k + 4) & 15]), e[(k + 8) & 15]));
    }
    const int s = max(bright, -dark) - 1;
    return s >= t ? s : 0;
}

// Stage the tile's level rows (clamped at the level's borders) into LDS with
// row stride W, and fill the score band (stride W); returns after a barrier.
// `lds` is 16-byte aligned; the staged rows start at the returned pointer.
// Interior tiles copy one contiguous range: aligned dwords (every load issued
// before the LDS stores), bytes at the two ragged ends; a tile whose halo
// leaves the level copies row by row with clamped row indices.
__device__ __forceinline__ unsigned char *stage_and_score(const OrbDetectArgs &a, int l, int y0, int rows,
                                                          unsigned char *lds)
{
    const int W = a.w[l], H = a.h[l];
    const FT_G uint8_t *img = a.pyr + a.off[l];
    const int n_staged = rows + 2 * kOrbHalo;
    unsigned char *px;
    if (y0 - kOrbHalo >= 0 && y0 + rows + kOrbHalo <= H) {
        const FT_G uint8_t *g0 = img + (int64_t)(y0 - kOrbHalo) * W;
        const int len = n_staged * W;
        const uintptr_t ga = reinterpret_cast<uintptr_t>(g0);
        const int sh = (int)(ga & 3u);
        px = lds + sh;                                   // px[i] = g0[i]; aligned dwords land aligned
        const int head = sh ? 4 - sh : 0;                // bytes before the first aligned dword
        const int nd = (len - head) >> 2;                // whole aligned dwords
        const FT_G uint32_t *gd = reinterpret_cast<const FT_G uint32_t *>(g0 + head);
        uint32_t *ld = reinterpret_cast<uint32_t *>(px + head);
        constexpr int kMaxPer = (kStaged * kMaxPyrW / 4 + kDetThreads - 1) / kDetThreads;
        uint32_t v[kMaxPer];
        _Pragma("unroll") for (int k = 0; k < kMaxPer; ++k)
        {
            const int j = (int)threadIdx.x + k * kDetThreads;
            if (j < nd) v[k] = gd[j];
        }
        _Pragma("unroll") for (int k = 0; k < kMaxPer; ++k)
        {
            const int j = (int)threadIdx.x + k * kDetThreads;
            if (j < nd) ld[j] = v[k];
        }
        const int tail0 = head + 4 * nd;
        if ((int)threadIdx.x < head) px[threadIdx.x] = g0[threadIdx.x];
        if ((int)threadIdx.x < len - tail0) px[tail0 + threadIdx.x] = g0[tail0 + threadIdx.x];
    } else {
        px = lds;
        for (int sr = 0; sr < n_staged; ++sr) {
            int yy = y0 - kOrbHalo + sr;
            yy = yy < 0 ? 0 : (yy > H - 1 ? H - 1 : yy);
            const FT_G uint8_t *src = img + (int64_t)yy * W;
            for (int x = threadIdx.x; x < W; x += kDetThreads) px[sr * W + x] = src[x];
        }
    }
    __syncthreads();
    const int S = W;
    unsigned char *sc = lds + 4 + kStaged * a.lds_w;    // after the staged rows and their slack
    const int E = a.edge;
    for (int r = 0; r < rows + 2; ++r) {
        const int yy = y0 - 1 + r;
        const bool row_in = yy >= E && yy < H - E;
        for (int x = threadIdx.x; x < W; x += kDetThreads) {
            int s = 0;
            if (row_in && x >= E && x < W - E) s = fast_score(px, S, r + kOrbHalo - 1, x, a.t);
            sc[r * S + x] = (unsigned char)s;
        }
    }
    __syncthreads();
    return px;
}

__device__ __forceinline__ unsigned char *score_band(const OrbDetectArgs &a, unsigned char *lds)
{
    return lds + 4 + kStaged * a.lds_w;
}

// A tile's kept corners (emission): strict suppression never keeps two
// 8-neighbours, so a tile holds at most (kOrbRows / 2) x ceil(W / 2) corners;
// lds_w is W rounded up to 4, so (kOrbRows / 2) x (lds_w / 2) entries suffice.
__device__ __forceinline__ uint32_t *corner_list(const OrbDetectArgs &a, unsigned char *lds)
{
    return reinterpret_cast<uint32_t *>(lds + 8 + (kStaged + kScoreRows) * a.lds_w);
}

// Is the corner at output row r, column x kept by the suppression?
__device__ __forceinline__ bool kept(const unsigned char *sc, int S, int r, int x, int W)
{
    if (x >= W) return false;
    const unsigned char *q = sc + (r + 1) * S + x;
    const int v = q[0];
    if (v == 0) return false;
    // window pixels are >= 19 from every border: the 8 neighbours exist
    return v > q[-S - 1] && v > q[-S] && v > q[-S + 1] && v > q[-1] && v > q[1] && v > q[S - 1] && v > q[S] &&
           v > q[S + 1];
}

constexpr int kDetWaves = kDetThreads / 64;

// Look-back state of a tile: epoch << 32 | flag << 30 | value (corners).
constexpr unsigned long long kAggregate = 1ull << 30, kInclusive = 2ull << 30;
constexpr uint32_t kValueMask = (1u << 30) - 1u;
constexpr int kMaxSpins = 1 << 16;       // bounds every wait (a tile found stuck poisons the prefix)
constexpr int kPoison = 1 << 29;         // prefix of a tile whose predecessors never published

__global__ __launch_bounds__(kDetThreads, 8) void k_orb_detect(OrbDetectArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int wave_n[kDetWaves];
    __shared__ int shared_tile, shared_prefix;
    // tiles by ticket: every lower tile has been taken by a running workgroup,
    // and none waits on a higher one, so each wait below ends
    if (threadIdx.x == 0) shared_tile = (int)(atomicAdd(a.ticket, 1u) - a.ticket_base);
    __syncthreads();
    const int tile = shared_tile;
    const int tiles = a.tile0[kLevels];
    const int l = level_of_tile(a, tile);
    const int W = a.w[l], H = a.h[l], S = W;
    const int y0 = (tile - a.tile0[l]) * kOrbRows;
    const int rows = min(kOrbRows, H - y0);
    const unsigned char *px = stage_and_score(a, l, y0, rows, lds);
    const unsigned char *sc = score_band(a, lds);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long ep = (unsigned long long)a.epoch << 32;
    // the tile's corners in (row, column) order, packed column | row << 11 |
    // score << 14
    uint32_t *tc = corner_list(a, lds);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int n = 0;
    for (int r = 0; r < rows; ++r)
        for (int x0 = 0; x0 < W; x0 += kDetThreads) {
            const int x = x0 + (int)threadIdx.x;
            const bool k = kept(sc, S, r, x, W);
            const uint64_t m = __ballot(k);
            if (lane == 0) wave_n[wave] = __popcll(m);
            __syncthreads();
            int off = n;
            for (int w = 0; w < wave; ++w) off += wave_n[w];
            int chunk = 0;
            _Pragma("unroll") for (int w = 0; w < kDetWaves; ++w) chunk += wave_n[w];
            __syncthreads();
            if (k) tc[off + __popcll(m & below)] = (uint32_t)x | ((uint32_t)r << 11) | ((uint32_t)sc[(r + 1) * S + x] << 14);
            n += chunk;
        }
    // decoupled look-back: the tile publishes its count; wave 0 then reads 64
    // predecessors' states at a time and adds the counts down to the nearest
    // inclusive prefix (a window with an unpublished state before it is read
    // again); the tile then publishes its own inclusive prefix
    if (wave == 0) {
        int prefix = 0;
        if (lane == 0)
            atomicExch(&a.tile_state[tile], ep | (tile == 0 ? kInclusive : kAggregate) | (unsigned long long)n);
        if (tile > 0) {
            int top = tile - 1, spins = 0;
            for (;;) {
                const int k = top - lane;
                unsigned long long v = ep | kInclusive;          // before tile 0: an inclusive 0
                if (k >= 0) v = atomicOr(&a.tile_state[k], 0ull);  // coherent read
                const bool pub = (v >> 32) == a.epoch && (v & (3ull << 30));
                const uint64_t inc = __ballot(pub && (v & kInclusive));
                const uint64_t unpub = __ballot(!pub);
                const int first = inc ? __ffsll((long long)inc) - 1 : 64;   // nearest inclusive lane
                const uint64_t upto = first == 64 ? ~0ull : (~0ull >> (63 - first));
                if (unpub & upto) {
                    if (++spins > kMaxSpins) {
                        prefix += kPoison;
                        break;
                    }
                    continue;
                }
                int add = (lane <= first) ? (int)(v & kValueMask) : 0;
                _Pragma("unroll") for (int o = 32; o > 0; o >>= 1) add += __shfl_xor(add, o);
                prefix += add;
                if (first < 64) break;
                top -= 64;
            }
            if (lane == 0)
                atomicExch(&a.tile_state[tile], ep | kInclusive | (unsigned long long)min(prefix + n, (int)kValueMask));
        }
        if (lane == 0) {
            shared_prefix = prefix;
            if (tile == tiles - 1) a.count[0] = prefix + n >= kPoison ? -1 : prefix + n;
        }
    }
    __syncthreads();
    const int before = shared_prefix;
    const float sf = a.sf[l];
    for (int k = threadIdx.x; k < n; k += kDetThreads) {
        const int i = before + k;
        if (i >= a.capacity) break;
        const uint32_t e = tc[k];
        const int x = (int)(e & 2047u), yy = y0 + (int)((e >> 11) & 7u);
        a.lx[i] = (int16_t)x;
        a.ly[i] = (int16_t)yy;
        a.oct[i] = (uint8_t)l;
        a.score[i] = (uint8_t)(e >> 14);
        a.x[i] = (float)x * sf;
        a.y[i] = (float)yy * sf;
    }
    if (a.blurred) {
        // smoothing: per column, horizontal sums of staged rows 1 .. rows + 6
        // (level rows y0 - 3 .. y0 + rows + 2, clamped), then the vertical taps
        FT_G uint8_t *dst = a.blurred + a.off[l];
        constexpr int kw[7] = {1, 6, 15, 20, 15, 6, 1};
        for (int x = threadIdx.x; x < W; x += kDetThreads) {
            int xs[7];
            _Pragma("unroll") for (int i = 0; i < 7; ++i)
            {
                const int v = x + i - 3;
                xs[i] = v < 0 ? 0 : (v > W - 1 ? W - 1 : v);
            }
            int hs[kOrbRows + 6];
            _Pragma("unroll") for (int k = 0; k < kOrbRows + 6; ++k)
            {
                const unsigned char *row = px + (k + 1) * S;
                int acc = 0;
                _Pragma("unroll") for (int i = 0; i < 7; ++i) acc += kw[i] * row[xs[i]];
                hs[k] = acc;
            }
            _Pragma("unroll") for (int r = 0; r < kOrbRows; ++r)
            {
                if (r < rows) {
                    int acc = 0;
                    _Pragma("unroll") for (int j = 0; j < 7; ++j) acc += kw[j] * hs[r + j];
                    dst[(int64_t)(y0 + r) * W + x] = (uint8_t)((acc + 2048) >> 12);
                }
            }
        }
    }
}

// The integer nearest num / sqrt(m2), halves away from zero, decided exactly:
// the largest k >= 0 with k = 0 or (2k - 1)^2 m2 <= 4 num^2, with num's sign;
// found from a binary64 estimate by exact integer corrections.
__device__ __forceinline__ int round_ratio_exact(int num, int64_t m2)
{
    const int64_t a = num < 0 ? -(int64_t)num : (int64_t)num;
    const int64_t a4 = 4 * a * a;
    int k = (int)floor((double)a / sqrt((double)m2) + 0.5);
    if (k < 0) k = 0;
    while (k > 0 && (int64_t)(2 * k - 1) * (2 * k - 1) * m2 > a4) --k;
    while ((int64_t)(2 * k + 1) * (2 * k + 1) * m2 <= a4) ++k;
    return num < 0 ? -k : k;
}

// The same integer from a binary32 estimate |num| * rsqrt(m10^2 + m01^2),
// the squares summed in binary32: every step is within a few units in the
// last place, and turned pattern coordinates are at most 13, so the estimate
// is within 1e-5 of the exact quotient and, unless it lies within 1e-4 of a
// half, rounds to the exact integer; `near` is set otherwise (the caller then
// decides exactly).
__device__ __forceinline__ int turn_fast(int num, float inv_r, bool &near)
{
    const int a = num < 0 ? -num : num;
    const float q = (float)a * inv_r;
    const float fr = q - floorf(q);
    near |= !(fabsf(fr - 0.5f) > 1e-4f);
    const int k = (int)(q + 0.5f);
    return num < 0 ? -k : k;
}

// Sum over the 64 lanes of a wave (every lane active) by DPP moves: shifts
// by 1, 2, 4 and 8 inside rows of 16 lanes, then lane 15 of rows 0 and 2 into
// rows 1 and 3, then lane 31 into rows 2 and 3; lane 63 holds the total.
__device__ __forceinline__ int wave_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ float angle_deg(int m10, int m01)
{
    double ang = atan2((double)m01, (double)m10) * (180.0 / 3.14159265358979323846);
    if (ang < 0.0) ang += 360.0;
    return (float)ang;
}

// Four waves per SIMD (at most 128 registers): a few values spill, but the
// extra waves hide more of the pixel gathers than the spills cost.
__global__ __launch_bounds__(kThreads, 4) void k_orb_describe(OrbDescribeArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = (int)((blockIdx.x * kThreads + threadIdx.x) >> 6);
    const int waves = (int)(gridDim.x * (kThreads / 64));
    int n = a.n_max;
    if (a.count) {
        const int c = a.count[0];
        n = c < n ? c : n;
    }
    // this lane's four tests (t = 64 q + lane), held for the whole kernel
    int tx1[4], ty1[4], tx2[4], ty2[4];
    _Pragma("unroll") for (int q = 0; q < 4; ++q)
    {
        const int t = q * 64 + lane;
        tx1[q] = a.pattern[t][0];
        ty1[q] = a.pattern[t][1];
        tx2[q] = a.pattern[t][2];
        ty2[q] = a.pattern[t][3];
    }
    // disc geometry of this lane: column dx for all 16 positions, rows dy0 + 2j
    const int dx = (lane & 31) - 15, dxl = dx < 15 ? dx : 15;
    const int dy0 = (lane >> 5) - 15;
    // angles: lane (slot % 64) keeps the moments of the wave's slot-th
    // keypoint; every 64 slots (and at the end) each lane converts its own
    int keep_i = -1, keep_m10 = 0, keep_m01 = 0;
    int slot = 0;
    for (int i = wave; i < n; i += waves, ++slot) {
        const int l = a.oct[i];
        const int u = a.lx[i], v = a.ly[i];
        const bool ok = l < kLevels && u >= 15 && v >= 15 && u < a.w[l < kLevels ? l : 0] - 15 &&
                        v < a.h[l < kLevels ? l : 0] - 15;
        FT_G uint8_t *d = a.desc + 32 * (int64_t)i;
        int m10 = 0, m01 = 0;
        if (!ok) {   // outside the window the disc and the turned pattern need
            if (lane < 8) reinterpret_cast<FT_G uint32_t *>(d)[lane] = 0u;
        } else {
            const int W = a.w[l];
            const FT_G uint8_t *img = a.pyr + a.off[l] + (int64_t)v * W + u;
            const FT_G uint8_t *B = a.blurred + a.off[l] + (int64_t)v * W + u;
            // the 32 x 32 square from (-15, -15): 16 positions per lane, every
            // load issued before any is used (row and column 16, outside the
            // disc, load a pixel of row or column 15 and weigh 0)
            int pix[16];
            _Pragma("unroll") for (int j = 0; j < 16; ++j)
            {
                const int dy = dy0 + 2 * j;
                pix[j] = img[(dy < 15 ? dy : 15) * W + dxl];
            }
            int sx = 0;
            _Pragma("unroll") for (int j = 0; j < 16; ++j)
            {
                const int dy = dy0 + 2 * j;
                const int w = (dx <= 15 && dx * dx + dy * dy <= 225) ? pix[j] : 0;
                sx += w;
                m01 += dy * w;
            }
            m10 = wave_sum(dx * sx);
            m01 = wave_sum(m01);
            const bool turned = (m10 | m01) != 0;   // the squared radius m10^2 + m01^2 is positive
            const float f10 = (float)m10, f01 = (float)m01;   // exact: |m| < 2^24
            const float inv_r = turned ? rsqrtf(f10 * f10 + f01 * f01) : 0.0f;
            // per test: the two turned points (binary32 estimates, the exact
            // decision when one lies near a half), then their smoothed pixels
            uint64_t mask[4];
            _Pragma("unroll") for (int q = 0; q < 4; ++q)
            {
                const int n0 = tx1[q] * m10 - ty1[q] * m01, n1 = tx1[q] * m01 + ty1[q] * m10;
                const int n2 = tx2[q] * m10 - ty2[q] * m01, n3 = tx2[q] * m01 + ty2[q] * m10;
                int c1 = tx1[q], r1 = ty1[q], c2 = tx2[q], r2 = ty2[q];
                if (turned) {
                    bool near = false;
                    c1 = turn_fast(n0, inv_r, near);
                    r1 = turn_fast(n1, inv_r, near);
                    c2 = turn_fast(n2, inv_r, near);
                    r2 = turn_fast(n3, inv_r, near);
                    if (near) {
                        const int64_t m2 = (int64_t)m10 * m10 + (int64_t)m01 * m01;
                        c1 = round_ratio_exact(n0, m2);
                        r1 = round_ratio_exact(n1, m2);
                        c2 = round_ratio_exact(n2, m2);
                        r2 = round_ratio_exact(n3, m2);
                    }
                }
                mask[q] = __ballot(B[r1 * W + c1] < B[r2 * W + c2]);
            }
            if (lane < 4) {
                const uint64_t mq = lane == 0 ? mask[0] : lane == 1 ? mask[1] : lane == 2 ? mask[2] : mask[3];
                reinterpret_cast<FT_G uint64_t *>(d)[lane] = mq;
            }
        }
        if (lane == (slot & 63)) {
            keep_i = ok ? i : -2 - i;
            keep_m10 = m10;
            keep_m01 = m01;
        }
        if ((slot & 63) == 63) {
            if (keep_i >= 0) a.angle[keep_i] = angle_deg(keep_m10, keep_m01);
            else if (keep_i < -1) a.angle[-2 - keep_i] = -1.0f;
            keep_i = -1;
        }
    }
    if (keep_i >= 0) a.angle[keep_i] = angle_deg(keep_m10, keep_m01);
    else if (keep_i < -1) a.angle[-2 - keep_i] = -1.0f;
}

}  // namespace

size_t orb_detect_lds(int lds_w)
{
    return (size_t)(kStaged + kScoreRows) * (size_t)lds_w + 8 + 4 * (size_t)(kOrbRows / 2) * (size_t)(lds_w / 2);
}

hipError_t launch_orb_detect(const OrbDetectArgs &a, hipStream_t s)
{
    const int tiles = a.tile0[kLevels];
    if (tiles <= 0) return hipSuccess;
    const size_t lds = orb_detect_lds(a.lds_w);
    hipLaunchKernelGGL(k_orb_detect, dim3(tiles), dim3(kDetThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_orb_describe(const OrbDescribeArgs &a, hipStream_t s)
{
    if (a.n_max <= 0) return hipSuccess;
    const int per_block = kThreads / 64;
    int blocks = (a.n_max + per_block - 1) / per_block;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_orb_describe, dim3(blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace ft
