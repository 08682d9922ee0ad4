// Host side of the C ABI declared in include/ft.h: context and preallocated
// workspace, synchronous argument validation, job descriptors, batch tickets,
// per-phase timing and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ft_internal.h"

using namespace ft;

namespace {

struct Slot {  // workspace of one frame
    int32_t *row_start, *best_j, *best_h, *h2, *sad, *flag, *qlist, *tlist, *counts;
    RowRec *rrec;
    uint8_t *tdesc;
    float *uR, *depth, *xyz;
    MatchRec *mrec;
    uint32_t *claimR;
    struct {
        int32_t *cell_off, *mp_k, *mp_h, *hist;
        CellRec *crec;
        uint32_t *claim;
    } view[2];
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Layout of one batch table: the tile prefix sums, then the job descriptors.
// One upload of the first upload_bytes(n) bytes moves everything a launch
// reads.
struct TableLayout {
    size_t prefix_off = 0, jobs_off = 0, total = 0;
    size_t upload_bytes(int n) const { return jobs_off + sizeof(DevJob) * (size_t)n; }
};

TableLayout table_layout(int max_frames)
{
    TableLayout t;
    t.jobs_off = align_up(sizeof(int32_t) * PH_COUNT * (size_t)(max_frames + 1), 256);
    t.total = align_up(t.jobs_off + sizeof(DevJob) * (size_t)max_frames, 256);
    return t;
}

// A lane's batch graph: the table upload followed by one kernel node per
// phase, in phase order.  Built once per shape setting; a submission sets the
// upload size and each kernel's grid and argument in the instantiated graph.
struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr;
    hipGraphNode_t kern[PH_COUNT] = {};
    void *fn[PH_COUNT] = {};
    int block[PH_COUNT] = {};
    int32_t n[PH_COUNT] = {};        // job count (kernel argument) each node was last set for
    int32_t grid[PH_COUNT] = {};     // grid each node was last set for
    bool off[PH_COUNT] = {};         // phase nodes disabled for the last submission (no tiles)
};

struct Lane {  // one batch in flight
    std::vector<Slot> slots;
    BatchGraph g;
    char *d_table = nullptr;   // device: prefixes | jobs
    char *h_table = nullptr;   // pinned staging of the same bytes
    hipEvent_t done = nullptr;
    uint64_t ticket = 0;
    bool used = false;
};

}  // namespace

struct ft_context {
    int device = 0;
    ft_limits lim{};
    char *base = nullptr;
    size_t bytes = 0;
    Slot direct{};
    std::vector<Lane> lanes;
    TableLayout layout{};
    ft_status sticky = FT_OK;
    std::string err;
    uint64_t next_ticket = 1;
    Shapes shapes;
    int32_t exec_mode = FT_EXEC_GRAPH;
    int64_t batch_kp_cap = 0, batch_map_cap = 0;   // per-submission totals (ft_limits)
    // per-phase timing: a ring of event sets, drained when it wraps or on read
    bool timing = false;
    std::vector<std::vector<hipEvent_t>> ev_sets;
    std::vector<uint8_t> ev_pending;   // 0 free, 1 per-phase marks pending
    std::vector<uint32_t> ev_mask;     // phases with a launched kernel, per event set
    size_t ev_next = 0;
    double phase_ms[kPhases] = {};
    int64_t phase_n[kPhases] = {};
    std::vector<std::pair<char *, size_t>> host_blocks;   // ft_host_alloc blocks (upload sources)
    // map edits: (hole, source) pairs written to a pinned ring that the move
    // kernel reads over the bus; an edit's chunk is reclaimed once the event
    // recorded after its kernels has completed (oldest first)
    struct EditChunk {
        size_t off, bytes;
        hipEvent_t ev;
    };
    static constexpr int kEditEvents = 64;
    char *edit_ring = nullptr;     // pinned
    char *d_edit_ring = nullptr;   // device mirror (same offsets) for staged batches of edits
    size_t edit_ring_bytes = 0, edit_head = 0;
    std::deque<EditChunk> edit_live;
    std::vector<hipEvent_t> edit_free_ev, edit_all_ev;
    std::vector<uint64_t> edit_marks;   // removed-slot bitmap of the edit being prepared (left all zero)
    // ORB detection: per-tile look-back state and a ticket counter, one set
    // per call in flight (round robin; a set is reused once the event after
    // its kernel ran).  The state is tagged with a per-set epoch and tickets
    // count on from a per-set base, so nothing is cleared between calls.
    static constexpr int kOrbSlots = 8;
    unsigned long long *orb_state[kOrbSlots] = {};
    uint32_t *orb_ticket[kOrbSlots] = {};
    uint32_t orb_epoch[kOrbSlots] = {};
    uint32_t orb_base[kOrbSlots] = {};
    hipEvent_t orb_ev[kOrbSlots] = {};
    bool orb_used[kOrbSlots] = {};
    int orb_next = 0;
};

namespace {

ft_status fail(ft_context *ctx, ft_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
        if (st == FT_ERR_DEVICE) ctx->sticky = FT_ERR_DEVICE;
    }
    return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, FT_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)


struct Bump {
    size_t off = 0;
    template <class T>
    T *take(char *base, size_t count)
    {
        off = align_up(off, 256);
        T *p = reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (count ? count : 1);
        return p;
    }
};

// Workspace of one search view: cell offsets, cell records (a keypoint in up
// to kMaxCellRep level bins), per-map-point candidates, claim table.
void carve_view(Slot &s, int v, char *base, Bump &b, size_t kp, size_t mp)
{
    s.view[v].cell_off = b.take<int32_t>(base, (size_t)kMaxCells + 1);
    s.view[v].crec = b.take<CellRec>(base, (size_t)kMaxCellRep * kp);
    s.view[v].mp_k = b.take<int32_t>(base, mp);
    s.view[v].mp_h = b.take<int32_t>(base, mp);
    s.view[v].claim = b.take<uint32_t>(base, kp);
    s.view[v].hist = b.take<int32_t>(base, kRotBinsMax);
}

void carve_slot(Slot &s, char *base, Bump &b, const ft_limits &L)
{
    const size_t kp = (size_t)L.max_kp_per_image, mp = (size_t)L.max_map_points;
    s.row_start = b.take<int32_t>(base, (size_t)kLevels * ((size_t)L.max_rows + 1));
    s.rrec = b.take<RowRec>(base, kp);
    s.tdesc = b.take<uint8_t>(base, 32 * kp);
    s.best_j = b.take<int32_t>(base, kp);
    s.best_h = b.take<int32_t>(base, kp);
    s.mrec = b.take<MatchRec>(base, kp);
    s.h2 = b.take<int32_t>(base, kp);
    s.sad = b.take<int32_t>(base, kp);
    s.flag = b.take<int32_t>(base, kp);
    s.qlist = b.take<int32_t>(base, kp);
    s.tlist = b.take<int32_t>(base, kp);
    s.counts = b.take<int32_t>(base, 16);
    s.uR = b.take<float>(base, kp);
    s.depth = b.take<float>(base, kp);
    s.xyz = b.take<float>(base, 3 * kp);
    s.claimR = b.take<uint32_t>(base, kp);
    for (int v = 0; v < 2; ++v) carve_view(s, v, base, b, kp, mp);
}

// Text of the last error of the context-free entry point on this thread.
thread_local char g_noalloc_err[256] = "";

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool valid_lanes(int g) { return g == 1 || g == 2 || g == 4 || g == 8 || g == 16; }

ft_status check_kps(ft_context *ctx, const ft_keypoints *k, const char *what)
{
    if (!k) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: null keypoints", what);
    if (k->n < 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: n < 0", what);
    if (k->n > ctx->lim.max_kp_per_image)
        return fail(ctx, FT_ERR_CAPACITY, "%s: %d keypoints exceed max_kp_per_image %d", what, k->n,
                    ctx->lim.max_kp_per_image);
    if (k->n > 0) {
        if (!k->x || !k->y || !k->octave || !k->desc)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: null array", what);
        if (!aligned(k->x, 4) || !aligned(k->y, 4) || !aligned(k->desc, 16))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: misaligned array", what);
    }
    return FT_OK;
}

ft_status check_scales(ft_context *ctx, const ft_scales *s)
{
    if (!s) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "null scales");
    if (s->n_levels != kLevels)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "scales: n_levels must be %d", kLevels);
    for (int l = 0; l < kLevels; ++l) {
        if (!(s->sf[l] > 0.0f) || !(s->inv_sf[l] > 0.0f) || !std::isfinite(s->sf[l]))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "scales: non-positive scale at level %d", l);
        if (l > 0 && !(s->sf[l] >= s->sf[l - 1]))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "scales: sf must be non-decreasing");
    }
    return FT_OK;
}

void fill_scales(DevJob &J, const ft_scales *s)
{
    for (int l = 0; l < kLevels; ++l) {
        J.sf[l] = s->sf[l];
        J.inv_sf[l] = s->inv_sf[l];
        J.sigma2[l] = s->sigma2[l];
    }
}

DevKps dev_kps(const ft_keypoints *k)
{
    DevKps d{};
    d.n = k->n;
    d.x = k->x;
    d.y = k->y;
    d.oct = k->octave;
    d.desc = k->desc;
    return d;
}

void bind_stereo_ws(DevJob &J, const Slot &s)
{
    J.row_start = s.row_start;
    J.rrec = s.rrec;
    J.tdesc = s.tdesc;
    J.best_j = s.best_j;
    J.best_h = s.best_h;
    J.mrec = s.mrec;
    J.h2 = s.h2;
    J.sad = s.sad;
    J.flag = s.flag;
    J.qlist = s.qlist;
    J.tlist = s.tlist;
    J.counts = s.counts;
    J.uR = s.uR;
    J.depth = s.depth;
    J.xyz = s.xyz;
    J.claimR = s.claimR;
}

// Level sizes and packed offsets of the pyramid of a width x height image.
bool pyramid_layout(int W, int H, const ft_scales *sc, ft_pyramid *pyr, int64_t *bytes)
{
    int64_t acc = 0;
    for (int l = 0; l < kLevels; ++l) {
        const float fw = (float)W * sc->inv_sf[l];
        const float fh = (float)H * sc->inv_sf[l];
        const int w = (int)std::floor(fw + 0.5f), h = (int)std::floor(fh + 0.5f);
        if (w < 1 || h < 1) return false;
        pyr->offset[l] = acc;
        pyr->width[l] = w;
        pyr->height[l] = h;
        acc += (int64_t)w * h;
    }
    *bytes = acc;
    return true;
}

// A level-0 image and the pyramid it is built into: sizes in range and the
// pyramid's levels exactly the packed layout.
ft_status check_pyramid_build(ft_context *ctx, const ft_image *img, const ft_scales *sc, const ft_pyramid *pyr,
                              const char *what)
{
    if (!img || !pyr) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: null image or pyramid", what);
    if (!img->data || !pyr->data) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: null image or pyramid data", what);
    if (img->width < 2 || img->height < 2 || img->pitch < img->width)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: image %dx%d pitch %d", what, img->width, img->height,
                    img->pitch);
    if (img->width > kMaxPyrW || img->height > kMaxRows)
        return fail(ctx, FT_ERR_CAPACITY, "%s: image %dx%d exceeds %dx%d", what, img->width, img->height, kMaxPyrW,
                    kMaxRows);
    ft_pyramid want{};
    int64_t bytes = 0;
    if (!pyramid_layout(img->width, img->height, sc, &want, &bytes))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: a pyramid level of the image would be empty", what);
    for (int l = 1; l < kLevels; ++l)   // levels shrink (the build stages at most kPyrRows + 1 rows per tile)
        if (want.width[l] > img->width || want.height[l] > img->height)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: pyramid level %d is larger than the image", what, l);
    for (int l = 0; l < kLevels; ++l)
        if (pyr->offset[l] != want.offset[l] || pyr->width[l] != want.width[l] || pyr->height[l] != want.height[l])
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: pyramid level %d is not the packed layout", what, l);
    return FT_OK;
}

void bind_pyramid_build(DevJob &J, const ft_image *L, const ft_image *R, const ft_pyramid *pl, const ft_pyramid *pr)
{
    J.imgL = L->data;
    J.imgR = R ? R->data : nullptr;
    J.pyr_outL = const_cast<uint8_t *>(pl->data);
    J.pyr_outR = pr ? const_cast<uint8_t *>(pr->data) : nullptr;
    J.img_w = L->width;
    J.img_h = L->height;
    J.img_pitch = L->pitch;
    for (int l = 0; l < kLevels; ++l) {
        J.lv_off[l] = pl->offset[l];
        J.lv_w[l] = pl->width[l];
        J.lv_h[l] = pl->height[l];
    }
}

ft_status build_pinhole(ft_context *ctx, DevJob &J, const ft_keypoints *L, const ft_keypoints *R,
                        const ft_pyramid *pl, const ft_pyramid *pr, const ft_scales *sc,
                        const ft_pinhole_stereo *cam, const ft_pinhole_params *p,
                        const ft_pinhole_out *o, const Slot &slot)
{
    ft_status st;
    if ((st = check_kps(ctx, L, "left")) || (st = check_kps(ctx, R, "right")) ||
        (st = check_scales(ctx, sc)))
        return st;
    if (!pl || !pr || !cam || !p || !o)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: null argument");
    if (!o->n_matches ||
        (L->n > 0 && (!o->right_idx || !o->dist || !o->u_right || !o->depth || !o->sad)))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: null output");
    if (!pl->data || !pr->data) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: null pyramid");
    if (cam->rows <= 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: rows <= 0");
    if (cam->rows > ctx->lim.max_rows)
        return fail(ctx, FT_ERR_CAPACITY, "pinhole: %d rows exceed max_rows %d", cam->rows,
                    ctx->lim.max_rows);
    if (!(cam->b > 0.0f) || !(cam->bf > 0.0f))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: baseline and bf must be > 0");
    if (p->half_win < 0 || p->half_win > 5)  /* (2w+1)^2 * 510 must stay below 2^16 */
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: half_win must be in [0, 5]");
    if (p->half_range < 1 || p->half_range > 31)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: half_range must be in [1, 31]");
    if (p->level_window < 0 || p->median_den <= 0 || p->median_num <= 0 || p->th_orb < 0)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: bad thresholds");
    if (!(p->band >= 0.0f) || !(p->band <= 64.0f))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: band must be in [0, 64]");
    for (int l = 0; l < kLevels; ++l) {
        if (pl->width[l] != pr->width[l] || pl->height[l] != pr->height[l] || pl->width[l] <= 0 ||
            pl->height[l] <= 0 || pl->offset[l] < 0 || pl->offset[l] != pr->offset[l])
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "pinhole: pyramid level %d mismatch", l);
    }
    J.flags |= JOB_STEREO_PINHOLE;
    J.L = dev_kps(L);
    J.R = dev_kps(R);
    fill_scales(J, sc);
    J.pyrL = pl->data;
    J.pyrR = pr->data;
    for (int l = 0; l < kLevels; ++l) {
        J.lv_off[l] = pl->offset[l];
        J.lv_w[l] = pl->width[l];
        J.lv_h[l] = pl->height[l];
    }
    J.bf = cam->bf;
    J.maxD = cam->bf / cam->b;
    J.band = p->band;
    J.rows = cam->rows;
    // a right keypoint whose band covers row r has its integer row within
    // ceil(band * sf_max) + 1 of r; one more bin absorbs the float rounding
    J.row_reach = (int)std::ceil(p->band * sc->sf[kLevels - 1]) + 2;
    // rows are binned per pyramid level when the (level, row) bins fit the
    // sort's LDS histogram: a query then scans only the levels of its window,
    // each over that level's own reach
    J.n_lb = (int64_t)kLevels * cam->rows <= kMaxCells ? kLevels : 1;
    for (int l = 0; l < kLevels; ++l)
        J.lv_reach[l] = J.n_lb == 1 ? J.row_reach : (int)std::ceil(p->band * sc->sf[l]) + 2;
    J.th_orb = p->th_orb;
    J.half_win = p->half_win;
    J.half_range = p->half_range;
    J.level_window = p->level_window;
    J.med_num = p->median_num;
    J.med_den = p->median_den;
    J.o_right_idx = o->right_idx;
    J.o_dist = o->dist;
    J.o_uR = o->u_right;
    J.o_depth = o->depth;
    J.o_sad = o->sad;
    J.o_nmatch = o->n_matches;
    bind_stereo_ws(J, slot);
    return FT_OK;
}

void kb8(float *dst, const ft_kb_intrinsics &k)
{
    dst[0] = k.fx; dst[1] = k.fy; dst[2] = k.cx; dst[3] = k.cy;
    for (int i = 0; i < 4; ++i) dst[4 + i] = k.k[i];
}

ft_status build_fisheye(ft_context *ctx, DevJob &J, const ft_keypoints *L, const ft_keypoints *R,
                        const ft_scales *sc, const ft_fisheye_stereo *cam,
                        const ft_fisheye_params *p, const ft_fisheye_out *o, const Slot &slot)
{
    ft_status st;
    if ((st = check_kps(ctx, L, "left")) || (st = check_kps(ctx, R, "right")) ||
        (st = check_scales(ctx, sc)))
        return st;
    if (!cam || !p || !o) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "fisheye: null argument");
    if (!o->n_matches || (L->n > 0 && (!o->right_idx || !o->dist || !o->depth || !o->xyz)))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "fisheye: null output");
    if (!(cam->overlap_left[0] <= cam->overlap_left[1]) || !(cam->overlap_right[0] <= cam->overlap_right[1]))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "fisheye: bad overlap range");
    if (p->ratio_den <= 0 || p->ratio_num <= 0 || p->newton_iters < 0 || p->newton_iters > 100)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "fisheye: bad parameters");
    if (!(cam->left.fx > 0.0f) || !(cam->left.fy > 0.0f) || !(cam->right.fx > 0.0f) || !(cam->right.fy > 0.0f))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "fisheye: focal lengths must be > 0");
    J.flags |= JOB_STEREO_FISHEYE;
    J.L = dev_kps(L);
    J.R = dev_kps(R);
    fill_scales(J, sc);
    kb8(J.kbL, cam->left);
    kb8(J.kbR, cam->right);
    memcpy(J.R_lr, cam->R_lr, sizeof J.R_lr);
    memcpy(J.t_lr, cam->t_lr, sizeof J.t_lr);
    J.ovl[0] = cam->overlap_left[0];
    J.ovl[1] = cam->overlap_left[1];
    J.ovr[0] = cam->overlap_right[0];
    J.ovr[1] = cam->overlap_right[1];
    J.ratio_num = p->ratio_num;
    J.ratio_den = p->ratio_den;
    J.newton_iters = p->newton_iters;
    J.cos_max = p->cos_parallax_max;
    J.chi2 = p->chi2;
    J.max_theta = p->max_theta;
    J.newton_tol = p->newton_tol;
    J.o_right_idx = o->right_idx;
    J.o_dist = o->dist;
    J.o_depth = o->depth;
    J.o_xyz = o->xyz;
    J.o_nmatch = o->n_matches;
    bind_stereo_ws(J, slot);
    return FT_OK;
}

ft_status check_search_common(ft_context *ctx, const ft_map_points *map, const ft_search_params *p)
{
    if (!map || !p) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: null argument");
    if (map->n < 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: map n < 0");
    if (map->n > ctx->lim.max_map_points)
        return fail(ctx, FT_ERR_CAPACITY, "search: %d map points exceed max_map_points %d", map->n,
                    ctx->lim.max_map_points);
    if (map->n > 0) {
        if (!map->pos || !map->normal || !map->dmin || !map->dmax || !map->desc)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: null map array");
        if (!aligned(map->pos, 4) || !aligned(map->normal, 4) || !aligned(map->desc, 16))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: misaligned map array");
    }
    if (p->th_high < 0 || p->th_high > 256 || p->ratio_den <= 0 || p->ratio_num < 0 ||
        p->level_lo < 0 || p->level_hi < 0 || !(p->th > 0.0f))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: bad parameters");
    return FT_OK;
}

void fill_search_common(DevJob &J, const ft_map_points *map, const ft_search_params *p)
{
    J.nM = map->n;
    J.pos = map->pos;
    J.normal = map->normal;
    J.dmin = map->dmin;
    J.dmax = map->dmax;
    J.mdesc = map->desc;
    J.th = p->th;
    J.cos_lim = p->view_cos_limit;
    J.cos_narrow = p->view_cos_narrow;
    J.r_narrow = p->r_narrow;
    J.r_wide = p->r_wide;
    J.dist_lo = p->dist_lo;
    J.dist_hi = p->dist_hi;
    J.lv_lo = p->level_lo;
    J.lv_hi = p->level_hi;
    J.th_high = p->th_high;
    J.s_ratio_num = p->ratio_num;
    J.s_ratio_den = p->ratio_den;
    J.same_level_only = p->ratio_same_level_only;
}

// Grid of a view's keypoint index.  When the level window spans at most
// kMaxCellRep octaves, the index holds one bin per predicted level with only
// the octaves that level's map points may match (a keypoint is copied into at
// most kMaxCellRep bins), and the caller's cells are merged by the smallest
// factor that fits kLevels bins into kMaxCells; otherwise it is the caller's
// grid with one bin.  The index only accelerates the search, which scans every
// cell that can hold a candidate, so the grid never changes a match.
void index_grid(const DevJob &J, int n, const ft_grid *grid, DevView &V)
{
    const int64_t rep = (int64_t)J.lv_lo + J.lv_hi + 1;
    V.n_pb = 1;
    V.cols = grid->cols;
    V.rows = grid->rows;
    if (rep > kMaxCellRep || rep * n > kMaxKp) return;
    int f = 1;
    while ((int64_t)kLevels * ((grid->cols + f - 1) / f) * ((grid->rows + f - 1) / f) > kMaxCells) ++f;
    V.n_pb = kLevels;
    V.cols = (grid->cols + f - 1) / f;
    V.rows = (grid->rows + f - 1) / f;
}

ft_status build_view(ft_context *ctx, DevJob &J, int v, int side, const ft_search_camera *cam,
                     const ft_keypoints *kps, const float *u_right, const uint8_t *pre,
                     const ft_grid *grid, const ft_search_out *o, const Slot &slot)
{
    ft_status st;
    if ((st = check_kps(ctx, kps, "search keypoints"))) return st;
    if (!cam || !grid || !o) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: null argument");
    if (!o->n_matches || (J.nM > 0 && (!o->mp_match || !o->mp_dist)) || (kps->n > 0 && !o->kp_match))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: null output");
    if (cam->model != FT_CAMERA_PINHOLE && cam->model != FT_CAMERA_KB)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: unknown camera model %d", cam->model);
    if (grid->cols <= 0 || grid->rows <= 0)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: grid must be positive");
    if ((int64_t)grid->cols * grid->rows > ctx->lim.max_grid_cells)
        return fail(ctx, FT_ERR_CAPACITY, "search: grid %dx%d exceeds max_grid_cells %d", grid->cols,
                    grid->rows, ctx->lim.max_grid_cells);
    if (!(cam->max_x > cam->min_x) || !(cam->max_y > cam->min_y))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "search: empty image bounds");
    if (u_right && !aligned(u_right, 4)) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "misaligned u_right");
    DevView &V = J.view[v];
    V.model = cam->model;
    index_grid(J, kps->n, grid, V);
    V.fx = cam->fx; V.fy = cam->fy; V.cx = cam->cx; V.cy = cam->cy; V.bf = cam->bf;
    for (int i = 0; i < 4; ++i) V.k[i] = cam->k[i];
    memcpy(V.R, cam->R, sizeof V.R);
    memcpy(V.t, cam->t, sizeof V.t);
    memcpy(V.O, cam->O, sizeof V.O);
    V.min_x = cam->min_x; V.max_x = cam->max_x; V.min_y = cam->min_y; V.max_y = cam->max_y;
    V.inv_cw = (float)V.cols / (cam->max_x - cam->min_x);
    V.inv_ch = (float)V.rows / (cam->max_y - cam->min_y);
    V.side = side;
    V.preassigned = pre;
    V.u_right = u_right;
    V.kdesc = kps->desc;
    V.mp_match = o->mp_match;
    V.mp_dist = o->mp_dist;
    V.kp_match = o->kp_match;
    V.n_matches = o->n_matches;
    V.cell_off = slot.view[v].cell_off;
    V.crec = slot.view[v].crec;
    V.mp_k = slot.view[v].mp_k;
    V.mp_h = slot.view[v].mp_h;
    V.claim = slot.view[v].claim;
    V.hist = slot.view[v].hist;
    J.flags |= (JOB_SEARCH0 << v);
    J.n_views = std::max(J.n_views, v + 1);
    if (side) J.R = dev_kps(kps);
    else J.L = dev_kps(kps);
    return FT_OK;
}

// ---------------------------------------------------------------- timing
constexpr size_t kEventSets = 64;

void drain_set(ft_context *ctx, size_t k)
{
    if (!ctx->ev_pending[k]) return;
    auto &ev = ctx->ev_sets[k];
    (void)hipEventSynchronize(ev[PH_COUNT]);   // a failure shows as a failed elapsed-time read below
    for (int p = 0; p < PH_COUNT; ++p) {
        if (!((ctx->ev_mask[k] >> p) & 1u)) continue;   // no kernel of this phase was launched
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[p], ev[p + 1]) == hipSuccess && ms > 0.0f) {
            ctx->phase_ms[p] += ms;
            ctx->phase_n[p] += 1;
        }
    }
    ctx->ev_pending[k] = 0;
}

// Event set for the next launch (nullptr when timing is off); only the phases
// with tiles are timed.
hipEvent_t *next_events(ft_context *ctx, const int32_t totals[PH_COUNT])
{
    if (!ctx->timing) return nullptr;
    const size_t k = ctx->ev_next;
    ctx->ev_next = (k + 1) % kEventSets;
    drain_set(ctx, k);
    ctx->ev_pending[k] = 1;
    uint32_t mask = 0;
    for (int p = 0; p < PH_COUNT; ++p)
        if (totals[p] > 0) mask |= 1u << p;
    ctx->ev_mask[k] = mask;
    return ctx->ev_sets[k].data();
}

ft_status set_timing(ft_context *ctx, bool enable)
{
    if (enable && ctx->ev_sets.empty()) {
        ctx->ev_sets.assign(kEventSets, std::vector<hipEvent_t>(kPhases + 1, nullptr));
        ctx->ev_pending.assign(kEventSets, 0);
        ctx->ev_mask.assign(kEventSets, 0);
        for (auto &set : ctx->ev_sets)
            for (auto &e : set) HIP_TRY(ctx, hipEventCreate(&e));
    }
    ctx->timing = enable;
    return FT_OK;
}

void read_timing(ft_context *ctx, double *ms, int64_t *n)
{
    for (size_t k = 0; k < ctx->ev_sets.size(); ++k) drain_set(ctx, k);
    for (int p = 0; p < kPhases; ++p) {
        ms[p] = ctx->phase_ms[p];
        n[p] = ctx->phase_n[p];
        ctx->phase_ms[p] = 0.0;
        ctx->phase_n[p] = 0;
    }
}

ft_status enter(ft_context *ctx)
{
    if (!ctx) return FT_ERR_INVALID_ARGUMENT;
    if (ctx->sticky) return ctx->sticky;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return fail(ctx, FT_ERR_DEVICE, "hipSetDevice(%d) failed", ctx->device);
    return FT_OK;
}

ft_status launch_one(ft_context *ctx, const DevJob &J, hipStream_t s, bool stereo, bool search)
{
    int32_t tot[PH_COUNT];
    job_tiles(J, ctx->shapes, stereo, search, tot);
    TileMap none{0, nullptr};
    HIP_TRY(ctx, launch_pipeline(nullptr, none, tot, J, ctx->shapes, s, next_events(ctx, tot)));
    return FT_OK;
}

// Validates every job of a batch into the lane's staging table.
ft_status build_batch(ft_context *ctx, Lane &lane, const ft_frame_job *jobs, int32_t n)
{
    ft_status st;
    DevJob *table = reinterpret_cast<DevJob *>(lane.h_table + ctx->layout.jobs_off);
    int64_t kp_total = 0, map_total = 0;
    for (int f = 0; f < n; ++f) {
        const ft_frame_job &jb = jobs[f];
        const bool stereo = jb.kind == FT_JOB_PINHOLE || jb.kind == FT_JOB_FISHEYE;
        kp_total += (stereo || jb.n_views > 0 ? (int64_t)jb.left.n : 0) + (stereo || jb.n_views > 1 ? (int64_t)jb.right.n : 0);
        map_total += jb.n_views > 0 ? (int64_t)jb.map.n : 0;
        DevJob &J = table[f];
        J = DevJob{};
        const Slot &slot = lane.slots[f];
        if (jb.kind == FT_JOB_PINHOLE) {
            if ((st = build_pinhole(ctx, J, &jb.left, &jb.right, &jb.pyr_left, &jb.pyr_right, &jb.scales,
                                    &jb.pinhole, &jb.pinhole_params, &jb.pinhole_out, slot)))
                return st;
            if (jb.build_pyramids) {
                if ((st = check_pyramid_build(ctx, &jb.image_left, &jb.scales, &jb.pyr_left, "left image")) ||
                    (st = check_pyramid_build(ctx, &jb.image_right, &jb.scales, &jb.pyr_right, "right image")))
                    return st;
                if (jb.image_left.width != jb.image_right.width || jb.image_left.height != jb.image_right.height ||
                    jb.image_left.pitch != jb.image_right.pitch)
                    return fail(ctx, FT_ERR_INVALID_ARGUMENT, "batch: job %d stereo images differ in size or pitch", f);
                bind_pyramid_build(J, &jb.image_left, &jb.image_right, &jb.pyr_left, &jb.pyr_right);
            }
        } else if (jb.kind == FT_JOB_FISHEYE) {
            if ((st = build_fisheye(ctx, J, &jb.left, &jb.right, &jb.scales, &jb.fisheye,
                                    &jb.fisheye_params, &jb.fisheye_out, slot)))
                return st;
        } else if (jb.kind == FT_JOB_SEARCH) {
            if ((st = check_scales(ctx, &jb.scales))) return st;
            fill_scales(J, &jb.scales);
        } else {
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "batch: job %d has unknown kind %d", f, jb.kind);
        }
        if (jb.n_views < 0 || jb.n_views > 2)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "batch: job %d n_views must be 0..2", f);
        if (jb.n_views > 0) {
            if ((st = check_search_common(ctx, &jb.map, &jb.search_params))) return st;
            fill_search_common(J, &jb.map, &jb.search_params);
        }
        for (int v = 0; v < jb.n_views; ++v) {
            const ft_keypoints *kps = v == 0 ? &jb.left : &jb.right;
            const float *ur = (v == 0 && jb.kind == FT_JOB_PINHOLE && jb.use_u_right)
                                  ? jb.pinhole_out.u_right : nullptr;
            if ((st = build_view(ctx, J, v, v, &jb.cam[v], kps, ur, jb.preassigned[v], &jb.grid[v],
                                 &jb.search_out[v], slot)))
                return st;
        }
    }
    if (kp_total > ctx->batch_kp_cap)
        return fail(ctx, FT_ERR_CAPACITY, "batch: %lld keypoints exceed max_batch_kp_total %lld",
                    (long long)kp_total, (long long)ctx->batch_kp_cap);
    if (map_total > ctx->batch_map_cap)
        return fail(ctx, FT_ERR_CAPACITY, "batch: %lld map points exceed max_batch_map_total %lld",
                    (long long)map_total, (long long)ctx->batch_map_cap);
    return FT_OK;
}

// Tile prefixes of every phase into the lane's staging table; returns the totals.
void plan_batch(ft_context *ctx, Lane &lane, int32_t n, const Shapes &sh, int32_t totals[PH_COUNT])
{
    const DevJob *table = reinterpret_cast<const DevJob *>(lane.h_table + ctx->layout.jobs_off);
    int32_t *pre = reinterpret_cast<int32_t *>(lane.h_table + ctx->layout.prefix_off);
    for (int p = 0; p < PH_COUNT; ++p) {
        pre[p * (n + 1)] = 0;
        totals[p] = 0;
    }
    for (int f = 0; f < n; ++f) {
        int32_t t[PH_COUNT];
        job_tiles(table[f], sh, true, true, t);
        for (int p = 0; p < PH_COUNT; ++p) {
            totals[p] += t[p];
            pre[p * (n + 1) + f + 1] = totals[p];
        }
    }
}

Lane *free_lane(ft_context *ctx, int *id, ft_status *st)
{
    *st = FT_OK;
    for (size_t i = 0; i < ctx->lanes.size(); ++i) {
        Lane &ln = ctx->lanes[i];
        if (!ln.used) { *id = (int)i; return &ln; }
        const hipError_t q = hipEventQuery(ln.done);
        if (q == hipSuccess) { *id = (int)i; return &ln; }
        if (q != hipErrorNotReady) {
            *st = fail(ctx, FT_ERR_DEVICE, "batch: event query failed: %s", hipGetErrorString(q));
            return nullptr;
        }
    }
    *st = fail(ctx, FT_ERR_CAPACITY, "batch: all %zu in-flight slots busy", ctx->lanes.size());
    return nullptr;
}

BatchArgs batch_args(const ft_context *ctx, const Lane &lane, int32_t n)
{
    const char *dtab = lane.d_table;
    return BatchArgs{reinterpret_cast<const DevJob *>(dtab + ctx->layout.jobs_off),
                     TileMap{n, reinterpret_cast<const int32_t *>(dtab + ctx->layout.prefix_off)}};
}

// Uploads the lane's staged table and launches one kernel per phase.
ft_status launch_batch(ft_context *ctx, Lane &lane, int32_t n, const Shapes &sh, hipStream_t s,
                       const int32_t totals[PH_COUNT], hipEvent_t *ev)
{
    HIP_TRY(ctx, hipMemcpyAsync(lane.d_table, lane.h_table, ctx->layout.upload_bytes(n), hipMemcpyHostToDevice, s));
    const BatchArgs a = batch_args(ctx, lane, n);
    const DevJob *staged = reinterpret_cast<const DevJob *>(lane.h_table + ctx->layout.jobs_off);
    HIP_TRY(ctx, launch_pipeline(a.p, a.map, totals, staged[0], sh, s, ev));
    return FT_OK;
}

void release_graph(BatchGraph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = BatchGraph{};
}

// Builds and instantiates the lane's batch graph for the context's shapes:
// table upload -> setup -> best match -> refinement -> triangulation ->
// stereo resolve -> search -> search resolve.  The grids (one workgroup) and
// arguments are placeholders that every submission replaces.
ft_status build_graph(ft_context *ctx, Lane &lane)
{
    release_graph(lane.g);
    BatchGraph &g = lane.g;
    HIP_TRY(ctx, hipGraphCreate(&g.graph, 0));
    HIP_TRY(ctx, hipGraphAddMemcpyNode1D(&g.copy, g.graph, nullptr, 0, lane.d_table, lane.h_table,
                                         ctx->layout.upload_bytes(1), hipMemcpyHostToDevice));
    batch_kernels(ctx->shapes, g.fn, g.block);
    BatchArgs a = batch_args(ctx, lane, 1);
    void *args[] = {&a};
    hipGraphNode_t prev = g.copy;
    for (int p = 0; p < PH_COUNT; ++p) {
        hipKernelNodeParams kp{};
        kp.func = g.fn[p];
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(g.block[p]);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        HIP_TRY(ctx, hipGraphAddKernelNode(&g.kern[p], g.graph, &prev, 1, &kp));
        prev = g.kern[p];
    }
    HIP_TRY(ctx, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    return FT_OK;
}

// Builds every lane's graph for the current shapes, after the lanes' batches
// in flight have finished.
ft_status rebuild_graphs(ft_context *ctx)
{
    for (auto &ln : ctx->lanes)
        if (ln.used) HIP_TRY(ctx, hipEventSynchronize(ln.done));
    for (auto &ln : ctx->lanes) {
        const ft_status st = build_graph(ctx, ln);
        if (st) return st;
    }
    return FT_OK;
}

// Launches the lane's graph for this batch: the table upload size and, for
// every phase whose grid or job count changed, the kernel node's grid and
// argument are set in the instantiated graph first.  The node of a phase
// without tiles is disabled for the launch (it then orders nothing and runs
// nothing).
ft_status launch_batch_graph(ft_context *ctx, Lane &lane, int32_t n, hipStream_t s,
                             const int32_t totals[PH_COUNT])
{
    BatchGraph &g = lane.g;
    if (!g.exec) return fail(ctx, FT_ERR_DEVICE, "batch graph missing");
    HIP_TRY(ctx, hipGraphExecMemcpyNodeSetParams1D(g.exec, g.copy, lane.d_table, lane.h_table,
                                                   ctx->layout.upload_bytes(n), hipMemcpyHostToDevice));
    BatchArgs a = batch_args(ctx, lane, n);
    void *args[] = {&a};
    for (int p = 0; p < PH_COUNT; ++p) {
        const bool off = totals[p] <= 0;
        if (off != g.off[p]) {
            HIP_TRY(ctx, hipGraphNodeSetEnabled(g.exec, g.kern[p], off ? 0u : 1u));
            g.off[p] = off;
        }
        if (off) continue;
        const int32_t grid = totals[p];
        if (grid == g.grid[p] && n == g.n[p]) continue;
        hipKernelNodeParams kp{};
        kp.func = g.fn[p];
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(g.block[p]);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        HIP_TRY(ctx, hipGraphExecKernelNodeSetParams(g.exec, g.kern[p], &kp));
        g.grid[p] = grid;
        g.n[p] = n;
    }
    HIP_TRY(ctx, hipGraphLaunch(g.exec, s));
    return FT_OK;
}

// ---------------------------------------------------------------- autotune
std::string workload_key(const ft_frame_job *jobs, int32_t n, const char *arch)
{
    double kp = 0, mp = 0;
    int pin = 0, fish = 0;
    for (int f = 0; f < n; ++f) {
        kp += jobs[f].left.n;
        mp += jobs[f].map.n;
        pin += jobs[f].kind == FT_JOB_PINHOLE;
        fish += jobs[f].kind == FT_JOB_FISHEYE;
    }
    auto p2 = [](double v) { return v <= 1 ? 0 : (int)std::lround(std::log2(v)); };
    std::ostringstream os;
    os << arch << ":frames=" << n << ":pinhole=" << pin << ":fisheye=" << fish
       << ":kp2=" << p2(kp / std::max(n, 1)) << ":map2=" << p2(mp / std::max(n, 1));
    return os.str();
}

bool cache_lookup(const std::string &path, const std::string &key, Shapes &out)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string tag = "\"key\": \"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(tag) == std::string::npos) continue;
        const size_t pb = line.find("\"best_lanes\": "), ps = line.find("\"search_lanes\": ");
        const size_t pa = line.find("\"aux_block\": ");
        if (pb == std::string::npos || ps == std::string::npos || pa == std::string::npos) continue;
        const int b = std::atoi(line.c_str() + pb + 14);
        const int s = std::atoi(line.c_str() + ps + 16);
        const int ka = std::atoi(line.c_str() + pa + 13);
        if (valid_lanes(b) && valid_lanes(s) && (ka == kWG || ka == kAuxWG)) {
            out.best_lanes = b;
            out.search_lanes = s;
            out.aux_block = ka;
            return true;
        }
    }
    return false;
}

bool cache_append(const std::string &path, const std::string &key, const Shapes &sh, double us)
{
    // one JSON object per line, so entries can be appended and grepped
    std::ofstream f(path, std::ios::app);
    if (!f) return false;
    f << "{\"key\": \"" << key << "\", \"best_lanes\": " << sh.best_lanes
      << ", \"search_lanes\": " << sh.search_lanes << ", \"aux_block\": " << sh.aux_block
      << ", \"us\": " << us << "}\n";
    return (bool)f;
}

void to_public(const Shapes &sh, ft_shapes *s)
{
    s->best_lanes = sh.best_lanes;
    s->search_lanes = sh.search_lanes;
    s->aux_block = sh.aux_block;
}

}  // namespace

extern "C" {

int32_t ft_version(void) { return 300; }

const char *ft_status_string(ft_status s)
{
    switch (s) {
    case FT_OK: return "ok";
    case FT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FT_ERR_CAPACITY: return "capacity exceeded";
    case FT_ERR_DEVICE: return "device error";
    case FT_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *ft_last_error(const ft_context *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_noalloc_err[0] ? g_noalloc_err : "null context";
}

ft_status ft_context_create(const ft_limits *lim, int32_t device, ft_context **out)
{
    if (!lim || !out) return FT_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (lim->max_kp_per_image < 1 || lim->max_kp_per_image > kMaxKp || lim->max_map_points < 1 ||
        lim->max_map_points > kMaxMap || lim->max_rows < 1 || lim->max_rows > kMaxRows ||
        lim->max_grid_cells < 1 || lim->max_grid_cells > kMaxCells || lim->max_batch_frames < 1 ||
        lim->max_batch_frames > 4096 || lim->max_inflight < 1 || lim->max_inflight > 64 ||
        lim->max_levels != kLevels || lim->max_batch_kp_total < 0 || lim->max_batch_map_total < 0)
        return FT_ERR_INVALID_ARGUMENT;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FT_ERR_DEVICE;
    if (device < 0 || device >= ndev) return FT_ERR_INVALID_ARGUMENT;
    if (hipSetDevice(device) != hipSuccess) return FT_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FT_ERR_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FT_ERR_UNSUPPORTED;

    ft_context *ctx = new ft_context();
    ctx->device = device;
    ctx->lim = *lim;
    ctx->batch_kp_cap = lim->max_batch_kp_total ? lim->max_batch_kp_total
                                                : (int64_t)lim->max_batch_frames * 2 * lim->max_kp_per_image;
    ctx->batch_map_cap = lim->max_batch_map_total ? lim->max_batch_map_total
                                                  : (int64_t)lim->max_batch_frames * lim->max_map_points;
    ctx->layout = table_layout(lim->max_batch_frames);
    Bump b;
    Slot tmp;
    carve_slot(tmp, nullptr, b, *lim);
    const size_t slot_bytes = align_up(b.off, 256);
    const size_t n_slots = 1 + (size_t)lim->max_inflight * lim->max_batch_frames;
    const size_t edit_bytes = align_up(sizeof(int32_t) * 2 * (size_t)lim->max_map_points, 256);
    const size_t orb_bytes = align_up(sizeof(unsigned long long) * (size_t)kOrbMaxTiles + 256, 256);
    ctx->edit_ring_bytes = std::max<size_t>(2 * edit_bytes, (size_t)8 << 20);
    ctx->bytes = slot_bytes * n_slots + ctx->layout.total * lim->max_inflight + orb_bytes * ft_context::kOrbSlots +
                 ctx->edit_ring_bytes;
    if (hipMalloc((void **)&ctx->base, ctx->bytes) != hipSuccess) {
        delete ctx;
        return FT_ERR_DEVICE;
    }
    size_t off = 0;
    auto carve_at = [&](Slot &s) {
        Bump bb;
        carve_slot(s, ctx->base + off, bb, *lim);
        off += slot_bytes;
    };
    carve_at(ctx->direct);
    for (int k = 0; k < ft_context::kOrbSlots; ++k) {
        ctx->orb_state[k] = reinterpret_cast<unsigned long long *>(ctx->base + off);
        ctx->orb_ticket[k] = reinterpret_cast<uint32_t *>(ctx->base + off + orb_bytes - 256);
        if (hipMemset(ctx->base + off, 0, orb_bytes) != hipSuccess ||   // epoch 0 is never used
            hipEventCreateWithFlags(&ctx->orb_ev[k], hipEventDisableTiming) != hipSuccess) {
            ft_context_destroy(ctx);
            return FT_ERR_DEVICE;
        }
        off += orb_bytes;
    }
    ctx->d_edit_ring = ctx->base + off;
    off += ctx->edit_ring_bytes;
    if (hipHostMalloc((void **)&ctx->edit_ring, ctx->edit_ring_bytes, hipHostMallocDefault) != hipSuccess) {
        ft_context_destroy(ctx);
        return FT_ERR_DEVICE;
    }
    for (int k = 0; k < ft_context::kEditEvents; ++k) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            ft_context_destroy(ctx);
            return FT_ERR_DEVICE;
        }
        ctx->edit_all_ev.push_back(e);
        ctx->edit_free_ev.push_back(e);
    }
    ctx->lanes.resize(lim->max_inflight);
    for (auto &ln : ctx->lanes) {
        ln.slots.resize(lim->max_batch_frames);
        for (auto &s : ln.slots) carve_at(s);
        ln.d_table = ctx->base + off;
        off += ctx->layout.total;
        if (hipHostMalloc((void **)&ln.h_table, ctx->layout.total, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
            ft_context_destroy(ctx);
            return FT_ERR_DEVICE;
        }
        memset(ln.h_table, 0, ctx->layout.total);
    }
    // every lane's batch graph, so that no submission instantiates one
    if (rebuild_graphs(ctx) != FT_OK) {
        ft_context_destroy(ctx);
        return FT_ERR_DEVICE;
    }
    *out = ctx;
    return FT_OK;
}

ft_status ft_context_enable_timing(ft_context *ctx, int32_t enable)
{
    ft_status st = enter(ctx);
    if (st) return st;
    return set_timing(ctx, enable != 0);
}

ft_status ft_context_read_timing(ft_context *ctx, double *ms, int64_t *launches)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!ms || !launches) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "read_timing: null output");
    read_timing(ctx, ms, launches);
    return FT_OK;
}

ft_status ft_context_destroy(ft_context *ctx)
{
    if (!ctx) return FT_ERR_INVALID_ARGUMENT;
    // Best effort: every resource is released whatever an earlier call
    // returned, so the individual results are not checked.
    (void)hipSetDevice(ctx->device);
    for (auto &set : ctx->ev_sets)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    for (auto &ln : ctx->lanes) {
        if (ln.done) {
            (void)hipEventSynchronize(ln.done);
            (void)hipEventDestroy(ln.done);
        }
        release_graph(ln.g);
        if (ln.h_table) (void)hipHostFree(ln.h_table);
    }
    for (int k = 0; k < ft_context::kOrbSlots; ++k)
        if (ctx->orb_ev[k]) {
            (void)hipEventSynchronize(ctx->orb_ev[k]);
            (void)hipEventDestroy(ctx->orb_ev[k]);
        }
    for (auto &c : ctx->edit_live) (void)hipEventSynchronize(c.ev);
    for (hipEvent_t e : ctx->edit_all_ev) (void)hipEventDestroy(e);
    if (ctx->edit_ring) (void)hipHostFree(ctx->edit_ring);
    if (ctx->base || !ctx->host_blocks.empty()) (void)hipDeviceSynchronize();
    for (auto &hb : ctx->host_blocks) (void)hipHostFree(hb.first);
    if (ctx->base) (void)hipFree(ctx->base);
    delete ctx;
    return FT_OK;
}

ft_status ft_host_alloc(ft_context *ctx, int64_t bytes, void **ptr)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!ptr || bytes <= 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "host_alloc: null ptr or size %lld", (long long)bytes);
    *ptr = nullptr;
    char *p = nullptr;
    HIP_TRY(ctx, hipHostMalloc((void **)&p, (size_t)bytes, hipHostMallocDefault));
    ctx->host_blocks.emplace_back(p, (size_t)bytes);
    *ptr = p;
    return FT_OK;
}

ft_status ft_host_free(ft_context *ctx, void *ptr)
{
    if (!ctx) return FT_ERR_INVALID_ARGUMENT;
    for (size_t i = 0; i < ctx->host_blocks.size(); ++i) {
        if (ctx->host_blocks[i].first != ptr) continue;
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipHostFree(ptr));
        ctx->host_blocks.erase(ctx->host_blocks.begin() + (ptrdiff_t)i);
        return FT_OK;
    }
    return fail(ctx, FT_ERR_INVALID_ARGUMENT, "host_free: %p is not a live ft_host_alloc block", ptr);
}

// Largest segment: keeps a launch's workgroup count (<= kUploadSegs segments)
// far below the grid limit.
constexpr int64_t kMaxUploadBytes = int64_t(1) << 36;

ft_status ft_upload(ft_context *ctx, void *stream, const ft_segment *segs, int32_t n)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (n < 0 || (n > 0 && !segs)) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "upload: %d segments, list %p", n, (const void *)segs);
    // validate everything before enqueueing anything
    for (int32_t i = 0; i < n; ++i) {
        const ft_segment &g = segs[i];
        const uintptr_t src = (uintptr_t)g.src, dst = (uintptr_t)g.dst;
        if (g.bytes < 0 || g.bytes > kMaxUploadBytes || !g.src || !g.dst || (src & 15) || (dst & 15))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "upload: segment %d null, misaligned or of size %lld", i,
                        (long long)g.bytes);
        bool inside = false;
        for (const auto &hb : ctx->host_blocks) {
            const uintptr_t b0 = (uintptr_t)hb.first;
            if (src >= b0 && src - b0 <= hb.second && (uint64_t)g.bytes <= hb.second - (src - b0)) {
                inside = true;
                break;
            }
        }
        if (!inside) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "upload: segment %d source outside every ft_host_alloc block", i);
    }
    hipStream_t s = (hipStream_t)stream;
    for (int32_t g0 = 0; g0 < n; g0 += kUploadSegs) {
        UploadArgs a{};
        a.n = std::min(kUploadSegs, n - g0);
        int64_t blocks = 0;
        for (int k = 0; k < a.n; ++k) {
            const ft_segment &g = segs[g0 + k];
            a.first[k] = (int32_t)blocks;
            a.src[k] = static_cast<const char *>(g.src);
            a.dst[k] = static_cast<char *>(g.dst);
            a.bytes[k] = g.bytes;
            blocks += (g.bytes + kUploadChunk - 1) / kUploadChunk;
        }
        a.first[a.n] = (int32_t)blocks;
        HIP_TRY(ctx, launch_upload(a, s));
    }
    return FT_OK;
}

ft_status ft_context_workspace_bytes(const ft_context *ctx, int64_t *bytes)
{
    if (!ctx || !bytes) return FT_ERR_INVALID_ARGUMENT;
    *bytes = (int64_t)ctx->bytes;
    return FT_OK;
}

ft_status ft_set_shapes(ft_context *ctx, const ft_shapes *s)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!s) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "shapes: null");
    if (!valid_lanes(s->best_lanes) || !valid_lanes(s->search_lanes))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "shapes: lanes must be 1, 2, 4, 8 or 16");
    if (s->aux_block != kWG && s->aux_block != kAuxWG)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "shapes: aux_block must be %d or %d", kWG, kAuxWG);
    Shapes sh;
    sh.best_lanes = s->best_lanes;
    sh.search_lanes = s->search_lanes;
    sh.aux_block = s->aux_block;
    if (sh == ctx->shapes) return FT_OK;
    ctx->shapes = sh;
    return rebuild_graphs(ctx);
}

ft_status ft_set_exec_mode(ft_context *ctx, int32_t mode)
{
    if (!ctx) return FT_ERR_INVALID_ARGUMENT;
    if (mode != FT_EXEC_EAGER && mode != FT_EXEC_GRAPH)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "exec mode %d unknown", mode);
    ctx->exec_mode = mode;
    return FT_OK;
}

ft_status ft_get_exec_mode(const ft_context *ctx, int32_t *mode)
{
    if (!ctx || !mode) return FT_ERR_INVALID_ARGUMENT;
    *mode = ctx->exec_mode;
    return FT_OK;
}

ft_status ft_get_shapes(const ft_context *ctx, ft_shapes *s)
{
    if (!ctx || !s) return FT_ERR_INVALID_ARGUMENT;
    to_public(ctx->shapes, s);
    return FT_OK;
}

ft_status ft_stereo_match_pinhole(ft_context *ctx, void *stream, const ft_keypoints *left,
                                  const ft_keypoints *right, const ft_pyramid *pyr_left,
                                  const ft_pyramid *pyr_right, const ft_scales *scales,
                                  const ft_pinhole_stereo *cam, const ft_pinhole_params *params,
                                  const ft_pinhole_out *out)
{
    ft_status st = enter(ctx);
    if (st) return st;
    DevJob J{};
    if ((st = build_pinhole(ctx, J, left, right, pyr_left, pyr_right, scales, cam, params, out,
                            ctx->direct)))
        return st;
    return launch_one(ctx, J, (hipStream_t)stream, true, false);
}

ft_status ft_stereo_match_fisheye(ft_context *ctx, void *stream, const ft_keypoints *left,
                                  const ft_keypoints *right, const ft_scales *scales,
                                  const ft_fisheye_stereo *cam, const ft_fisheye_params *params,
                                  const ft_fisheye_out *out)
{
    ft_status st = enter(ctx);
    if (st) return st;
    DevJob J{};
    if ((st = build_fisheye(ctx, J, left, right, scales, cam, params, out, ctx->direct))) return st;
    return launch_one(ctx, J, (hipStream_t)stream, true, false);
}

ft_status ft_search_local_points(ft_context *ctx, void *stream, const ft_map_points *map,
                                 const ft_search_camera *cam, const ft_keypoints *kps,
                                 const float *u_right, const uint8_t *preassigned,
                                 const ft_grid *grid, const ft_scales *scales,
                                 const ft_search_params *params, const ft_search_out *out)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if ((st = check_scales(ctx, scales)) || (st = check_search_common(ctx, map, params))) return st;
    DevJob J{};
    fill_scales(J, scales);
    fill_search_common(J, map, params);
    if ((st = build_view(ctx, J, 0, 0, cam, kps, u_right, preassigned, grid, out, ctx->direct))) return st;
    return launch_one(ctx, J, (hipStream_t)stream, false, true);
}

ft_status ft_search_local_points_noalloc(void *stream, const ft_map_points *map,
                                         const ft_search_camera *cam, const ft_keypoints *kps,
                                         const float *u_right, const uint8_t *preassigned,
                                         const ft_grid *grid, const ft_scales *scales,
                                         const ft_search_params *params, const ft_search_out *out)
{
    g_noalloc_err[0] = 0;
    // a context on the host stack carries the limits the validators check and
    // the error text; it owns no device memory
    ft_context tmp;
    auto done = [&](ft_status st) {
        if (st) snprintf(g_noalloc_err, sizeof g_noalloc_err, "%s", tmp.err.c_str());
        return st;
    };
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return done(fail(&tmp, FT_ERR_DEVICE, "noalloc: hipGetDevice failed"));
    tmp.device = dev;
    tmp.lim.max_kp_per_image = FT_NOALLOC_MAX_KP;
    tmp.lim.max_map_points = FT_NOALLOC_MAX_MAP;
    tmp.lim.max_rows = kMaxRows;
    tmp.lim.max_grid_cells = kMaxCells;
    tmp.lim.max_batch_frames = 1;
    tmp.lim.max_inflight = 1;
    tmp.lim.max_levels = kLevels;
    ft_status st;
    if ((st = check_scales(&tmp, scales)) || (st = check_search_common(&tmp, map, params))) return done(st);
    bool gfx950 = false;
    char *base = nullptr;
    const hipError_t e = noalloc_scratch(dev, &base, &gfx950);
    if (e != hipSuccess)
        return done(fail(&tmp, FT_ERR_DEVICE, "noalloc: device scratch lookup failed: %s", hipGetErrorString(e)));
    if (!gfx950) return done(fail(&tmp, FT_ERR_UNSUPPORTED, "noalloc: device %d is not gfx950", dev));
    Slot slot{};
    Bump b;
    carve_view(slot, 0, base, b, FT_NOALLOC_MAX_KP, FT_NOALLOC_MAX_MAP);
    if (b.off > kNoallocScratchBytes)
        return done(fail(&tmp, FT_ERR_UNSUPPORTED, "noalloc: workspace %zu B exceeds the %zu B scratch", b.off,
                         kNoallocScratchBytes));
    DevJob J{};
    fill_scales(J, scales);
    fill_search_common(J, map, params);
    if ((st = build_view(&tmp, J, 0, 0, cam, kps, u_right, preassigned, grid, out, slot))) return done(st);
    return done(launch_one(&tmp, J, (hipStream_t)stream, false, true));
}

ft_status ft_pyramid_layout(int32_t width, int32_t height, const ft_scales *scales, ft_pyramid *pyr,
                            int64_t *bytes)
{
    if (!scales || !pyr || !bytes || scales->n_levels != kLevels) return FT_ERR_INVALID_ARGUMENT;
    if (width < 1 || height < 1 || width > 65536 || height > 65536) return FT_ERR_INVALID_ARGUMENT;
    ft_pyramid p{};
    int64_t b = 0;
    if (!pyramid_layout(width, height, scales, &p, &b)) return FT_ERR_INVALID_ARGUMENT;
    for (int l = 0; l < kLevels; ++l) {
        pyr->offset[l] = p.offset[l];
        pyr->width[l] = p.width[l];
        pyr->height[l] = p.height[l];
    }
    *bytes = b;
    return FT_OK;
}

ft_status ft_build_pyramid(ft_context *ctx, void *stream, const ft_image *image, const ft_scales *scales,
                           const ft_pyramid *pyr)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if ((st = check_scales(ctx, scales)) || (st = check_pyramid_build(ctx, image, scales, pyr, "pyramid")))
        return st;
    DevJob J{};
    fill_scales(J, scales);
    bind_pyramid_build(J, image, nullptr, pyr, nullptr);
    return launch_one(ctx, J, (hipStream_t)stream, true, false);
}

ft_status ft_search_last_frame(ft_context *ctx, void *stream, const ft_last_points *last,
                               const ft_search_camera *cam, const ft_keypoints *kps, const float *kp_angle,
                               const float *u_right, const uint8_t *preassigned, const ft_grid *grid,
                               const ft_scales *scales, const ft_last_params *params,
                               const ft_search_out *out)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if ((st = check_scales(ctx, scales))) return st;
    if (!last || !params || !kps) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: null argument");
    if (last->n < 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: n < 0");
    if (last->n > ctx->lim.max_map_points)
        return fail(ctx, FT_ERR_CAPACITY, "last frame: %d points exceed max_map_points %d", last->n,
                    ctx->lim.max_map_points);
    const bool rot = params->check_orientation != 0;
    if (!(params->th > 0.0f) || params->th_high < 0 || params->th_high > 256 || params->direction < -1 ||
        params->direction > 1 || params->check_orientation < 0 || params->check_orientation > 1 ||
        params->bins < 1 || params->bins > kRotBinsMax)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: bad parameters");
    if (last->n > 0) {
        if (!last->pos || !last->desc || !last->octave || (rot && !last->angle))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: null point array");
        if (!aligned(last->pos, 4) || !aligned(last->desc, 16) || (last->angle && !aligned(last->angle, 4)))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: misaligned point array");
    }
    if (rot && kps->n > 0 && (!kp_angle || !aligned(kp_angle, 4)))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "last frame: null or misaligned keypoint angles");
    DevJob J{};
    fill_scales(J, scales);
    J.nM = last->n;
    J.pos = last->pos;
    J.mdesc = last->desc;
    J.l_oct = last->octave;
    J.l_ang = last->angle;
    J.k_ang = kp_angle;
    J.th = params->th;
    J.th_high = params->th_high;
    J.direction = params->direction;
    J.check_rot = rot ? 1 : 0;
    J.rot_bins = params->bins;
    // the window's levels are not centred on a predicted level: one-bin index
    J.lv_lo = kLevels;
    J.lv_hi = kLevels;
    if ((st = build_view(ctx, J, 0, 0, cam, kps, u_right, preassigned, grid, out, ctx->direct))) return st;
    HIP_TRY(ctx, launch_last_frame(J, 4, (hipStream_t)stream));
    return FT_OK;
}

namespace {

// One validated map edit: the removed slots (ascending), the (hole, source)
// pairs, and the new count; nothing is changed until it is committed.
struct PreparedEdit {
    int n1 = 0, m = 0, n_holes = 0;
    std::vector<int32_t> rem, pairs;
};

ft_status prepare_edit(ft_context *ctx, const ft_map_points *map, int32_t capacity, const ft_map_edit *edit,
                       PreparedEdit &pe)
{
    if (!map || !edit) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: null argument");
    const int n = map->n, nr = edit->n_remove, m = edit->insert.n;
    if (n < 0 || capacity < n || capacity > kMaxMap || nr < 0 || m < 0)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: n %d, capacity %d, %d removed, %d inserted", n,
                    capacity, nr, m);
    if (nr > ctx->lim.max_map_points || m > ctx->lim.max_map_points)
        return fail(ctx, FT_ERR_CAPACITY, "map update: %d removed / %d inserted exceed max_map_points %d", nr, m,
                    ctx->lim.max_map_points);
    if (nr > 0 && !edit->remove) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: null removal list");
    auto arrays_ok = [](const ft_map_points &p) {
        return p.pos && p.normal && p.dmin && p.dmax && p.desc && aligned(p.pos, 4) && aligned(p.normal, 4) &&
               aligned(p.dmin, 4) && aligned(p.dmax, 4) && aligned(p.desc, 16);
    };
    if (capacity > 0 && !arrays_ok(*map))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: null or misaligned map array");
    if (m > 0 && !arrays_ok(edit->insert))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: null or misaligned insert array");
    if (m > 0) {
        // host insert arrays: every one wholly inside an ft_host_alloc block
        const ft_map_points &q = edit->insert;
        const void *ptr[5] = {q.pos, q.normal, q.dmin, q.dmax, q.desc};
        const size_t len[5] = {12 * (size_t)m, 12 * (size_t)m, 4 * (size_t)m, 4 * (size_t)m, 32 * (size_t)m};
        int in_host = 0, touches = 0;
        for (int f = 0; f < 5; ++f) {
            const uintptr_t p0 = (uintptr_t)ptr[f];
            for (const auto &hb : ctx->host_blocks) {
                const uintptr_t b0 = (uintptr_t)hb.first;
                if (p0 >= b0 && p0 - b0 < hb.second) {
                    ++touches;
                    if (len[f] <= hb.second - (p0 - b0)) ++in_host;
                    break;
                }
            }
        }
        if (touches != 0 && (touches != 5 || in_host != 5))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT,
                        "map update: host insert arrays must all lie wholly inside ft_host_alloc blocks");
    }
    const ft_map_ids *rec = edit->ids;
    std::vector<int32_t> &rem = pe.rem;
    rem.assign(edit->remove, edit->remove + nr);
    if (rec) {
        // removals named by point id: their slots from the record
        if (!rec->slot_id || !rec->slot_of || rec->id_count < 0 || (m > 0 && !edit->insert_ids))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: incomplete id record");
        for (int i = 0; i < nr; ++i) {
            const int id = rem[i];
            if (id < 0 || id >= rec->id_count)
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: id %d outside [0, %d)", id, rec->id_count);
            rem[i] = rec->slot_of[id];
            if (rem[i] < 0 || rem[i] >= n || rec->slot_id[rem[i]] != id)
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: id %d is not in the map", id);
        }
        // inserted ids: in range, not in the map, distinct (marked -2 in slot_of while checked, then restored)
        int32_t *sof = rec->slot_of;
        int bad = -1, j = 0;
        for (; j < m; ++j) {
            const int id = edit->insert_ids[j];
            if (id < 0 || id >= rec->id_count || sof[id] != -1) {
                bad = id;
                break;
            }
            sof[id] = -2;
        }
        for (int k = 0; k < j; ++k) sof[edit->insert_ids[k]] = -1;
        if (bad != -1 || j < m)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: inserted id %d out of range, in the map or listed twice",
                        bad);
    }
    // removed slots: range and duplicates through a bitmap over [0, n), which
    // also yields the holes below n1 in ascending order without a sort
    std::vector<uint64_t> &mk = ctx->edit_marks;
    if (mk.size() < (size_t)(n + 63) / 64) mk.resize((size_t)(n + 63) / 64, 0);
    auto unmark = [&](int upto) {
        for (int i = 0; i < upto; ++i) mk[rem[i] >> 6] &= ~(1ull << (rem[i] & 63));
    };
    for (int i = 0; i < nr; ++i) {
        const int r = rem[i];
        if (r < 0 || r >= n) {
            unmark(i);
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: index %d outside [0, %d)", r, n);
        }
        const uint64_t bit = 1ull << (r & 63);
        if (mk[r >> 6] & bit) {
            unmark(i);
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: index %d listed twice", r);
        }
        mk[r >> 6] |= bit;
    }
    const int n1 = n - nr;
    if ((int64_t)n1 + m > capacity) {
        unmark(nr);
        return fail(ctx, FT_ERR_CAPACITY, "map update: %d points exceed the capacity %d", n1 + m, capacity);
    }
    // (hole, source) pairs: removed slots below n1 and surviving points from n1 up, both ascending
    std::vector<int32_t> holes;
    holes.reserve(nr);
    for (int w = 0; w < (n1 + 63) / 64; ++w) {
        uint64_t bits = mk[w];
        if (w == n1 / 64) bits &= (n1 % 64) ? ((1ull << (n1 % 64)) - 1) : 0ull;
        while (bits) {
            holes.push_back(w * 64 + __builtin_ctzll(bits));
            bits &= bits - 1;
        }
    }
    const int n_holes = (int)holes.size();
    pe.pairs.resize(2 * (size_t)n_holes);
    int src = n1;
    for (int h = 0; h < n_holes; ++h) {
        while (mk[src >> 6] & (1ull << (src & 63))) ++src;
        pe.pairs[2 * h] = holes[h];
        pe.pairs[2 * h + 1] = src++;
    }
    unmark(nr);
    if (rec) {   // the moved points' record entries must be consistent before anything is enqueued
        for (int h = 0; h < n_holes; ++h) {
            const int id = rec->slot_id[pe.pairs[2 * h + 1]];
            if (id < 0 || id >= rec->id_count || rec->slot_of[id] != pe.pairs[2 * h + 1])
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update: id record inconsistent at slot %d",
                            pe.pairs[2 * h + 1]);
        }
    }
    pe.n1 = n1;
    pe.m = m;
    pe.n_holes = n_holes;
    return FT_OK;
}

// The id record follows an enqueued edit (removed ids leave, moved ids take
// their holes, inserted ids follow n1).
void commit_record(const ft_map_edit *edit, const PreparedEdit &pe)
{
    ft_map_ids *rec = edit->ids;
    if (!rec) return;
    int32_t *sid = rec->slot_id, *sof = rec->slot_of;
    for (int32_t r : pe.rem) sof[sid[r]] = -1;
    for (int h = 0; h < pe.n_holes; ++h) {
        const int id = sid[pe.pairs[2 * h + 1]];
        sid[pe.pairs[2 * h]] = id;
        sof[id] = pe.pairs[2 * h];
    }
    for (int j = 0; j < pe.m; ++j) {
        sid[pe.n1 + j] = edit->insert_ids[j];
        sof[edit->insert_ids[j]] = pe.n1 + j;
    }
}

// A chunk of `need` bytes of the pinned edit ring (and of its device mirror
// at the same offset): completed chunks are reclaimed first; a chunk the new
// one would overlap (or the oldest, when every event is in use) is waited for.
ft_status take_edit_chunk(ft_context *ctx, size_t need, size_t *off_out)
{
    auto &live = ctx->edit_live;
    auto pop_front = [&](bool wait) -> hipError_t {
        hipError_t e = wait ? hipEventSynchronize(live.front().ev) : hipSuccess;
        ctx->edit_free_ev.push_back(live.front().ev);
        live.pop_front();
        return e;
    };
    while (!live.empty() && hipEventQuery(live.front().ev) == hipSuccess) (void)pop_front(false);
    size_t off = ctx->edit_head + need <= ctx->edit_ring_bytes ? ctx->edit_head : 0;
    auto overlaps = [&]() {
        for (const auto &c : live)
            if (off < c.off + c.bytes && c.off < off + need) return true;
        return false;
    };
    while (!live.empty() && (overlaps() || ctx->edit_free_ev.empty())) HIP_TRY(ctx, pop_front(true));
    ctx->edit_head = off + need;
    *off_out = off;
    return FT_OK;
}

ft_status finish_edit_chunk(ft_context *ctx, size_t off, size_t need, hipStream_t s)
{
    hipEvent_t ev = ctx->edit_free_ev.back();
    HIP_TRY(ctx, hipEventRecord(ev, s));
    ctx->edit_free_ev.pop_back();
    ctx->edit_live.push_back({off, need, ev});
    return FT_OK;
}

}  // namespace

ft_status ft_map_update(ft_context *ctx, void *stream, ft_map_points *map, int32_t capacity,
                        const ft_map_edit *edit)
{
    ft_status st = enter(ctx);
    if (st) return st;
    PreparedEdit pe;
    if ((st = prepare_edit(ctx, map, capacity, edit, pe))) return st;
    const size_t need = align_up(sizeof(int32_t) * 2 * (size_t)std::max(pe.n_holes, 1), 256);
    size_t off = 0;
    if ((st = take_edit_chunk(ctx, need, &off))) return st;
    int32_t *pairs = reinterpret_cast<int32_t *>(ctx->edit_ring + off);
    if (pe.n_holes) memcpy(pairs, pe.pairs.data(), sizeof(int32_t) * pe.pairs.size());
    hipStream_t s = (hipStream_t)stream;
    MapEditArgs a{};
    a.pos = const_cast<float *>(map->pos);
    a.normal = const_cast<float *>(map->normal);
    a.dmin = const_cast<float *>(map->dmin);
    a.dmax = const_cast<float *>(map->dmax);
    a.desc = const_cast<uint8_t *>(map->desc);
    a.pairs = pairs;                  // pinned staging, read by the move kernel over the bus
    a.n_pairs = pe.n_holes;
    a.ipos = edit->insert.pos;
    a.inormal = edit->insert.normal;
    a.idmin = edit->insert.dmin;
    a.idmax = edit->insert.dmax;
    a.idesc = edit->insert.desc;
    a.n1 = pe.n1;
    a.n_insert = pe.m;
    HIP_TRY(ctx, launch_map_edit(a, s));
    if ((st = finish_edit_chunk(ctx, off, need, s))) return st;
    commit_record(edit, pe);
    map->n = pe.n1 + pe.m;
    return FT_OK;
}

ft_status ft_map_update_many(ft_context *ctx, void *stream, int32_t n, ft_map_points *const *maps,
                             const int32_t *capacities, const ft_map_edit *edits)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (n < 0 || (n > 0 && (!maps || !capacities || !edits)))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update many: %d edits, null list", n);
    if (n > kMaxManyEdits)
        return fail(ctx, FT_ERR_CAPACITY, "map update many: %d edits exceed %d", n, kMaxManyEdits);
    std::vector<PreparedEdit> pe(n);
    int64_t moves = 0, apps = 0;
    for (int i = 0; i < n; ++i) {
        if ((st = prepare_edit(ctx, maps[i], capacities[i], &edits[i], pe[i]))) return st;
        for (int k = 0; k < i; ++k) {
            if (maps[k]->pos == maps[i]->pos)
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update many: edits %d and %d name one map", k, i);
            if (edits[i].ids && edits[k].ids &&
                (edits[k].ids == edits[i].ids || edits[k].ids->slot_of == edits[i].ids->slot_of))
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "map update many: edits %d and %d share an id record", k, i);
        }
        moves += pe[i].n_holes;
        apps += pe[i].m;
    }
    if (n == 0) return FT_OK;
    // one chunk: the edits' descriptors, moves (edit, hole, source), appends (edit, j)
    const size_t d_bytes = align_up(sizeof(MapEditDesc) * (size_t)n, 256);
    const size_t m_bytes = align_up(sizeof(int32_t) * 3 * (size_t)std::max<int64_t>(moves, 1), 256);
    const size_t a_bytes = align_up(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(apps, 1), 256);
    const size_t need = d_bytes + m_bytes + a_bytes;
    if (need > ctx->edit_ring_bytes / 2)
        return fail(ctx, FT_ERR_CAPACITY, "map update many: %lld moves and %lld inserts exceed the staging",
                    (long long)moves, (long long)apps);
    size_t off = 0;
    if ((st = take_edit_chunk(ctx, need, &off))) return st;
    char *h = ctx->edit_ring + off;
    MapEditDesc *desc = reinterpret_cast<MapEditDesc *>(h);
    int32_t *mv = reinterpret_cast<int32_t *>(h + d_bytes);
    int32_t *ap = reinterpret_cast<int32_t *>(h + d_bytes + m_bytes);
    int64_t mk = 0, ak = 0;
    for (int i = 0; i < n; ++i) {
        const ft_map_points &mp = *maps[i];
        const ft_map_points &ins = edits[i].insert;
        MapEditDesc &d = desc[i];
        d.pos = const_cast<float *>(mp.pos);
        d.normal = const_cast<float *>(mp.normal);
        d.dmin = const_cast<float *>(mp.dmin);
        d.dmax = const_cast<float *>(mp.dmax);
        d.desc = const_cast<uint8_t *>(mp.desc);
        d.ipos = ins.pos;
        d.inormal = ins.normal;
        d.idmin = ins.dmin;
        d.idmax = ins.dmax;
        d.idesc = ins.desc;
        d.n1 = pe[i].n1;
        d.pad = 0;
        for (int k = 0; k < pe[i].n_holes; ++k, ++mk) {
            mv[3 * mk] = i;
            mv[3 * mk + 1] = pe[i].pairs[2 * k];
            mv[3 * mk + 2] = pe[i].pairs[2 * k + 1];
        }
        for (int j = 0; j < pe[i].m; ++j, ++ak) {
            ap[2 * ak] = i;
            ap[2 * ak + 1] = j;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    char *d = ctx->d_edit_ring + off;
    HIP_TRY(ctx, hipMemcpyAsync(d, h, need, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_map_edit_many(reinterpret_cast<const MapEditDesc *>(d),
                                      reinterpret_cast<const int32_t *>(d + d_bytes), (int)moves,
                                      reinterpret_cast<const int32_t *>(d + d_bytes + m_bytes), (int)apps, s));
    if ((st = finish_edit_chunk(ctx, off, need, s))) return st;
    for (int i = 0; i < n; ++i) {
        commit_record(&edits[i], pe[i]);
        maps[i]->n = pe[i].n1 + pe[i].m;
    }
    return FT_OK;
}

// ------------------------------------------------------------ ORB extraction
namespace {

ft_status check_orb_pyramid(ft_context *ctx, const ft_pyramid *pyr, const char *what)
{
    if (!pyr || !pyr->data) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: null pyramid", what);
    for (int l = 0; l < kLevels; ++l) {
        if (pyr->width[l] < 1 || pyr->height[l] < 1 || pyr->offset[l] < 0)
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "%s: level %d is %dx%d at offset %lld", what, l, pyr->width[l],
                        pyr->height[l], (long long)pyr->offset[l]);
        if (pyr->width[l] > kMaxPyrW || pyr->height[l] > kMaxRows)
            return fail(ctx, FT_ERR_CAPACITY, "%s: level %d is %dx%d, above %dx%d", what, l, pyr->width[l],
                        pyr->height[l], kMaxPyrW, kMaxRows);
    }
    return FT_OK;
}

}  // namespace

ft_status ft_orb_detect(ft_context *ctx, void *stream, const ft_pyramid *pyr, const ft_scales *scales,
                        const ft_orb_params *params, uint8_t *blurred, const ft_orb_corners *out)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if ((st = check_scales(ctx, scales)) || (st = check_orb_pyramid(ctx, pyr, "orb detect"))) return st;
    if (!params || !out) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb detect: null argument");
    if (params->threshold < 1 || params->threshold > 254 || params->edge < 19 || params->edge > kMaxRows)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb detect: threshold %d (1..254), edge %d (>= 19)",
                    params->threshold, params->edge);
    if (out->capacity < 0 || !out->count || !aligned(out->count, 4))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb detect: capacity %d, count %p", out->capacity,
                    (const void *)out->count);
    if (out->capacity > 0 && (!out->lx || !out->ly || !out->octave || !out->score || !out->x || !out->y ||
                              !aligned(out->lx, 2) || !aligned(out->ly, 2) || !aligned(out->x, 4) ||
                              !aligned(out->y, 4)))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb detect: null or misaligned output array");
    OrbDetectArgs a{};
    a.pyr = pyr->data;
    a.blurred = blurred;
    int tiles = 0, wmax = 0;
    for (int l = 0; l < kLevels; ++l) {
        a.off[l] = pyr->offset[l];
        a.w[l] = pyr->width[l];
        a.h[l] = pyr->height[l];
        a.sf[l] = scales->sf[l];
        a.tile0[l] = tiles;
        tiles += (pyr->height[l] + kOrbRows - 1) / kOrbRows;
        wmax = std::max(wmax, (int)pyr->width[l]);
    }
    a.tile0[kLevels] = tiles;
    a.t = params->threshold;
    a.edge = params->edge;
    a.capacity = out->capacity;
    a.lds_w = (wmax + 3) & ~3;
    a.lx = out->lx;
    a.ly = out->ly;
    a.oct = out->octave;
    a.score = out->score;
    a.x = out->x;
    a.y = out->y;
    a.count = out->count;
    const int slot = ctx->orb_next;
    ctx->orb_next = (slot + 1) % ft_context::kOrbSlots;
    if (ctx->orb_used[slot]) HIP_TRY(ctx, hipEventSynchronize(ctx->orb_ev[slot]));
    a.tile_state = ctx->orb_state[slot];
    a.ticket = ctx->orb_ticket[slot];
    a.ticket_base = ctx->orb_base[slot];
    a.epoch = ++ctx->orb_epoch[slot];
    if (a.epoch == 0) a.epoch = ++ctx->orb_epoch[slot];   // 0 marks never-written state
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, launch_orb_detect(a, s));
    ctx->orb_base[slot] += (uint32_t)tiles;   // the kernel takes exactly `tiles` tickets
    HIP_TRY(ctx, hipEventRecord(ctx->orb_ev[slot], s));
    ctx->orb_used[slot] = true;
    return FT_OK;
}

ft_status ft_orb_describe(ft_context *ctx, void *stream, const ft_pyramid *pyr, const uint8_t *blurred,
                          int32_t n_max, const int32_t *count, const int16_t *lx, const int16_t *ly,
                          const uint8_t *octave, const int8_t *pattern, float *angle, uint8_t *desc)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if ((st = check_orb_pyramid(ctx, pyr, "orb describe"))) return st;
    if (!blurred || !pattern || n_max < 0)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb describe: null smoothed pyramid or pattern, or n %d", n_max);
    if (n_max > 0 && (!lx || !ly || !octave || !angle || !desc || !aligned(lx, 2) || !aligned(ly, 2) ||
                      !aligned(angle, 4) || !aligned(desc, 8) || (count && !aligned(count, 4))))
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb describe: null or misaligned array");
    OrbDescribeArgs a{};
    for (int t = 0; t < kOrbTests; ++t)
        for (int c = 0; c < 2; ++c) {
            const int px = pattern[4 * t + 2 * c], py = pattern[4 * t + 2 * c + 1];
            if (px * px + py * py > 169)
                return fail(ctx, FT_ERR_INVALID_ARGUMENT, "orb describe: pattern point %d of test %d lies beyond radius 13",
                            c, t);
            a.pattern[t][2 * c] = (int8_t)px;
            a.pattern[t][2 * c + 1] = (int8_t)py;
        }
    a.pyr = pyr->data;
    a.blurred = blurred;
    for (int l = 0; l < kLevels; ++l) {
        a.off[l] = pyr->offset[l];
        a.w[l] = pyr->width[l];
        a.h[l] = pyr->height[l];
    }
    a.n_max = n_max;
    a.count = count;
    a.lx = lx;
    a.ly = ly;
    a.oct = octave;
    a.angle = angle;
    a.desc = desc;
    HIP_TRY(ctx, launch_orb_describe(a, (hipStream_t)stream));
    return FT_OK;
}

ft_status ft_batch_submit(ft_context *ctx, void *stream, const ft_frame_job *jobs, int32_t n,
                          uint64_t *ticket)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!jobs || !ticket || n <= 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "batch: bad arguments");
    if (n > ctx->lim.max_batch_frames)
        return fail(ctx, FT_ERR_CAPACITY, "batch: %d frames exceed max_batch_frames %d", n,
                    ctx->lim.max_batch_frames);
    int lane_id = -1;
    Lane *lane = free_lane(ctx, &lane_id, &st);
    if (!lane) return st;
    if ((st = build_batch(ctx, *lane, jobs, n))) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t totals[PH_COUNT];
    plan_batch(ctx, *lane, n, ctx->shapes, totals);
    if (ctx->exec_mode == FT_EXEC_EAGER || ctx->timing)
        st = launch_batch(ctx, *lane, n, ctx->shapes, s, totals, next_events(ctx, totals));
    else
        st = launch_batch_graph(ctx, *lane, n, s, totals);
    if (st) return st;
    HIP_TRY(ctx, hipEventRecord(lane->done, s));
    lane->used = true;
    lane->ticket = (ctx->next_ticket++ << 8) | (uint64_t)lane_id;
    *ticket = lane->ticket;
    return FT_OK;
}

ft_status ft_batch_poll(ft_context *ctx, uint64_t ticket, int32_t *done)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!done) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "poll: null done");
    const size_t lane_id = ticket & 0xFF;
    if (lane_id >= ctx->lanes.size() || ticket == 0 || (ticket >> 8) >= ctx->next_ticket)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "poll: unknown ticket");
    Lane &ln = ctx->lanes[lane_id];
    if (ln.ticket != ticket) {  // the lane was reused, so this ticket completed earlier
        *done = 1;
        return FT_OK;
    }
    const hipError_t q = hipEventQuery(ln.done);
    if (q == hipSuccess) {
        *done = 1;
        return FT_OK;
    }
    if (q == hipErrorNotReady) *done = 0;
    else return fail(ctx, FT_ERR_DEVICE, "poll: %s", hipGetErrorString(q));
    return FT_OK;
}

ft_status ft_batch_wait(ft_context *ctx, uint64_t ticket)
{
    ft_status st = enter(ctx);
    if (st) return st;
    const size_t lane_id = ticket & 0xFF;
    if (lane_id >= ctx->lanes.size() || ticket == 0 || (ticket >> 8) >= ctx->next_ticket)
        return fail(ctx, FT_ERR_INVALID_ARGUMENT, "wait: unknown ticket");
    Lane &ln = ctx->lanes[lane_id];
    if (ln.ticket != ticket) return FT_OK;
    HIP_TRY(ctx, hipEventSynchronize(ln.done));
    return FT_OK;
}

ft_status ft_autotune(ft_context *ctx, void *stream, const ft_frame_job *jobs, int32_t n,
                      const char *cache_path, ft_shapes *chosen)
{
    ft_status st = enter(ctx);
    if (st) return st;
    if (!jobs || n <= 0) return fail(ctx, FT_ERR_INVALID_ARGUMENT, "autotune: bad arguments");
    if (n > ctx->lim.max_batch_frames)
        return fail(ctx, FT_ERR_CAPACITY, "autotune: %d frames exceed max_batch_frames %d", n,
                    ctx->lim.max_batch_frames);
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
    const std::string key = workload_key(jobs, n, prop.gcnArchName);
    Shapes best = ctx->shapes;
    if (!(cache_path && cache_lookup(cache_path, key, best))) {
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(ctx, hipStreamSynchronize(s));
        int lane_id = -1;
        Lane *lane = free_lane(ctx, &lane_id, &st);
        if (!lane) return st;
        if ((st = build_batch(ctx, *lane, jobs, n))) return st;
        const bool was_timing = ctx->timing;
        if ((st = set_timing(ctx, true))) return st;
        double ms[kPhases];
        int64_t cnt[kPhases];
        read_timing(ctx, ms, cnt);   // start from zero
        // one phase for one candidate: 1 warm-up + 3 timed runs, median
        auto time_phase = [&](const Shapes &sh, int phase, double *us) -> ft_status {
            std::vector<double> v;
            for (int r = 0; r < 4; ++r) {
                int32_t totals[PH_COUNT];
                plan_batch(ctx, *lane, n, sh, totals);
                ft_status e = launch_batch(ctx, *lane, n, sh, s, totals, next_events(ctx, totals));
                if (e) return e;
                HIP_TRY(ctx, hipStreamSynchronize(s));
                read_timing(ctx, ms, cnt);
                if (r > 0) v.push_back(ms[phase] * 1e3);
            }
            std::sort(v.begin(), v.end());
            *us = v[v.size() / 2];
            return FT_OK;
        };
        const int cands[] = {1, 2, 4, 8, 16};
        double best_a = 1e30, best_s = 1e30;
        for (int g : cands) {
            Shapes sh = best;
            sh.best_lanes = g;
            double us;
            if ((st = time_phase(sh, PH_STEREO_A, &us))) return st;
            if (us < best_a) {
                best_a = us;
                best.best_lanes = g;
            }
        }
        {   // setup sorts + stereo resolve: 256 or 1024 threads
            double t[2][2];
            const int blocks[2] = {kWG, kAuxWG};
            for (int w = 0; w < 2; ++w) {
                Shapes sh = best;
                sh.aux_block = blocks[w];
                if ((st = time_phase(sh, PH_SETUP, &t[w][0]))) return st;
                if ((st = time_phase(sh, PH_STEREO_C, &t[w][1]))) return st;
            }
            best.aux_block = t[1][0] + t[1][1] < t[0][0] + t[0][1] ? kAuxWG : kWG;
        }
        for (int g : cands) {
            Shapes sh = best;
            sh.search_lanes = g;
            double us;
            if ((st = time_phase(sh, PH_SEARCH, &us))) return st;
            if (us < best_s) {
                best_s = us;
                best.search_lanes = g;
            }
        }
        set_timing(ctx, was_timing);
        if (cache_path && !cache_append(cache_path, key, best, best_a + best_s))
            return fail(ctx, FT_ERR_INVALID_ARGUMENT, "autotune: cannot write %s", cache_path);
    }
    if (!(best == ctx->shapes)) {
        ctx->shapes = best;
        if ((st = rebuild_graphs(ctx))) return st;
    }
    if (chosen) to_public(ctx->shapes, chosen);
    return FT_OK;
}

}  // extern "C"
