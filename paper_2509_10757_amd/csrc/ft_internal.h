// Internal device-side job description shared by the host API and the kernels.
// A DevJob is a plain struct: passed by value as a kernel argument for the
// single-frame calls, or stored in a device job table for batches.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "ft.h"

namespace ft {

constexpr int kLevels = FT_LEVELS;
constexpr int kWG = 256;              // every kernel runs 256-thread workgroups (4 wave64s)
constexpr int kMaxRows = 4096;
constexpr int kMaxCells = 8192;
constexpr int kMaxKp = 65535;
constexpr int kMaxCellRep = 3;       // copies of a keypoint in a level-binned cell index (level window <= 3 octaves)
constexpr int kMaxMap = (1 << 23) - 1;
constexpr int kKnnQueriesPerWG = 32;  // fisheye all-pairs: queries per 256-thread subgroup (16-row MFMA blocks)
constexpr int kKnnTilesInFlight = 8;  // fisheye all-pairs: target tiles whose descriptor loads a wave keeps in flight
constexpr int kRefinePerWG = 4;       // pinhole refinement: one wave per match
constexpr int kRefineLds = 1024;      // bytes of LDS per refining wave (patch + strip)
constexpr int kRefineQPerWG = 16;     // ... 11x11 window, +-5 shifts: four matches per wave
constexpr int kRefineQLds = 800;      // bytes of LDS per match (11 x 12 + 11 x 24 16-bit values)
constexpr int kPyrRows = 16;          // image pyramid: level-0 rows per workgroup
constexpr int kMaxPyrW = 1536;        // widest level-0 image the pyramid build stages in LDS
constexpr int kRotBinsMax = 64;       // rotation histogram bins of the last-frame search

enum Phase : int {
    PH_PYRAMID = 0,  // image pyramids of the stereo images (when the job builds them)
    PH_SETUP,        // row sort / overlap lists / cell sort
    PH_STEREO_A,     // pinhole best match | fisheye all-pairs top-2
    PH_REFINE,       // pinhole SAD refinement
    PH_TRI,          // fisheye ratio + triangulation check
    PH_STEREO_C,     // stereo resolve + outputs
    PH_SEARCH,       // search by projection
    PH_SEARCH_FIN,   // search resolve + outputs
    PH_COUNT
};

enum JobFlags : int32_t {
    JOB_STEREO_PINHOLE = 1,
    JOB_STEREO_FISHEYE = 2,
    JOB_SEARCH0 = 4,
    JOB_SEARCH1 = 8,
};

// Right keypoint sorted by integer row (pinhole row index): 16 bytes.
struct RowRec {
    float x;
    uint32_t band;   // rows lo | hi << 16 covered by the keypoint's band (empty: lo > hi)
    uint32_t meta;   // octave | index << 16
    uint32_t pad;
};

// An accepted pinhole best match, appended by the best-match phase so that the
// refinement runs over matches only and reads everything it needs at once.
struct MatchRec {
    int32_t i, j, h;   // left keypoint, right keypoint, Hamming distance
    float bx;          // x of the right keypoint
    float x, y;        // left keypoint
    int32_t oct, pad;  // left keypoint octave
};

// Keypoint sorted by grid cell (search by projection): 16 bytes + descriptor.
// Pointers the kernels dereference are global-memory pointers in the kernels'
// device code (FT_KERNELS is defined by the kernel sources), so loads and
// stores through them are global, not flat, instructions; host code sees
// plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__) && defined(FT_KERNELS)
#define FT_G __attribute__((address_space(1)))
#else
#define FT_G
#endif

struct CellRec {
    float x, y;
    uint32_t meta;   // octave | preassigned << 8 | index << 16
    uint32_t pad;
};

struct DevKps {
    int32_t n;
    const FT_G float *x, *y;
    const FT_G uint8_t *oct;
    const FT_G uint8_t *desc;
};

struct DevView {
    int32_t model;
    int32_t cols, rows;              // cells of the keypoint index (the caller's grid, coarser when binned)
    float fx, fy, cx, cy, bf;
    float k[4];
    float R[9], t[3], O[3];
    float min_x, max_x, min_y, max_y;
    float inv_cw, inv_ch;            // cols/(max_x-min_x), rows/(max_y-min_y)
    int32_t n_pb;                    // level bins of the cell index: kLevels (bin p holds the
                                     // octaves a map point predicted at level p may match) or 1
    int32_t side;                    // keypoints of the left (0) or right (1) image
    const FT_G uint8_t *preassigned;      // nullable
    const FT_G float *u_right;            // nullable
    const FT_G uint8_t *kdesc;            // descriptors of the view's keypoints
    FT_G int32_t *mp_match, *mp_dist, *kp_match, *n_matches;
    // workspace
    FT_G int32_t *cell_off;          // [n_pb][rows][cols] + 1 record offsets
    FT_G CellRec *crec;              // records sorted by (level bin, cell)
    FT_G int32_t *mp_k, *mp_h;
    FT_G uint32_t *claim;
    FT_G int32_t *hist;              // rotation histogram of the last-frame search [kRotBinsMax]
};

struct DevJob {
    int32_t flags;
    int32_t nM;
    int32_t n_views;
    DevKps L, R;
    float sf[kLevels], inv_sf[kLevels], sigma2[kLevels];
    // pinhole stereo
    const FT_G uint8_t *pyrL, *pyrR;
    int64_t lv_off[kLevels];
    int32_t lv_w[kLevels], lv_h[kLevels];
    float bf, maxD, band;
    int32_t rows, row_reach;          // bins scanned on each side of a query row (one level bin)
    int32_t n_lb;                     // level bins of the row index: kLevels (rows binned per
                                      // pyramid level) or 1 (one bin for every level)
    int32_t lv_reach[kLevels];        // per level bin: rows scanned on each side of a query row
    int32_t th_orb, half_win, half_range, level_window, med_num, med_den;
    // fisheye stereo
    float kbL[8], kbR[8], R_lr[9], t_lr[3], ovl[2], ovr[2];
    int32_t ratio_num, ratio_den, newton_iters;
    double cos_max, chi2, max_theta, newton_tol;
    // stereo outputs (caller memory)
    FT_G int32_t *o_right_idx, *o_dist, *o_sad, *o_nmatch;
    FT_G float *o_uR, *o_depth, *o_xyz;
    // stereo workspace
    FT_G int32_t *row_start;               // [n_lb][rows + 1] record offsets of (level bin, row)
    FT_G RowRec *rrec;                     // right keypoints sorted by row
    FT_G uint8_t *tdesc;                   // right descriptors in overlap order (fisheye)
    FT_G int32_t *best_j, *best_h, *h2, *sad, *flag, *qlist, *tlist, *counts;
    FT_G MatchRec *mrec;                   // pinhole: accepted best matches, counts[2] of them
    FT_G float *uR, *depth, *xyz;
    FT_G uint32_t *claimR;
    // search by projection
    const FT_G float *pos, *normal, *dmin, *dmax;
    const FT_G uint8_t *mdesc;
    float th, cos_lim, cos_narrow, r_narrow, r_wide, dist_lo, dist_hi;
    int32_t lv_lo, lv_hi, th_high, s_ratio_num, s_ratio_den, same_level_only;
    DevView view[2];
    // image pyramids built on the device (pinhole stereo images)
    const FT_G uint8_t *imgL, *imgR;  // level-0 images, row pitch img_pitch (null: no build)
    FT_G uint8_t *pyr_outL, *pyr_outR;
    int32_t img_w, img_h, img_pitch;
    // last-frame search by projection (view 0; pos / mdesc / nM hold the points)
    const FT_G uint8_t *l_oct;        // octave of the last-frame keypoint of each point
    const FT_G float *l_ang, *k_ang;  // orientations (degrees): last-frame keypoints, current keypoints
    int32_t direction, check_rot, rot_bins;
};

// Launch shapes of one submission (the autotuner chooses them).  Defaults:
// the shapes the autotuner picks for mixed pinhole/fisheye batches.
constexpr int kAuxWG = 1024;          // the wide option for the setup sorts and the stereo resolve
struct Shapes {
    int best_lanes = 8;        // lanes cooperating on one pinhole left keypoint
    int search_lanes = 1;      // lanes cooperating on one map point (1 = record-dealt search)
    int aux_block = kAuxWG;    // threads per workgroup of the setup sorts and the stereo resolve
    bool operator==(const Shapes &o) const
    {
        return best_lanes == o.best_lanes && search_lanes == o.search_lanes && aux_block == o.aux_block;
    }
};

// Tiles of each phase for each job, as prefix sums: batch launches map a flat
// block index to (job, tile) with a binary search over them.
struct TileMap {
    int32_t n_jobs;
    const FT_G int32_t *prefix;  // device [PH_COUNT][n_jobs + 1]
};

// Argument of every batch kernel: the device job table and its tile prefixes.
struct BatchArgs {
    const DevJob *p;
    TileMap map;
};

// Per-job tile counts of each phase for the given shapes.
void job_tiles(const DevJob &J, const Shapes &s, bool do_stereo, bool do_search,
               int32_t out[PH_COUNT]);

// Optional per-phase event timing: when `ev` is non-null, ev[p] and ev[p+1]
// bracket phase p on the launch stream (ev has kPhases + 1 events).
constexpr int kPhases = FT_PHASES;
static_assert(kPhases == PH_COUNT, "one timing slot per phase");

// Launchers (ft_kernels.hip).  `table` == nullptr: one job passed by value;
// otherwise a device job table whose flat tiles are described by `map`.
// `totals` holds the number of workgroups of each phase.
hipError_t launch_pipeline(const DevJob *table, const TileMap &map, const int32_t totals[PH_COUNT],
                           const DevJob &one, const Shapes &shapes, hipStream_t stream, hipEvent_t *ev);
// Last-frame search of one job's view 0: setup, search (`lanes` per point),
// claim resolution with the rotation histogram, rotation check and outputs.
hipError_t launch_last_frame(const DevJob &J, int lanes, hipStream_t stream);
// Batch kernel of every phase for these shapes (JobTable argument), and its
// workgroup size: the nodes of a lane's batch graph.
void batch_kernels(const Shapes &shapes, void *fn[PH_COUNT], int block[PH_COUNT]);

// Allocation-free search (ft_noalloc.hip): the workspace of one view in a
// fixed device array of every GPU, kNoallocScratchBytes long, sized for
// FT_NOALLOC_MAX_KP keypoints, FT_NOALLOC_MAX_MAP map points and kMaxCells
// grid cells.  noalloc_scratch returns the current device's address of it
// and whether the device is a gfx950 (both looked up once per device).
constexpr size_t kNoallocScratchBytes = FT_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch(int device, char **out, bool *gfx950);

// Local-map edit (ft_kernels.hip): the (hole, source) pairs move first, then
// the inserted points are appended at n1 (two launches: an append may land on
// a source slot).
struct MapEditArgs {
    FT_G float *pos, *normal, *dmin, *dmax;
    FT_G uint8_t *desc;
    const FT_G int32_t *pairs;   // [n_pairs][2]: hole, source
    int32_t n_pairs;
    const FT_G float *ipos, *inormal, *idmin, *idmax;
    const FT_G uint8_t *idesc;
    int32_t n1, n_insert;
};
hipError_t launch_map_edit(const MapEditArgs &a, hipStream_t stream);
// Several maps' edits in two launches (ft_map.hip): descriptors, moves (edit,
// hole, source) and appends (edit, j), all in device memory.
constexpr int kMaxManyEdits = 4096;
struct MapEditDesc {
    FT_G float *pos, *normal, *dmin, *dmax;
    FT_G uint8_t *desc;
    const FT_G float *ipos, *inormal, *idmin, *idmax;
    const FT_G uint8_t *idesc;
    int32_t n1, pad;
};
hipError_t launch_map_edit_many(const MapEditDesc *descs, const int32_t *moves, int n_moves, const int32_t *apps,
                                int n_apps, hipStream_t stream);

// ORB extraction (ft_orb.hip).  Detection runs over row tiles of every level
// of one pyramid: kOrbRows output rows per workgroup, the level rows they need
// staged in LDS (kOrbHalo above and below: the FAST ring and the
// suppression), so a pyramid has at most kOrbMaxTiles tiles.
constexpr int kOrbRows = 8;
constexpr int kOrbHalo = 4;
constexpr int kOrbMaxTiles = kLevels * (kMaxRows / kOrbRows);
constexpr int kOrbTests = 256;
struct OrbDetectArgs {
    const FT_G uint8_t *pyr;
    FT_G uint8_t *blurred;            // null: no smoothing
    int64_t off[kLevels];
    int32_t w[kLevels], h[kLevels];
    float sf[kLevels];
    int32_t tile0[kLevels + 1];       // first tile of each level; tile0[kLevels] = tiles
    int32_t t, edge, capacity, lds_w; // lds_w: LDS row stride (the widest level, rounded up to 4)
    // single-pass emission: tiles are taken by ticket (ticket counter - ticket_base), and each
    // publishes its count and then its inclusive prefix in tile_state, tagged with this call's epoch
    FT_G unsigned long long *tile_state;  // [kOrbMaxTiles]
    FT_G uint32_t *ticket;
    uint32_t ticket_base, epoch;
    FT_G int16_t *lx, *ly;
    FT_G uint8_t *oct, *score;
    FT_G float *x, *y;
    FT_G int32_t *count;
};
struct OrbDescribeArgs {
    const FT_G uint8_t *pyr, *blurred;
    int64_t off[kLevels];
    int32_t w[kLevels], h[kLevels];
    int32_t n_max;
    const FT_G int32_t *count;        // nullable: n = min(n_max, *count)
    const FT_G int16_t *lx, *ly;
    const FT_G uint8_t *oct;
    FT_G float *angle;
    FT_G uint8_t *desc;
    int8_t pattern[kOrbTests][4];     // x1, y1, x2, y2 of each test
};
size_t orb_detect_lds(int lds_w);
hipError_t launch_orb_detect(const OrbDetectArgs &a, hipStream_t stream);
hipError_t launch_orb_describe(const OrbDescribeArgs &a, hipStream_t stream);

// Gather-list copy (ft_upload.hip): up to kUploadSegs segments per launch,
// passed by value; each workgroup copies one kUploadChunk-byte chunk of one
// segment.  `first[s]` is the first workgroup of segment s, first[n] the grid.
constexpr int kUploadSegs = 64;
constexpr int kUploadChunk = 32768;
struct UploadArgs {
    int32_t n;
    int32_t first[kUploadSegs + 1];
    const char *src[kUploadSegs];
    char *dst[kUploadSegs];
    int64_t bytes[kUploadSegs];
};
hipError_t launch_upload(const UploadArgs &a, hipStream_t stream);

}  // namespace ft
