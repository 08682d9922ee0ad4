/* ft.h -- C ABI of the MI355X tracking correspondence search.
 *
 * The library implements the two GPU-resident steps of visual tracking that
 * FastTrack (arXiv 2509.10757) moves off the CPU:
 *   - stereo matching: each left keypoint gets its most similar right keypoint
 *     (Section II-B; Section IV-C "Stereo Matching"), rectified pinhole pairs by
 *     an epipolar row-band search refined among nearby pixels, fisheye pairs by
 *     a brute-force search of the overlap region;
 *   - search by projection: each local map point gets its correspondence among
 *     the current frame's keypoints, each map point independently of the others
 *     (Section II-D "Track Local Map"; Section IV-E "Search Local Points").
 * Memory is allocated once when a context is created and reused for every
 * frame (Section IV-A: allocate at start, release at shutdown), so no call
 * after ft_context_create allocates device memory (ft_host_alloc, which
 * allocates pinned host memory, is the one set-up call besides it).
 *
 * Conventions for every entry point:
 *   - Pointers inside ft_keypoints, ft_pyramid, ft_map_points and the *_out
 *     structs are DEVICE pointers; the structs themselves, the scale tables,
 *     cameras, grids and parameters are HOST values copied during the call.
 *   - Descriptors are 256-bit ORB descriptors stored as uint8_t[n][32],
 *     16-byte aligned; bit t of byte q is descriptor bit 8q+t.
 *   - Coordinates are level-0 pixels; `octave` is the pyramid level (0..7).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is only
 *     enqueued: outputs are valid once the stream (or the batch ticket) has
 *     completed.  The single-frame calls of one context share one workspace,
 *     so they must be ordered on one stream (or by the caller).  Each batch in
 *     flight owns a workspace lane of its own, so batches may run on
 *     different streams at the same time.
 *   - The caller owns every buffer.  The library neither frees nor keeps any
 *     caller pointer past the completion of that call's device work; inputs
 *     must stay alive and unchanged until then.
 *   - Every output element is written (-1 marks "no match"), so outputs need
 *     no pre-fill.
 *   - Arguments are validated synchronously.  A call that returns an error has
 *     enqueued nothing.  FT_ERR_DEVICE is sticky: once a HIP call fails the
 *     context reports it from every later call.
 *   - A context is not thread safe; use one context per submitting thread.
 *   - Ties between equal distances go to the smaller candidate index; two
 *     queries that claim one target are resolved in favour of the smaller
 *     (distance, query index) pair and the other becomes unmatched.  Results
 *     are therefore bit-identical run to run and independent of batching.
 */
#ifndef FT_H
#define FT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ft_status;
#define FT_OK 0
#define FT_ERR_INVALID_ARGUMENT 1 /* null/misaligned pointer, bad size or parameter */
#define FT_ERR_CAPACITY 2         /* input exceeds the context's ft_limits */
#define FT_ERR_DEVICE 3           /* a HIP call failed (sticky) */
#define FT_ERR_UNSUPPORTED 4      /* feature or device not supported */

#define FT_LEVELS 8               /* pyramid levels (ORB scale pyramid) */
#define FT_DESC_BYTES 32          /* 256-bit descriptor */

typedef struct ft_context ft_context;

/* Capacity of a context, fixed at creation; the workspace is sized from it. */
typedef struct ft_limits {
    int32_t max_kp_per_image;  /* keypoints per image, <= 65535 */
    int32_t max_map_points;    /* map points per search, <= 8388607 */
    int32_t max_rows;          /* level-0 image rows of a pinhole pair, <= 4096 */
    int32_t max_grid_cells;    /* grid cols * rows, <= 8192 */
    int32_t max_batch_frames;  /* frames per ft_batch_submit */
    int32_t max_inflight;      /* batch tickets in flight at once */
    int32_t max_levels;        /* pyramid levels: must be FT_LEVELS (8) */
    int32_t max_batch_kp_total;   /* keypoints (left + right) of all frames of one batch;
                                     0 = max_batch_frames * 2 * max_kp_per_image */
    int32_t max_batch_map_total;  /* map points of all frames of one batch;
                                     0 = max_batch_frames * max_map_points */
} ft_limits;

/* One image's keypoints (structure of arrays, device memory). */
typedef struct ft_keypoints {
    int32_t n;
    const float *x;            /* [n] level-0 column */
    const float *y;            /* [n] level-0 row */
    const uint8_t *octave;     /* [n] pyramid level */
    const uint8_t *desc;       /* [n][32] descriptor bytes, 16-byte aligned */
} ft_keypoints;

/* Image pyramid kept on the device (Section IV-B: the pyramid built by the
 * feature extractor stays in GPU memory for stereo matching). */
typedef struct ft_pyramid {
    const uint8_t *data;       /* device: every level, row-major, pitch = width */
    int64_t offset[FT_LEVELS]; /* byte offset of each level in data */
    int32_t width[FT_LEVELS];
    int32_t height[FT_LEVELS];
} ft_pyramid;

/* Scale tables of the pyramid (host values). */
typedef struct ft_scales {
    int32_t n_levels;          /* must be FT_LEVELS */
    float sf[FT_LEVELS];       /* scale of level l (sf[0] = 1, increasing) */
    float inv_sf[FT_LEVELS];   /* 1 / sf[l] */
    float sigma2[FT_LEVELS];   /* sf[l]^2 */
} ft_scales;

/* ------------------------------------------------------------------------ */
/* Rectified pinhole stereo (Section II-B: matches lie on epipolar lines, so  */
/* the search is restricted to a region along them; Section IV-C: a best-    */
/* match kernel, then a refinement among nearby pixels in shared memory).    */
/* ------------------------------------------------------------------------ */
typedef struct ft_pinhole_stereo {
    float fx;                  /* focal length in pixels */
    float bf;                  /* baseline * fx; disparity range is [0, bf/b) */
    float b;                   /* baseline in metres */
    int32_t rows;              /* level-0 image height (rows of the row index) */
} ft_pinhole_stereo;

typedef struct ft_pinhole_params {
    int32_t th_orb;            /* accept the best match when distance < th_orb (75) */
    int32_t half_win;          /* patch half size w (5): (2w+1)^2 pixels */
    int32_t half_range;        /* shifts -L..L searched by the refinement (5) */
    int32_t level_window;      /* right level within +-level_window of the left (1) */
    int32_t median_num;        /* reject when median_den*SAD >= median_num*median */
    int32_t median_den;        /*   (21 / 10) */
    float band;                /* right keypoint j covers rows y_j +- band*sf[o_j] (2) */
} ft_pinhole_params;

typedef struct ft_pinhole_out {
    int32_t *right_idx;        /* [nL] matched right keypoint or -1 */
    int32_t *dist;             /* [nL] Hamming distance or -1 */
    float *u_right;            /* [nL] sub-pixel right column or -1 */
    float *depth;              /* [nL] bf / disparity or -1 */
    int32_t *sad;              /* [nL] SAD at the best shift or -1 */
    int32_t *n_matches;        /* [1] number of matched left keypoints */
} ft_pinhole_out;

/* Matches every left keypoint of a rectified pinhole pair: candidates are the
 * right keypoints whose row band covers the left row, at most level_window
 * levels apart, with disparity in [0, bf/b]; the nearest by Hamming distance
 * is refined by a centre-subtracted SAD over shifts -L..L at the left
 * keypoint's pyramid level with a parabola through the best three shifts;
 * duplicates are resolved; outliers above 2.1x the median SAD are dropped.
 * Requirements: L->n, R->n <= max_kp_per_image; cam->rows <= max_rows;
 * scales->n_levels == 8; pyramids hold the level images in bounds.  Errors:
 * FT_ERR_INVALID_ARGUMENT, FT_ERR_CAPACITY, FT_ERR_DEVICE. */
ft_status ft_stereo_match_pinhole(ft_context *ctx, void *stream,
                                  const ft_keypoints *left, const ft_keypoints *right,
                                  const ft_pyramid *pyr_left, const ft_pyramid *pyr_right,
                                  const ft_scales *scales, const ft_pinhole_stereo *cam,
                                  const ft_pinhole_params *params, const ft_pinhole_out *out);

/* ------------------------------------------------------------------------ */
/* Fisheye stereo (Section II-B: for fisheye cameras every right keypoint is  */
/* searched for each left keypoint; Section IV-C: one kernel, no refinement). */
/* ------------------------------------------------------------------------ */
typedef struct ft_kb_intrinsics {
    float fx, fy, cx, cy;      /* Kannala-Brandt: r = f * theta*(1+k1 t^2+k2 t^4+k3 t^6+k4 t^8) */
    float k[4];
} ft_kb_intrinsics;

typedef struct ft_fisheye_stereo {
    ft_kb_intrinsics left, right;
    float R_lr[9];             /* row-major; X_left = R_lr * X_right + t_lr */
    float t_lr[3];
    float overlap_left[2];     /* [a, b]: left keypoints with a <= x <= b are queries */
    float overlap_right[2];    /* [a, b]: right keypoints with a <= x <= b are targets */
} ft_fisheye_stereo;

typedef struct ft_fisheye_params {
    int32_t ratio_num;         /* accept when ratio_den*d1 < ratio_num*d2 (7 / 10) */
    int32_t ratio_den;
    int32_t newton_iters;      /* unprojection Newton iterations (10) */
    int32_t pad_;
    double cos_parallax_max;   /* reject rays more parallel than this (0.9998) */
    double chi2;               /* reprojection gate chi2 * sigma2[level] (5.991) */
    double max_theta;          /* reject unprojected rays at or beyond (rad) */
    double newton_tol;         /* Newton step tolerance (1e-12) */
} ft_fisheye_params;

typedef struct ft_fisheye_out {
    int32_t *right_idx;        /* [nL] matched right keypoint or -1 */
    int32_t *dist;             /* [nL] Hamming distance or -1 */
    float *depth;              /* [nL] left-camera depth or -1 */
    float *xyz;                /* [nL][3] left-camera point, 0 when unmatched */
    int32_t *n_matches;        /* [1] */
} ft_fisheye_out;

/* Two nearest right keypoints (overlap region) of every overlap left keypoint
 * by Hamming distance, computed exactly as an int8 +-1 dot product on the
 * matrix cores; a ratio test; a parallax, triangulation (linear least
 * squares, float64), positive-depth and reprojection check; duplicates
 * resolved.  Errors as for ft_stereo_match_pinhole. */
ft_status ft_stereo_match_fisheye(ft_context *ctx, void *stream,
                                  const ft_keypoints *left, const ft_keypoints *right,
                                  const ft_scales *scales, const ft_fisheye_stereo *cam,
                                  const ft_fisheye_params *params, const ft_fisheye_out *out);

/* ------------------------------------------------------------------------ */
/* Search by projection (Section II-D; Section IV-E: one map point per        */
/* thread-level task, the map split into fine-grained structures).           */
/* ------------------------------------------------------------------------ */
typedef struct ft_map_points {
    int32_t n;
    const float *pos;          /* [n][3] world position */
    const float *normal;       /* [n][3] mean viewing direction (unit) */
    const float *dmin;         /* [n] scale-invariance distance bounds */
    const float *dmax;         /* [n] */
    const uint8_t *desc;       /* [n][32] representative descriptor, 16-byte aligned */
} ft_map_points;

#define FT_CAMERA_PINHOLE 0
#define FT_CAMERA_KB 1

typedef struct ft_search_camera {
    int32_t model;             /* FT_CAMERA_PINHOLE or FT_CAMERA_KB */
    float fx, fy, cx, cy;
    float k[4];                /* KB coefficients (ignored for pinhole) */
    float bf;                  /* pinhole stereo: baseline*fx for the right coordinate */
    float R[9];                /* row-major world-to-camera rotation */
    float t[3];                /* world-to-camera translation */
    float O[3];                /* camera centre in the world */
    float min_x, max_x, min_y, max_y; /* image bounds of a valid projection */
} ft_search_camera;

/* Keypoint grid over the image bounds (floor + clamp cell placement).  It only
 * accelerates the search: the matches are those of a scan over every keypoint.
 * With a level window of at most three octaves the library indexes keypoints
 * per predicted level on a coarser grid of its own (cells merged until eight
 * level bins fit 8192 entries); otherwise it uses this grid as given. */
typedef struct ft_grid {
    int32_t cols, rows;
} ft_grid;

typedef struct ft_search_params {
    float th;                  /* window multiplier (2) */
    float view_cos_limit;      /* reject when viewing cosine < this (0.5) */
    float view_cos_narrow;     /* cosine above which the narrow radius applies (0.998) */
    float r_narrow, r_wide;    /* base radii (2.5, 4.0) */
    float dist_lo, dist_hi;    /* distance gate [dist_lo*dmin, dist_hi*dmax] (0.8, 1.2) */
    int32_t level_lo;          /* keypoint level in [pred-level_lo, pred+level_hi] (1, 1) */
    int32_t level_hi;
    int32_t th_high;           /* accept when distance <= th_high (100) */
    int32_t ratio_num;         /* reject when ratio_den*d1 > ratio_num*d2 (4 / 5) */
    int32_t ratio_den;
    int32_t ratio_same_level_only; /* apply the ratio test only if both share a level */
} ft_search_params;

typedef struct ft_search_out {
    int32_t *mp_match;         /* [n_map] matched keypoint or -1 */
    int32_t *mp_dist;          /* [n_map] Hamming distance or -1 */
    int32_t *kp_match;         /* [n_kp] matched map point or -1 */
    int32_t *n_matches;        /* [1] */
} ft_search_out;

/* Projects every map point with the camera pose, keeps those in the image at
 * a distance inside their scale-invariance range and seen within the viewing
 * angle, predicts the pyramid level, and takes the best and second best
 * keypoints (by Hamming distance) inside a level- and angle-dependent window;
 * keypoints flagged in `preassigned` (device, nullable) are skipped, and when
 * `u_right` (device, nullable) is given, keypoints with u_right > 0 must agree
 * with the projected right coordinate.  Requirements: map->n <=
 * max_map_points, kps->n <= max_kp_per_image, grid cols*rows <=
 * max_grid_cells.  Errors as above. */
ft_status ft_search_local_points(ft_context *ctx, void *stream, const ft_map_points *map,
                                 const ft_search_camera *cam, const ft_keypoints *kps,
                                 const float *u_right, const uint8_t *preassigned,
                                 const ft_grid *grid, const ft_scales *scales,
                                 const ft_search_params *params, const ft_search_out *out);

/* ------------------------------------------------------------------------ */
/* Image pyramid (Section IV-B: the ORB extractor the paper reuses builds the */
/* pyramid on the device and stereo matching reads it there; 90% of stereo's  */
/* input bytes).                                                               */
/* ------------------------------------------------------------------------ */
typedef struct ft_image {
    const uint8_t *data;       /* device, level-0 image, row-major */
    int32_t width, height;     /* 2 <= width <= FT_PYRAMID_MAX_WIDTH, 2 <= height <= 4096 */
    int32_t pitch;             /* bytes from one row to the next, >= width */
} ft_image;

#define FT_PYRAMID_MAX_WIDTH 1536

/* Level sizes and packed offsets of the pyramid of a width x height image:
 * level l is floor(width * inv_sf[l] + 0.5) x floor(height * inv_sf[l] + 0.5)
 * (binary32 product), levels stored row-major one after another from offset
 * 0.  Fills offset, width and height of *pyr (not data) and the total byte
 * count in *bytes.  Host only, no context.  A level of size 0 or a size out of
 * range: FT_ERR_INVALID_ARGUMENT. */
ft_status ft_pyramid_layout(int32_t width, int32_t height, const ft_scales *scales, ft_pyramid *pyr,
                            int64_t *bytes);

/* Builds the pyramid of `image` into pyr->data (device, the layout's bytes;
 * pyr's offsets and sizes must equal ft_pyramid_layout's): level 0 is a copy
 * of the image and every other level a bilinear resample of level 0, all
 * levels in one launch.  The source coordinate of output index x of a level n
 * wide over a level-0 axis N long is (x + 1/2) * N / n - 1/2, taken exactly;
 * the weights are floor(256 * fraction), the taps clamp at the borders, and
 * the value (sum of weight products + 2^15) >> 16.  Every level must be no
 * larger than the image (scale factors >= 1), else FT_ERR_INVALID_ARGUMENT.
 * Errors as above. */
ft_status ft_build_pyramid(ft_context *ctx, void *stream, const ft_image *image, const ft_scales *scales,
                           const ft_pyramid *pyr);

/* ------------------------------------------------------------------------ */
/* Last-frame search by projection (Section II-C, Initial Pose Estimation:   */
/* the previous frame's map points are projected into the current frame and */
/* matched against its keypoints; Section IV-E: one kernel serves both call  */
/* sites).                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct ft_last_points {
    int32_t n;
    const float *pos;          /* [n][3] world position of each matched map point */
    const uint8_t *desc;       /* [n][32] its descriptor, 16-byte aligned */
    const uint8_t *octave;     /* [n] octave of the last-frame keypoint that observed it */
    const float *angle;        /* [n] orientation of that keypoint, degrees (nullable when the
                                  rotation check is off) */
} ft_last_points;

typedef struct ft_last_params {
    float th;                  /* window half-size = th * sf[last octave] (7) */
    int32_t th_high;           /* accept when distance <= th_high (100) */
    int32_t direction;         /* keypoint levels searched: 0 = octave-1..octave+1, 1 = the camera
                                  moves forward: octave..7, -1 = backward: 0..octave */
    int32_t check_orientation; /* 1: keep only matches in the three fullest rotation bins */
    int32_t bins;              /* rotation bins over 360 degrees (30), 1..64 */
} ft_last_params;

/* For every last-frame point: project with the current camera (pinhole or the
 * left/right KB view, as in ft_search_local_points), keep it if in front of
 * the camera and inside the image, and take the best keypoint (distance, then
 * index) inside the window, at the allowed levels, not preassigned and, when
 * `u_right` is given, within the window of the projected right coordinate
 * where u_right > 0; accept at distance <= th_high.  Two points claiming one
 * keypoint: the smaller (distance, point index) keeps it.  With the rotation
 * check, the rotation last angle - current angle (kp_angle, device [kps->n],
 * degrees) of each match falls in bin round(rot * bins / 360) mod bins; the
 * three fullest bins are kept (ties to the lower bin), the second and third
 * only while 10 * count >= the fullest count, and other matches are dropped.
 * Outputs as for ft_search_local_points, indexed by last-frame point
 * (mp_match / mp_dist) and by keypoint (kp_match holds the point index).
 * Requirements: last->n <= max_map_points, kps->n <= max_kp_per_image, grid
 * cols*rows <= max_grid_cells.  Errors as above. */
ft_status ft_search_last_frame(ft_context *ctx, void *stream, const ft_last_points *last,
                               const ft_search_camera *cam, const ft_keypoints *kps, const float *kp_angle,
                               const float *u_right, const uint8_t *preassigned, const ft_grid *grid,
                               const ft_scales *scales, const ft_last_params *params,
                               const ft_search_out *out);

/* ------------------------------------------------------------------------ */
/* Local-map maintenance on the device (Update Local Map's output set kept  */
/* where Search Local Points reads it: Section IV-D, IV-E).                  */
/* ------------------------------------------------------------------------ */
/* The caller's record of which point each slot of a device map holds, for
 * callers that name map points by id (0 .. id_count - 1) rather than by slot:
 * ft_map_update translates removals given as ids and keeps both arrays. */
typedef struct ft_map_ids {
    int32_t *slot_id;          /* HOST [capacity]: point id held by slot s, for s < map->n */
    int32_t *slot_of;          /* HOST [id_count]: slot of point id i, -1 when i is not in the map */
    int32_t id_count;
} ft_map_ids;

typedef struct ft_map_edit {
    int32_t n_remove;
    const int32_t *remove;     /* HOST [n_remove]: slots of the current map (distinct, each < map->n),
                                  or, with `ids`, point ids in the map (distinct) */
    ft_map_points insert;      /* arrays of the insert.n points to append (a map's layout): DEVICE
                                  memory, or HOST memory inside ft_host_alloc blocks (all five), which
                                  the append kernel reads over the bus: no copy command */
    const int32_t *insert_ids; /* with `ids`: HOST [insert.n] ids of the inserted points (distinct,
                                  none in the map); otherwise ignored */
    ft_map_ids *ids;           /* nullable: the slot record, translated and updated by the call */
} ft_map_edit;

/* Edits a device-resident map in place.  The listed points leave the map;
 * with n1 = map->n - n_remove, the removed slots below n1 take the surviving
 * points at or above n1 (the k-th slot in ascending order the k-th point in
 * ascending order) and the inserted points are appended at n1 in order, so
 * the call moves 64 B per removed slot below n1 plus 64 B per inserted point.
 * `map` holds device arrays with room for `capacity` points; map->n (host) is
 * set to n1 + insert.n when the call returns, while the moves run on `stream`
 * (the map must not be read on another stream before they complete; host
 * insert arrays must stay unchanged until then).  The (slot, source) pairs
 * are read by the move kernel from the context's pinned staging, so an edit
 * enqueues two kernels and no copy.  With `edit->ids` the removals are point
 * ids, and slot_id / slot_of are updated on the host for the moved, removed
 * and inserted points only (time proportional to the edit).
 * Errors: a repeated or out-of-range index (or id: outside [0, id_count), not
 * in the map when removed, already in the map when inserted), null or
 * misaligned arrays, host insert arrays partly outside the ft_host_alloc
 * blocks: FT_ERR_INVALID_ARGUMENT; a result above `capacity`, or n_remove or
 * insert.n above max_map_points: FT_ERR_CAPACITY.  On error map->n and the
 * id record are unchanged and nothing is enqueued. */
ft_status ft_map_update(ft_context *ctx, void *stream, ft_map_points *map, int32_t capacity,
                        const ft_map_edit *edit);

/* n edits of n distinct maps in one call (Update Local Map for every frame of
 * a batch): edits[i] is applied to *maps[i] (HOST array of pointers; each
 * map's n is updated) within capacities[i], with ft_map_update's rule and
 * checks.  Every edit is validated before anything is enqueued: on any error
 * no map, no id record changes and nothing is enqueued.  The edits' pairs and
 * appends are staged together in the context's pinned staging, copied to the
 * device in one command, and applied by two kernels for all n maps.  Errors:
 * as ft_map_update, two edits naming one map or sharing an id record:
 * FT_ERR_INVALID_ARGUMENT; more
 * than 4096 edits, or staging above half the context's edit staging (which is
 * max(16 x max_map_points, 8 MiB) bytes; a call stages 88 B per edit, 12 B per
 * moved point and 8 B per inserted point): FT_ERR_CAPACITY. */
ft_status ft_map_update_many(ft_context *ctx, void *stream, int32_t n, ft_map_points *const *maps,
                             const int32_t *capacities, const ft_map_edit *edits);

/* ------------------------------------------------------------------------ */
/* ORB extraction on the device-resident pyramid (Section II-A: keypoints   */
/* extracted on every scale of the pyramid and described; Section IV-B:    */
/* the extraction runs on the device, next to the pyramid stereo reads).    */
/* The paper gives no detector details; this library computes FAST-9        */
/* corners with strict 3x3 suppression, intensity-centroid orientation and  */
/* a descriptor over a caller-supplied pattern turned exactly by it.        */
/* Filtering and distributing the corners is left to the caller.           */
/* ------------------------------------------------------------------------ */
#define FT_ORB_TESTS 256

typedef struct ft_orb_params {
    int32_t threshold;         /* FAST threshold t, 1..254: a corner has nine consecutive ring pixels
                                  (distance 3) all brighter than centre + t or all darker than centre - t */
    int32_t edge;              /* detection window of level l: x in [edge, w_l - edge), y in
                                  [edge, h_l - edge); edge >= 19 */
} ft_orb_params;

typedef struct ft_orb_corners {
    int32_t capacity;          /* entries of each output array */
    int16_t *lx, *ly;          /* DEVICE [capacity]: column and row on the corner's level */
    uint8_t *octave, *score;   /* DEVICE [capacity]: level; FAST score (the largest threshold it passes) */
    float *x, *y;              /* DEVICE [capacity]: lx * sf[level], ly * sf[level] (binary32) */
    int32_t *count;            /* DEVICE [1]: corners found; when above capacity, the first capacity
                                  (in order) are written */
} ft_orb_corners;

/* Detects the corners of every level of `pyr` (device, the packed layout of
 * ft_pyramid_layout or any per-level layout with widths <= FT_PYRAMID_MAX_WIDTH):
 * a pixel of the window is a corner when its FAST-9 score (over the 16 arcs of
 * nine ring pixels and both signs, the largest smallest difference from the
 * centre, minus one) reaches the threshold, and it is kept when its score
 * exceeds each of its 8 neighbours' (non-corners count 0).  Corners are
 * written in (level, row, column) order.  When `blurred` (DEVICE, the
 * pyramid's layout) is not null it receives every level smoothed for the
 * descriptor: the separable binomial [1 6 15 20 15 6 1] / 64 per direction,
 * borders clamped, rounded once ((sum + 2^11) >> 12).  Two kernels on
 * `stream`; *count and the outputs are valid when they complete.  Errors:
 * bad threshold, edge, pyramid or null / misaligned outputs (lx, ly 2-byte,
 * x, y, count 4-byte aligned): FT_ERR_INVALID_ARGUMENT; a level above
 * FT_PYRAMID_MAX_WIDTH x 4096: FT_ERR_CAPACITY.  Up to 8 detections may be
 * in flight per context (a ninth waits for the first to complete). */
ft_status ft_orb_detect(ft_context *ctx, void *stream, const ft_pyramid *pyr, const ft_scales *scales,
                        const ft_orb_params *params, uint8_t *blurred, const ft_orb_corners *out);

/* Orientation and descriptor of keypoints on the pyramid's levels (for
 * example the output of ft_orb_detect, filtered or not): n = n_max, or
 * min(n_max, *count) when `count` (DEVICE) is not null.  Orientation: the
 * intensity centroid over the disc dx^2 + dy^2 <= 225 of the level image,
 * angle[i] = atan2(m01, m10) in degrees, [0, 360].  Descriptor (32 bytes, bit
 * t in bit t % 8 of byte t / 8): test t of `pattern` (HOST int8
 * [FT_ORB_TESTS][4] = x1, y1, x2, y2, each point within radius 13) turns both
 * points exactly by the centroid angle (each coordinate the integer nearest
 * (x m10 - y m01) / |m| and (x m01 + y m10) / |m|, halves away from zero; no
 * turn when m = 0) and sets the bit when `blurred` (DEVICE, from
 * ft_orb_detect) is darker at the first point than at the second.  A keypoint
 * closer than 15 pixels to its level's border, or of a level >= FT_LEVELS,
 * gets angle -1 and a zero descriptor.  Errors: null or misaligned arrays
 * (desc 8-byte aligned), a pattern point beyond radius 13:
 * FT_ERR_INVALID_ARGUMENT. */
ft_status ft_orb_describe(ft_context *ctx, void *stream, const ft_pyramid *pyr, const uint8_t *blurred,
                          int32_t n_max, const int32_t *count, const int16_t *lx, const int16_t *ly,
                          const uint8_t *octave, const int8_t *pattern, float *angle, uint8_t *desc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid allocation): the search of
 * ft_search_local_points, same kernels and bit-identical outputs, with no
 * context.  Its workspace is a fixed device array that every GPU the library
 * runs on holds for the life of the process (FT_NOALLOC_SCRATCH_BYTES, 1 MiB);
 * the call allocates nothing and runs on the calling thread's current device.
 * Limits: kps->n <= FT_NOALLOC_MAX_KP, map->n <= FT_NOALLOC_MAX_MAP, grid
 * cols*rows <= 8192, else FT_ERR_CAPACITY with nothing enqueued; other errors
 * as for ft_search_local_points (FT_ERR_UNSUPPORTED on a device that is not
 * gfx950).  Every call on one GPU uses that GPU's one array, so two calls
 * whose device work overlaps (different streams, or different threads) race
 * and both outputs are undefined: order them on one stream.  The array holds
 * whatever the last call left; the kernels initialise every part they read.
 * The text of the last error of this entry point on the calling thread is
 * ft_last_error(NULL). */
#define FT_NOALLOC_MAX_KP 8192
#define FT_NOALLOC_MAX_MAP 65536
#define FT_NOALLOC_SCRATCH_BYTES 1048576
ft_status ft_search_local_points_noalloc(void *stream, const ft_map_points *map,
                                         const ft_search_camera *cam, const ft_keypoints *kps,
                                         const float *u_right, const uint8_t *preassigned,
                                         const ft_grid *grid, const ft_scales *scales,
                                         const ft_search_params *params, const ft_search_out *out);

/* ------------------------------------------------------------------------ */
/* Batched frames: many frames of uneven size in one submission.             */
/* ------------------------------------------------------------------------ */
#define FT_JOB_PINHOLE 1       /* pinhole stereo + left-view search */
#define FT_JOB_FISHEYE 2       /* fisheye stereo + left- and right-view search */
#define FT_JOB_SEARCH 3        /* search only (views as given) */

typedef struct ft_frame_job {
    int32_t kind;              /* FT_JOB_* */
    int32_t n_views;           /* search views: 1 (left) or 2 (left, right) */
    ft_keypoints left, right;
    ft_scales scales;
    /* pinhole stereo */
    ft_pyramid pyr_left, pyr_right;
    ft_pinhole_stereo pinhole;
    ft_pinhole_params pinhole_params;
    ft_pinhole_out pinhole_out;
    int32_t use_u_right;       /* pinhole: gate the left view with the stereo u_right */
    int32_t build_pyramids;    /* pinhole: build pyr_left / pyr_right from image_left /
                                  image_right first (as ft_build_pyramid) */
    ft_image image_left, image_right;
    /* fisheye stereo */
    ft_fisheye_stereo fisheye;
    ft_fisheye_params fisheye_params;
    ft_fisheye_out fisheye_out;
    /* search by projection (view 0 uses `left`, view 1 uses `right`) */
    ft_map_points map;
    ft_search_camera cam[2];
    ft_grid grid[2];
    const uint8_t *preassigned[2];
    ft_search_params search_params;
    ft_search_out search_out[2];
} ft_frame_job;

/* Enqueues every job on `stream` as one batch and returns a ticket.  Results
 * are bit-identical to running each job through the single-frame calls.
 * Requires n <= max_batch_frames and a free in-flight slot (else
 * FT_ERR_CAPACITY).  The job array is copied during the call. */
ft_status ft_batch_submit(ft_context *ctx, void *stream, const ft_frame_job *jobs,
                          int32_t n, uint64_t *ticket);
/* Non-blocking: *done = 1 when the ticket's work has completed. */
ft_status ft_batch_poll(ft_context *ctx, uint64_t ticket, int32_t *done);
/* Blocks until the ticket's work has completed. */
ft_status ft_batch_wait(ft_context *ctx, uint64_t ticket);

/* How a batch is executed on the device:
 *   FT_EXEC_EAGER  the table upload and one kernel per phase, launched on the
 *                  stream one by one;
 *   FT_EXEC_GRAPH  the same work as one HIP graph launch (the default).  Each
 *                  in-flight lane holds one instantiated graph, built when the
 *                  context is created and rebuilt only by ft_set_shapes and
 *                  ft_autotune; a submission updates the graph's nodes (table
 *                  size, grid of every phase) in place and launches it, so
 *                  batches of any shape run without capture or allocation.
 * Results are identical in both modes.  While per-phase timing is enabled,
 * graph batches run eagerly so that each phase can be bracketed by events.
 * Returns FT_ERR_INVALID_ARGUMENT for an unknown mode. */
#define FT_EXEC_EAGER 0
#define FT_EXEC_GRAPH 1
ft_status ft_set_exec_mode(ft_context *ctx, int32_t mode);
ft_status ft_get_exec_mode(const ft_context *ctx, int32_t *mode);

/* Launch shapes of the batch kernels.  Results never depend on them, only the
 * time does. */
typedef struct ft_shapes {
    int32_t best_lanes;        /* lanes per pinhole left keypoint of the best match:
                                  1, 2, 4, 8 or 16 */
    int32_t search_lanes;      /* lanes per map point of the search: 1 (record-dealt: a wave deals
                                  its 64 map points' window records evenly over its lanes),
                                  2, 4, 8 or 16 (lane groups stride each window) */
    int32_t aux_block;         /* threads per workgroup of the setup sorts and the stereo
                                  resolve: 256 or 1024 */
} ft_shapes;

/* A new context starts with best_lanes 8, search_lanes 1, aux_block 1024 (the
 * shapes the autotuner picks for mixed pinhole/fisheye batches).  Setting
 * shapes rebuilds the in-flight lanes' batch graphs (a set-up call: it waits
 * for the batches in flight, and graph instantiation may allocate). */
ft_status ft_set_shapes(ft_context *ctx, const ft_shapes *shapes);
ft_status ft_get_shapes(const ft_context *ctx, ft_shapes *shapes);

/* Autotuner: runs the given batch once per candidate shape (outputs are
 * overwritten; the call synchronizes `stream`), times the affected kernels
 * with HIP events and keeps the fastest shapes in the context.  When
 * `cache_path` is non-null it is a JSON file keyed by device and workload
 * class (frame count and mean keypoint / map sizes in powers of two): a cached
 * entry is used without timing, a new one is appended.  `chosen` (nullable)
 * receives the shapes in use.  Errors as for ft_batch_submit, plus
 * FT_ERR_INVALID_ARGUMENT for an unreadable or unwritable cache. */
ft_status ft_autotune(ft_context *ctx, void *stream, const ft_frame_job *jobs, int32_t n,
                      const char *cache_path, ft_shapes *chosen);

/* ------------------------------------------------------------ frame upload
 * A tracker hands each frame's keypoints to the GPU once (Section IV-E: move
 * only the data the kernels need).  When many camera streams are served, the
 * frames of one batch sit in separate host buffers, and one copy command per
 * frame costs a command submission each; ft_upload moves a whole gather list
 * with one kernel that reads pinned host memory directly over the bus.
 *
 * ft_host_alloc returns `bytes` of pinned (page-locked, device-mapped) host
 * memory owned by the context; it stays valid until ft_host_free or
 * ft_context_destroy.  It is the only memory an ft_upload source may lie in,
 * so the library can check every source range.  Allocate at set-up: like
 * ft_context_create it allocates, no other call does.  bytes <= 0 or a null
 * ptr: FT_ERR_INVALID_ARGUMENT; allocation failure: FT_ERR_DEVICE.
 * ft_host_free of a pointer that ft_host_alloc did not return, or that was
 * freed already: FT_ERR_INVALID_ARGUMENT.  The caller must not free memory
 * that an enqueued upload still reads. */
typedef struct ft_segment {
    const void *src;           /* pinned host memory from ft_host_alloc, 16-byte aligned */
    void *dst;                 /* device memory, 16-byte aligned */
    int64_t bytes;             /* >= 0; [src, src + bytes) inside one ft_host_alloc block */
} ft_segment;

ft_status ft_host_alloc(ft_context *ctx, int64_t bytes, void **ptr);
ft_status ft_host_free(ft_context *ctx, void *ptr);
/* Enqueues the copy of every segment on `stream` (one kernel per 64
 * segments); the segments list itself is read during the call.  The
 * destinations must not overlap each other; the sources must stay unchanged
 * until the stream has passed the copy.  n == 0 enqueues nothing.  A null
 * list with n > 0, n < 0, a misaligned pointer, a negative size or a source
 * range outside every ft_host_alloc block: FT_ERR_INVALID_ARGUMENT, and
 * nothing is enqueued. */
ft_status ft_upload(ft_context *ctx, void *stream, const ft_segment *segs, int32_t n);

/* ------------------------------------------------------------------------ */
ft_status ft_context_create(const ft_limits *limits, int32_t device, ft_context **out);
ft_status ft_context_destroy(ft_context *ctx);
/* Device bytes held by the context's preallocated workspace. */
ft_status ft_context_workspace_bytes(const ft_context *ctx, int64_t *bytes);
const char *ft_status_string(ft_status status);
const char *ft_last_error(const ft_context *ctx);
/* Per-phase kernel timing (for measurement tools).  When enabled, every
 * submission records HIP events on its own stream around each phase kernel:
 * 0 image pyramids (jobs that build them), 1 setup (row index / overlap
 * lists / grids), 2 stereo best match (pinhole row band or fisheye
 * all-pairs), 3 pinhole refinement, 4 fisheye triangulation check, 5 stereo
 * resolve + outputs, 6 search by projection, 7 search resolve + outputs.
 * ft_context_read_timing waits for the recorded work, returns the summed
 * milliseconds and launch counts per phase (arrays of FT_PHASES), and resets
 * them.  Enabling timing adds event records between kernels. */
#define FT_PHASES 8
ft_status ft_context_enable_timing(ft_context *ctx, int32_t enable);
ft_status ft_context_read_timing(ft_context *ctx, double *ms, int64_t *launches);
/* Library version as major*10000 + minor*100 + patch. */
int32_t ft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FT_H */
