/* Plain, slow, single-threaded CPU oracle of the tracking correspondence search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant with the
 * device path.
 *
 * What it computes (the paper's problem statements, Section II-B to II-D and
 * Section IV-C/IV-E of FastTrack, arXiv 2509.10757):
 *   - stereo matching: for each left keypoint, the most similar right keypoint
 *     (pinhole: restricted to the epipolar row band, then refined among nearby
 *     pixels; fisheye: brute force over the overlap region);
 *   - search by projection: for each local map point, its correspondence among
 *     the frame's keypoints, each map point independent of the others.
 * Every search is an exhaustive scan over the candidate set that the
 * predicates define (no row index, no grid: those are accelerators of the
 * device path).  Ties go to the smaller candidate index; two queries that
 * claim one target are resolved in favour of the smaller (distance, query
 * index) key and the loser becomes unmatched.
 *
 * Arithmetic: binary32 for pinhole and projection steps, binary64 for the
 * Kannala-Brandt model and triangulation; every expression is evaluated left
 * to right as written, built with -ffp-contract=off (no fused multiply-add).
 *
 * Parity pinning: see the header comment of each function; functions whose
 * result has no independent pin say "parity unpinned".
 */
#ifndef FT_ORACLE_H
#define FT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int oracle_hamming(const uint8_t *a, const uint8_t *b);

/* Rectified pinhole stereo.  i-params: th_orb, half_win, half_range,
 * level_window, median_num, median_den.  stats (int64[8]): hamming evals,
 * refine attempts, refined ok, after conflict, median, final matches. */
void oracle_stereo_pinhole(
    int nL, const float *xL, const float *yL, const uint8_t *oL, const uint8_t *dL,
    int nR, const float *xR, const float *yR, const uint8_t *oR, const uint8_t *dR,
    const uint8_t *pyrL, const uint8_t *pyrR, const int64_t *lv_off,
    const int32_t *lv_w, const int32_t *lv_h, const float *sf, const float *inv_sf,
    float bf, float b, int rows, const int32_t *ip, float band,
    int32_t *out_j, int32_t *out_h, float *out_ur, float *out_depth, int32_t *out_sad,
    int64_t *stats);

/* Fisheye (Kannala-Brandt) stereo.  kb = {fx, fy, cx, cy, k1, k2, k3, k4}.
 * ip = {ratio_num, ratio_den, newton_iters}; dp = {cos_parallax_max, chi2,
 * max_theta_rad, newton_tol}.  out_h2 (nullable): second-nearest distance of
 * every overlap query (-1 elsewhere).  stats: |Q|, |T|, ratio ok, tri ok, final,
 * then the queries past the ratio test rejected by the parallax test, by a
 * depth <= 0 in either camera, and by the reprojection test of either view. */
void oracle_stereo_fisheye(
    int nL, const float *xL, const float *yL, const uint8_t *oL, const uint8_t *dL,
    int nR, const float *xR, const float *yR, const uint8_t *oR, const uint8_t *dR,
    const float *kbL, const float *kbR, const float *R_lr, const float *t_lr,
    const float *ovl, const float *ovr, const float *sigma2,
    const int32_t *ip, const double *dp,
    int32_t *out_j, int32_t *out_h, float *out_depth, float *out_xyz, int32_t *out_h2,
    int64_t *stats);

/* Local-map search by projection for one camera.
 * cam = {fx, fy, cx, cy, k1, k2, k3, k4, bf}; model 0 = pinhole, 1 = KB.
 * fp = {th, view_cos_limit, view_cos_narrow, r_narrow, r_wide, dist_lo, dist_hi}
 * ip = {level_lo, level_hi, th_high, ratio_num, ratio_den, same_level_only}
 * stats: visible, candidates, accepted before conflict, matches, then the
 * map points rejected by each visibility test in order: behind the camera or
 * outside the image bounds, nearer than dist_lo*dmin, farther than
 * dist_hi*dmax, viewing cosine below the limit. */
void oracle_search_local_points(
    int nM, const float *pos, const float *normal, const float *dmin, const float *dmax,
    const uint8_t *mdesc,
    int nK, const float *kx, const float *ky, const uint8_t *ko, const uint8_t *kdesc,
    const float *u_right, const uint8_t *preassigned,
    int model, const float *cam, const float *R, const float *t, const float *O,
    const float *bounds, const float *sf, int n_levels,
    const float *fp, const int32_t *ip,
    int32_t *mp_match, int32_t *mp_dist, int32_t *kp_match, int64_t *stats);

/* Search by projection of the last frame's matched map points into the
 * current frame (Section II-C, Initial Pose Estimation; Section IV-E: the same
 * kernel serves both call sites).  Last-frame point i has world position
 * lpos[i], descriptor ldesc[i], and the octave lo[i] and orientation la[i]
 * (degrees) of the last-frame keypoint that observed it.  For each point:
 * project with the current pose (as in the local-map search); keep it if
 * Z_c > 0 and inside the image bounds; radius th * sf[lo[i]]; keypoint levels
 * [lo - 1, lo + 1] (direction 0), [lo, n_levels - 1] (1, camera moving
 * forward) or [0, lo] (-1, moving backward); candidates |x - u| < r,
 * |y - v| < r, not preassigned, and within r of the projected right
 * coordinate where u_right > 0; best (distance, keypoint) accepted when
 * distance <= th_high.  Two points claiming one keypoint: the smaller
 * (distance, point) key keeps it.  Then, when check_orientation is set, the
 * rotation rot = la[i] - ka[k] (plus 360 when negative) of every surviving
 * match falls in bin roundf(rot * bins / 360) mod bins; the
 * three fullest bins are kept (ties: the lower bin), the second and third
 * only while 10 * count >= the fullest count; matches in other bins are
 * dropped.  cam, model, R, t, bounds as for oracle_search_local_points.
 * fp = {th}; ip = {th_high, direction, check_orientation, bins}.
 * stats: projected inside the image, candidates, accepted, after the
 * conflict rule, after the rotation check, then the three kept bins. */
void oracle_search_last_frame(
    int nL, const float *lpos, const uint8_t *ldesc, const uint8_t *lo, const float *la,
    int nK, const float *kx, const float *ky, const uint8_t *ko, const uint8_t *kdesc,
    const float *ka, const float *u_right, const uint8_t *preassigned,
    int model, const float *cam, const float *R, const float *t, const float *bounds,
    const float *sf, int n_levels, const float *fp, const int32_t *ip,
    int32_t *l_match, int32_t *l_dist, int32_t *kp_match, int64_t *stats);

/* Local-map maintenance in place (Update Local Map's output set kept where
 * the search reads it; Section IV-D and IV-E).  The map is SoA (pos [n][3],
 * normal [n][3], dmin, dmax, desc [n][32]) with room for `capacity` points.
 * The n_remove indices in `remove` (distinct, each < n) leave the map; with
 * n1 = n - n_remove, the removed slots below n1 ("holes", ascending) take the
 * surviving points at or above n1 ("sources", ascending), the k-th hole the
 * k-th source; then the n_insert new points are appended at n1, in order.
 * Returns the new count n1 + n_insert, or -1 (map untouched) when an index is
 * out of range or repeated or the result exceeds the capacity.  Pinned by
 * invariants: the new map holds exactly the surviving and inserted records,
 * survivors below n1 keep their slots, holes take the tail survivors in
 * order, inserted points follow in order; edge cases (nothing, everything,
 * only head or only tail points removed, exact capacity, invalid lists). */
int oracle_map_update(int n, int capacity, float *pos, float *normal, float *dmin, float *dmax, uint8_t *desc,
                      int n_remove, const int32_t *remove, int n_insert, const float *ipos,
                      const float *inormal, const float *idmin, const float *idmax, const uint8_t *idesc);

/* Rotation bin of a match and the bins kept by the three-fullest rule, exposed
 * so tests can pin them on their own. */
int oracle_rotation_bin(float a_last, float a_cur, int bins);
void oracle_three_fullest(const int32_t *count, int bins, int32_t *kept);

/* Stage helpers of the pinhole refinement and of the level prediction,
 * exported so tests can pin each stage on its own. */
int oracle_sad_window(const uint8_t *IL, const uint8_t *IR, int Wl, int Hl,
                      int su, int sv, int su0, int w, int L, int *sad);
int oracle_subpixel(const int *sad, int L, int *kbest, int *sad_best, float *delta);
int oracle_median_keep(int n, const int32_t *sad, int num, int den, uint8_t *keep);
int oracle_predict_level(float ratio, const float *sf, int n_levels);

/* Image pyramid (Section IV-B: the pyramid is built on the device and kept
 * there for stereo matching; the extractor it reuses computes every level at
 * once).  Level l is round(W * inv_sf[l]) x round(H * inv_sf[l]) (binary32
 * product, then floor(v + 0.5)); level 0 is the image; every other level is a
 * bilinear resample of level 0 with pixel centres aligned, source coordinate
 * s = (x + 1/2) * W / w - 1/2 taken exactly as a fraction, 8-bit weights
 * floor(256 * frac(s)), clamp at the borders, and the result rounded as
 * (v + 2^15) >> 16.  oracle_pyramid_layout fills the level sizes and packed
 * offsets and returns the total byte count; oracle_pyramid writes the levels
 * (img row-major with `pitch` bytes per row).  Pinned by closed forms:
 * constant images, linear ramps (round-half-up of the exact source
 * coordinate), exact 2x downscaling (rounded 2x2 box average), the level
 * sizes of the paper's image shapes, and a numpy brute force. */
int64_t oracle_pyramid_layout(int W, int H, const float *inv_sf, int n_levels,
                              int32_t *w, int32_t *h, int64_t *off);
void oracle_pyramid(const uint8_t *img, int W, int H, int pitch, const float *inv_sf, int n_levels,
                    uint8_t *out);

/* ORB extraction on the pyramid (Section II-A: keypoints are extracted on
 * every scale of the image pyramid and each gets a descriptor; Section IV-B:
 * the extraction runs on the device, next to the pyramid).  The paper gives
 * no detector, score, orientation or descriptor details; the readings:
 *   - FAST-9 score of a pixel: the ring of 16 pixels at distance 3, the
 *     largest (over the 16 arcs of nine consecutive ring pixels and both
 *     signs) smallest difference ring - centre (or centre - ring) minus one;
 *     a corner when the score reaches the threshold t (1..254), i.e. nine
 *     consecutive ring pixels all brighter than centre + t or all darker than
 *     centre - t;
 *   - detection window of level l: x in [edge, w_l - edge), y in
 *     [edge, h_l - edge) with edge >= 19 (the orientation disc and the turned
 *     pattern plus the smoothing stay inside the level);
 *   - non-maximum suppression: a corner is kept when its score exceeds the
 *     score of each of its 8 neighbours (non-corners count 0), so plateaus
 *     of equal scores keep none;
 *   - order: (level, y, x); coordinates lx, ly on the level and x = lx *
 *     sf[l], y = ly * sf[l] in binary32; when more than `cap` corners exist
 *     the first cap are written and the count is returned;
 *   - orientation: intensity centroid over the disc dx^2 + dy^2 <= 225 of the
 *     level image: m10 = sum dx I, m01 = sum dy I (exact integers); angle =
 *     atan2(m01, m10) in degrees (binary64, times 180 / pi, plus 360 when
 *     negative), stored in binary32;
 *   - smoothing for the descriptor: per level, the separable binomial
 *     [1 6 15 20 15 6 1] horizontally then vertically, borders clamped,
 *     rounded once: (sum + 2^11) >> 12;
 *   - descriptor: 256 tests of a caller-supplied pattern of point pairs
 *     (x1, y1, x2, y2), each point within radius 13; each point is turned by
 *     the centroid angle exactly: column = the integer nearest (x m10 -
 *     y m01) / sqrt(m10^2 + m01^2), row = the integer nearest (x m01 +
 *     y m10) / sqrt(...), halves away from zero, decided in integers (no
 *     turn when m10 = m01 = 0); bit t (bit t % 8 of byte t / 8) is set when
 *     the smoothed level is darker at the first turned point than at the
 *     second.
 * Pinned by closed forms (a lone bright pixel, straight edges, the strict
 * threshold, invariance under an added constant, inversion, transposition
 * and half turns; orientation of linear ramps in four directions, the disc's
 * size; the blur of impulses, constants and ramps; descriptors of ramps, which
 * equal the unturned pattern's x order in every direction), by an
 * independent numpy brute force, and by planted mistakes. */
void oracle_fast_score_map(const uint8_t *img, int w, int h, int t, int edge, uint8_t *out);
int64_t oracle_orb_detect(const uint8_t *pyr, const int64_t *off, const int32_t *w, const int32_t *h,
                          int n_levels, const float *sf, int t, int edge, int64_t cap, int16_t *lx,
                          int16_t *ly, uint8_t *oct, uint8_t *score, float *x, float *y);
void oracle_orb_blur(const uint8_t *img, int w, int h, uint8_t *out);
void oracle_orb_describe(const uint8_t *pyr, const uint8_t *blurred, const int64_t *off, const int32_t *w,
                         int n, const int16_t *lx, const int16_t *ly, const uint8_t *oct,
                         const int8_t *pattern, float *angle, uint8_t *desc);

/* Kannala-Brandt helpers, exposed so tests can pin them (round trips). */
int oracle_kb_unproject(const float *kb, float u, float v, int iters, double tol,
                        double max_theta, double *ray);
void oracle_kb_project(const float *kb, const double *X, double *uv);
int oracle_triangulate(const double *r1, const double *r2, const float *R_lr,
                       const float *t_lr, double *X);

#ifdef __cplusplus
}
#endif
#endif
