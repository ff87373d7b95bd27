/* C ABI of the front end of the pose-graph library: keypoint descriptor
 * matching and coarse registration by RANSAC (Sec. IV-B), keyframe selection
 * and the novelty test of the memory pool (Sec. IV-C, IV-E) of BundleTrack
 * (Wen & Bekris, IROS 2021), on the GPU.
 * Same library and status codes as posegraph.h. */
#ifndef PG_FRONTEND_H
#define PG_FRONTEND_H

#include "posegraph.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PG_MATCH_MAX_PAIRS 96       /* descriptor-set pairs per call                   */
#define PG_MATCH_MAX_ROWS 4096      /* descriptors per set                             */
/* partial column minima the allocation-free variant holds: sum over the pairs
 * of ceil(rows of set a / 64) x rows of set b */
#define PG_MATCH_SCRATCH_PARTIALS (1 << 19)
/* rows the allocation-free variant holds: sum over the pairs of rows of set a */
#define PG_MATCH_SCRATCH_ROWS (1 << 16)

/* Mutual nearest-neighbour matching of keypoint descriptors (Sec. IV-B: the
 * keypoints of the current frame are matched against those of the keyframes
 * on the GPU, several pairs at once).  For pair q, with A = descriptor set
 * pair_a[q] (na rows) and B = set pair_b[q] (nb rows): row x of A is matched
 * to the row y of B nearest to it in squared Euclidean distance (lowest y
 * among equal distances) when x is also the row of A nearest to y (lowest x
 * among equals) and, for ratio < 1, when d1 < ratio^2 d2 (d1, d2: the
 * squared distances from x to its nearest and second-nearest rows of B, the
 * second equal to the first when two rows of B tie); else -1.  Distances are
 * FP64, |a|^2 + |b|^2 - 2 a.b with the dot products on the FP64 matrix cores
 * (rounding-level differences from the difference form can change a decision
 * only between near-equal distances).
 *
 *   desc      device memory, FP32, row-major: set s is rows set_off[s] ..
 *             set_off[s + 1] - 1, dim values per row
 *   set_off   host array of n_sets + 1 non-decreasing row offsets (set_off[0]
 *             is the first row used), each set at most PG_MATCH_MAX_ROWS rows
 *   dim       32, 64, 128 or 256
 *   pair_a, pair_b   host arrays of n_pairs set indices (1..PG_MATCH_MAX_PAIRS
 *             pairs; a set may be matched against itself)
 *   ratio     ratio test threshold; >= 1 disables the test
 *   match     device memory, int32: pair q's na results at out_off(q) = sum of
 *             the na of pairs before q (local row indices of B, or -1)
 *   d1, d2    device memory, FP64, same layout; may be NULL; infinity where
 *             B is empty (and d2 where B has one row)
 *   hip_stream   the stream the work is ordered on (NULL: the null stream);
 *             the call returns once the work is enqueued
 * Ownership stays with the caller; nothing is kept after the call.  Errors:
 * PG_ERR_INVALID_ARG (null, host or out-of-range pointers and sizes),
 * PG_ERR_CAPACITY (limits above), PG_ERR_OUT_OF_MEMORY / PG_ERR_HIP.
 * The scratch of the column minima is allocated and freed on the stream. */
pg_status pg_match_descriptors(const float* desc, const int* set_off, int n_sets, int dim, const int* pair_a,
                               const int* pair_b, int n_pairs, double ratio, int* match, double* d1, double* d2,
                               void* hip_stream);

/* pg_match_descriptors for callers that cannot allocate device memory (code
 * under stream capture, serving loops): the same results from the same
 * kernels, with the scratch in a fixed array of the library on each device
 * (PG_MATCH_SCRATCH_PARTIALS column minima, PG_MATCH_SCRATCH_ROWS rows; about
 * 9.5 MB, held until the process ends).  Larger calls fail with
 * PG_ERR_CAPACITY.  Calls that overlap on one device share that array and
 * race: order them on one stream. */
pg_status pg_match_descriptors_noalloc(const float* desc, const int* set_off, int n_sets, int dim,
                                       const int* pair_a, const int* pair_b, int n_pairs, double ratio, int* match,
                                       double* d1, double* d2, void* hip_stream);

#define PG_RANSAC_MAX_MATCHES 512   /* matches of one pair                              */
#define PG_RANSAC_MAX_HYP 8192      /* hypotheses per pair                              */

/* Coarse registration by RANSAC (Sec. IV-B): for each of n_pairs ordered node
 * pairs (pi[q], pj[q]) of graph g, its matched keypoints (pixel coordinates
 * uv_i in frame pi[q], uv_j in frame pj[q], entries match_off[q] ..
 * match_off[q + 1] - 1, at most PG_RANSAC_MAX_MATCHES) are lifted to 3-D
 * points and normals at their nearest pixels (pi_D^-1 of Eq. 3; a match is
 * valid when both pixels hold a valid point).  Hypothesis h of pair q is the
 * least-squares rigid transform (Arun et al.) of the three matches
 * samples[3 (q n_hyp + h) ..] (indices local to the pair; the random draws are
 * the caller's), unusable (score -1) when a match is invalid or repeated or
 * either triangle has an area below 1e-8 m^2; its score is the number of
 * valid matches m with |R b_m + t - a_m| < delta_m and
 * (R n_b) . n_a > cos(alpha_rad) (a: point in frame pi, b: in frame pj).
 *   best[q]    the hypothesis with the highest score (lowest index among
 *              equals), -1 when none is usable
 *   T[16 q..]  its transform, frame pj camera -> frame pi camera, row-major
 *              4 x 4 FP64 (the identity when best[q] is -1)
 *   score      n_pairs x n_hyp scores, may be NULL
 *   inlier     one byte per match (match_off layout), the best hypothesis'
 *              inlier flags, may be NULL
 *   install    nonzero: each pair with a usable hypothesis gets its inliers
 *              as the feature matches of the pair (Eq. 2; the C_ij the
 *              optimisation reuses), replacing earlier ones (none: removed)
 * All arrays are host memory, copied; the call is synchronous on the graph's
 * stream.  Rounding-level differences from an FP64 reference can change a
 * decision only for matches at the delta or alpha boundary.  Errors:
 * PG_ERR_INVALID_ARG, PG_ERR_CAPACITY (limits above), PG_ERR_OUT_OF_MEMORY,
 * PG_ERR_HIP; the message is pose_graph_last_error(g). */
pg_status pose_graph_ransac(pg_graph* g, int n_pairs, const int* pi, const int* pj, const int* match_off,
                            const float* uv_i, const float* uv_j, int n_hyp, const int* samples, double delta_m,
                            double alpha_rad, int install, int* best, int* score, double* T, uint8_t* inlier);

#define PG_POOL_MAX 2048            /* keyframes of a memory pool                       */

/* Keyframe selection from the memory pool (Sec. IV-C) and the novelty test of
 * its augmentation (Sec. IV-E), on the GPU.  The geodesic distance of two
 * poses' rotations is arccos((tr(R_a^T R_b) - 1) / 2) (cosine clamped to
 * [-1, 1]).  Starting from {keyframe 0} (the initial frame, always kept),
 * the keyframe with the smallest sum of geodesic distances to the current
 * frame and to every keyframe selected so far is added (lowest index among
 * equal sums) until min(K, n_pool) are selected: the paper's greedy
 * solution of the minimum H-subgraph problem.
 *   T_pool     n_pool poses, 16 doubles each (row-major 4 x 4, object ->
 *              camera), host or device memory (copied)
 *   T_cur      the current frame's pose (16 doubles, host)
 *   selected   host, K entries: pool indices in selection order; n_selected
 *              receives their count
 *   novel      host, may be NULL: 1 when every keyframe is farther than
 *              novel_rad from the current frame (the frame joins the pool)
 *   cost       host, may be NULL, n_pool entries: each keyframe's final sum
 *              (a selected keyframe's as it was when chosen)
 * Synchronous on hip_stream (NULL: the null stream).  Errors:
 * PG_ERR_INVALID_ARG, PG_ERR_CAPACITY (n_pool > PG_POOL_MAX), PG_ERR_HIP. */
pg_status pg_select_keyframes(const double* T_pool, int n_pool, const double* T_cur, int K, double novel_rad,
                              int* selected, int* n_selected, int* novel, double* cost, void* hip_stream);

/* Message of the last failed front-end call on this thread ("" if none). */
const char* pg_frontend_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PG_FRONTEND_H */
