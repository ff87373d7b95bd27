/*
 * FP64 CPU oracle for the online pose-graph optimisation of BundleTrack
 * (Wen & Bekris, IROS 2021), Sec. IV-D: the total energy of Eq. (1), the
 * feature term of Eq. (2), the dense point-to-plane term of Eq. (3), and the
 * IRLS Gauss-Newton iteration with the first keyframe held fixed.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library never does,
 * and the two share no source.
 *
 * Conventions (the readings of the paper this oracle fixes):
 *   pose T maps object to camera, x_cam = R x_obj + t, 4x4 row-major doubles;
 *   twist xi = [v; w] (translation first), update T <- Exp(delta) T;
 *   Gauss-Newton step delta = -(J^T W J)^-1 J^T W r over the free nodes.
 */
#ifndef BT_ORACLE_H
#define BT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_SINGULAR = -5 };

/* One keyframe window and the method's parameters.  All arrays are borrowed. */
typedef struct {
    int n_frames, width, height;
    double fx, fy, cx, cy;
    const float *depth;          /* n_frames*H*W, metres; 0 or non-finite = no depth */
    const unsigned char *mask;   /* n_frames*H*W, nonzero = object                   */
    const int *fixed;            /* n_frames, nonzero = pose held constant           */
    int n_match_sets;            /* sets of sparse matches, one per node pair        */
    const int *match_i, *match_j;/* n_match_sets node ids, i != j                    */
    const int *match_n;          /* n_match_sets match counts                        */
    const int *match_off;        /* n_match_sets offsets into uv_i/uv_j (in matches) */
    const float *uv_i, *uv_j;    /* 2 floats (u,v) per match, pixel coordinates      */
    double lambda_f, lambda_g;   /* Eq. (1) weights; 0 disables a term               */
    double huber_f, huber_g;     /* Huber thresholds (metres)                        */
    double gate_dist;            /* dense association distance gate (metres)         */
    double gate_angle;           /* dense association normal-angle gate (radians)    */
    /* learned weighting (project addition; NULL mlp = Huber weights only):
     * dense weight = Huber weight * sigmoid(MLP(features)), energy sigma * rho */
    const double *mlp;           /* ORC_MLP_PARAMS parameters                        */
    const unsigned char *keep;   /* n_frames*H*W kept source pixels, or NULL          */
    double prune_frac;           /* optimize: fraction of source pixels pruned at its
                                    start when keep is NULL (0 = none)                */
    int mlp_iters;               /* iteration-feature normalisation (GN iterations)  */
    int iteration;               /* iteration feature of orc_linearize*              */
} orc_problem;

/* Per-call statistics. */
typedef struct {
    double energy_f, energy_g;   /* lambda-weighted Huber energies at the given poses */
    long long n_valid_g;         /* gated-in dense residuals (ordered pairs)          */
    long long n_valid_f;         /* valid matches, each counted once                   */
} orc_lin_stats;

#define ORC_MAX_ITERS 64
typedef struct {
    int iters_done;
    double energy_f[ORC_MAX_ITERS], energy_g[ORC_MAX_ITERS];
    long long n_valid_g[ORC_MAX_ITERS], n_valid_f[ORC_MAX_ITERS];
} orc_opt_stats;

/* Threads used by the ordered-pair loop (1 = sequential).  Results do not
 * depend on it: per-pair sums are added in a fixed order. */
void orc_set_threads(int n);
int  orc_get_threads(void);

/* Per-frame preprocessing: vertex map (3*H*W), normal map (3*H*W) and a
 * per-pixel code: bit0 = depth/mask valid, bit1 = normal valid. */
int orc_preprocess_frame(const orc_problem *pb, int f, double *vertex, double *normal,
                         unsigned char *valid);

/* Normal equations at the given poses (n_frames*16 doubles): H (6N x 6N,
 * row-major), g (6N), and per entry the sum of |contributions| to H and g
 * (scales of the rounding a different summation order may introduce).
 * Any of H_abs/g_abs/st may be NULL. */
int orc_linearize(const orc_problem *pb, const double *poses, double *H, double *g,
                  double *H_abs, double *g_abs, orc_lin_stats *st);

/* As orc_linearize, with the dense association decisions given instead of
 * taken by S2: targets holds, for every ordered pair in lexicographic order
 * ((0,1), (0,2), ..., (1,0), (1,2), ...), H*W target pixel indices of the
 * source pixels of frame i (negative = no residual).  Used to compare the
 * arithmetic of another implementation on its own decision set. */
int orc_linearize_given(const orc_problem *pb, const double *poses, const int *targets, double *H,
                        double *g, double *H_abs, double *g_abs, orc_lin_stats *st);

/* Fixed number of IRLS Gauss-Newton iterations; poses updated in place.  On a
 * singular system the poses of the last completed iteration are kept and
 * ORC_ERR_SINGULAR is returned. */
int orc_optimize(const orc_problem *pb, double *poses, int iters, orc_opt_stats *st);

/* Dense association of the ordered pair (i, j) at the given poses.  For every
 * pixel of frame i: target[x] = target pixel index, or a negative code
 *   -1 not a valid source, -2 behind camera, -3 outside image,
 *   -4 invalid target, -5 distance gate, -6 normal gate;
 * r[x] = point-to-plane residual (0 where rejected); proj[2x..2x+1] = the
 * continuous projection (u', v') where computed (NaN otherwise); gate[2x..] =
 * (|s-p|, cosine of the normal angle) where computed. */
int orc_associate(const orc_problem *pb, const double *poses, int i, int j,
                  int *target, double *r, double *proj, double *gate);

/* Residuals and Jacobian rows of frozen associations, without gating: for the
 * n source pixels src[k] of frame i associated with target pixels tgt[k] of
 * frame j, r[k] and J[12k..12k+11] = [dr/d(xi_i), dr/d(xi_j)] at the poses. */
int orc_dense_frozen(const orc_problem *pb, const double *poses, int i, int j, int n,
                     const int *src, const int *tgt, double *r, double *J);

/* Feature residual e (3) and Jacobian (3x12, [de/dxi_i | de/dxi_j], row-major)
 * of match k of set s at the given poses.  Returns 1 if the match is valid. */
int orc_feature_eval(const orc_problem *pb, const double *poses, int s, int k,
                     double *e, double *J);

/* SE(3) exponential of xi = [v; w] as a 4x4 row-major matrix. */
void orc_se3_exp(const double *xi, double *T);

/* Huber loss and IRLS weight at s >= 0 with threshold delta. */
double orc_huber_rho(double s, double delta);
double orc_huber_weight(double s, double delta);

/* Dense Cholesky solve of the SPD system A x = b (n x n row-major).
 * Returns ORC_ERR_SINGULAR when a pivot is <= 1e-12 * max diagonal. */
int orc_cholesky_solve(int n, const double *A, const double *b, double *x);

/* ---- learned correspondence weighting (a project addition to the IRLS
 * weights W of Sec. IV-D): a 6-32-32-1 multilayer perceptron,
 * y = sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3).  Parameters are 1313
 * doubles in the order W1 (32x6, row-major), b1 (32), W2 (32x32), b2 (32),
 * W3 (1x32), b3 (1). */
#define ORC_MLP_PARAMS 1313
#define ORC_MLP_IN 6
#define ORC_MLP_HID 32

/* Features of one gated-in pixel-pair: r / huber_g, normal angle / 30 deg,
 * source depth / 0.8 m, pixel radius / half-diagonal, |s - p| / gate_dist,
 * iteration / (mlp_iters - 1).  For every pixel x of frame i associated into
 * frame j at the given poses, features[6x..6x+5] (zeros where rejected) and
 * the decision code as orc_associate. */
int orc_pair_features(const orc_problem *pb, const double *poses, int i, int j, int iteration,
                      int *target, double *features);

/* orc_pair_features for n_pairs ordered pairs (pi[q], pj[q]) at once:
 * target holds n_pairs*H*W codes and features n_pairs*H*W*6 values (either
 * may be NULL), pair q's block after pair q-1's. */
int orc_pairs_features(const orc_problem *pb, const double *poses, int n_pairs, const int *pi,
                       const int *pj, int iteration, int *target, double *features);

/* Pruning scores at the given poses (iteration feature 0): for every source
 * pixel the largest network output over its gated-in pairs (0 if none), -1
 * where the pixel is not a valid source; n_frames*H*W doubles. */
int orc_prune_scores(const orc_problem *pb, const double *poses, double *score);

/* Pruning decision from scores: per frame, the floor(frac * V) valid source
 * pixels lowest in (score, row-major position) order are dropped; keep gets 1
 * for the others (n_frames*H*W bytes). */
int orc_prune_select(const orc_problem *pb, const double *score, double frac, unsigned char *keep);

/* Output of the network for each of n inputs (n x 6, row-major). */
void orc_mlp_forward(const double *params, int n, const double *x, double *y);

/* The network as the dense term evaluates it, "in FP16" (the learned
 * weighting's 6-32-32-1 network): the parameters are binary16 values and the
 * input of every layer (the features and both hidden layers' activations) is
 * rounded to binary16 (nearest, ties to even) before it enters that layer's
 * products; products and sums are exact here (FP64).  Used by the dense term,
 * orc_pair_features' consumers and orc_prune_scores whenever pb->mlp is set. */
void orc_mlp_forward_half(const double *params, int n, const double *x, double *y);

/* The same evaluation, returning for each of the n inputs the exact
 * pre-activations of the two hidden layers (s1, s2: n x 32, each from its
 * layer's rounded inputs; either may be NULL) and the logit z (n, may be
 * NULL).  Lets a caller find activations that lie next to a binary16 rounding
 * boundary. */
void orc_mlp_trace_half(const double *params, int n, const double *x, double *s1, double *s2,
                        double *z);

/* x rounded to the nearest IEEE binary16 value (ties to even; overflow to
 * +-inf; subnormals kept), returned as a double. */
double orc_round_half(double x);

/* Mean binary cross-entropy of the outputs against labels in {0, 1} and its
 * gradient with respect to the parameters (1313 doubles; grad may be NULL). */
double orc_mlp_bce(const double *params, int n, const double *x, const double *labels,
                   double *grad);

/* ---- coarse registration by RANSAC (Sec. IV-B) ----
 * Least-squares rigid transform of k >= 3 point pairs (Arun et al.): T (4x4
 * row-major) minimising sum |R b_m + t - a_m|^2, from the SVD of the
 * cross-covariance with the reflection correction.  ORC_ERR_SINGULAR when the
 * points are collinear. */
int orc_arun(int k, const double *a, const double *b, double *T);

/* Score of one hypothesis: sample holds three match indices; the hypothesis
 * is orc_arun of those three pairs.  Returns -1 for an unusable sample (an
 * index out of range, repeated or of an invalid match, or a triangle of area
 * below 1e-8 m^2 in either frame), else the number of valid matches m with
 * |R b_m + t - a_m| < delta and (R nb_m) . na_m > cos(alpha).  T (16) and
 * inlier (n) receive the hypothesis and its inlier flags (either may be
 * NULL). */
int orc_ransac_score(int n, const double *a, const double *na, const double *b, const double *nb,
                     const unsigned char *valid, const int *sample, double delta, double alpha,
                     double *T, unsigned char *inlier);

/* RANSAC over the matches of n_pairs ordered node pairs (pi[q], pj[q]): pair
 * q's matches are uv_i/uv_j entries match_off[q] .. match_off[q+1]-1 (pixel
 * coordinates in frames pi[q] and pj[q]); a match's points a (frame pi) and b
 * (frame pj) and their normals are taken at the nearest pixels and the match
 * is valid when both are valid sources (depth, mask, normal).  samples holds
 * n_pairs * n_hyp triples of match indices (local to the pair).  best[q] =
 * the hypothesis with the most inliers (lowest index among equals; -1 when no
 * sample is usable), T[16q..] = its transform (frame pj camera -> frame pi
 * camera; identity when best is -1), inlier[match_off[q] + m] = its inlier
 * flags; score (may be NULL) = every hypothesis' score. */
int orc_ransac_pairs(const orc_problem *pb, int n_pairs, const int *pi, const int *pj, const int *match_off,
                     const float *uv_i, const float *uv_j, int n_hyp, const int *samples, double delta,
                     double alpha, int *best, int *score, double *T, unsigned char *inlier);

/* ---- keypoint matching (Sec. IV-B) ----
 * Descriptors A (na x dim) of frame a and B (nb x dim) of frame b, FP32
 * row-major.  match[x] = the nearest descriptor of B to A[x] (squared
 * Euclidean distance, exact in FP64; lowest index among equals) when A[x] is
 * also the nearest of A to it (lowest index among equals) and, for ratio < 1,
 * when d1 < ratio^2 d2 (d1, d2: the squared distances to the nearest and the
 * second nearest); else -1.  d1_out, d2_out (na, may be NULL) receive d1 and
 * d2 (infinity where undefined). */
int orc_match_descriptors(int na, const float *A, int nb, const float *B, int dim, double ratio, int *match,
                          double *d1_out, double *d2_out);

/* ---- keyframe memory pool (Sec. IV-C, IV-E) ----
 * Poses are 4x4 row-major (object -> camera); only their rotations matter.
 * Geodesic distance of two rotations: arccos((tr(R_a^T R_b) - 1) / 2), the
 * cosine clamped to [-1, 1]. */
double orc_rot_geodesic(const double *Ta, const double *Tb);

/* Greedy keyframe selection (Sec. IV-C): starting from {pool[0]} (the initial
 * frame), repeatedly add the keyframe with the smallest sum of geodesic
 * distances to the current frame and to every keyframe selected so far
 * (lowest index among equal sums), until min(K, n_pool) are selected.
 * selected[0..*n_selected) receives the pool indices in selection order;
 * cost (may be NULL, n_pool) the final sums (those of selected keyframes as
 * they were when chosen). */
int orc_select_keyframes(int n_pool, const double *T_pool, const double *T_cur, int K, int *selected,
                         int *n_selected, double *cost);

/* Novel view (Sec. IV-E): 1 when the current frame's rotation is farther
 * than thresh (radians) from every keyframe of the pool, else 0. */
int orc_novel_view(int n_pool, const double *T_pool, const double *T_cur, double thresh);

#ifdef __cplusplus
}
#endif
#endif
