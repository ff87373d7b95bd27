/*
 * posegraph.h - C ABI of the MI355X pose-graph optimiser.
 *
 * The library implements the online pose-graph optimisation of BundleTrack
 * (Wen & Bekris, IROS 2021), Sec. IV-D: the nodes are the object poses of a
 * window of RGB-D keyframes (current frame plus selected keyframes); the
 * total energy of Eq. (1) sums, over every ordered node pair, a sparse
 * feature term (Eq. 2) and a dense point-to-plane term with projective data
 * association (Eq. 3), both under the Huber M-estimator; it is minimised by
 * iteratively re-weighted Gauss-Newton with the first keyframe's pose held
 * constant and updates applied in the tangent space.
 *
 * Conventions shared by every entry point:
 *  - Pose T maps object to camera coordinates (the object pose in the camera
 *    frame, Sec. III): x_cam = R x_obj + t; passed as 16 doubles, 4x4
 *    row-major, bottom row (0,0,0,1), R orthonormal within 1e-6.
 *  - Twist xi = [v; w] (3 translation then 3 rotation parameters, Sec. IV-D);
 *    an update is T <- Exp(delta) T.
 *  - Depth is metres (float); 0, negative or non-finite means no depth.
 *    Mask is uint8, nonzero = object pixel (the binary mask of Sec. IV-A).
 *  - Pixel (u, v) has its centre at integer coordinates; u is the column.
 *  - Every input pointer may be host or device memory (detected); inputs are
 *    always copied, so the caller keeps ownership and may free them on return.
 *    Output pointers are host memory unless stated.
 *  - All GPU work is ordered on the stream given at creation (a hipStream_t,
 *    NULL = the null stream).  Calls that return results synchronise it.
 *  - Every call returns a pg_status; no exception or abort crosses the ABI.
 *    pose_graph_last_error() gives a message for the last failed call.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef POSEGRAPH_H
#define POSEGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pg_graph pg_graph; /* opaque, library-owned */

typedef enum {
    PG_OK = 0,
    PG_ERR_INVALID_ARG = -1,   /* bad pointer, size, id, intrinsics or pose       */
    PG_ERR_NO_DEVICE = -2,     /* no usable GPU                                    */
    PG_ERR_OUT_OF_MEMORY = -3, /* device allocation failed                         */
    PG_ERR_CAPACITY = -4,      /* more frames than max_frames, or too many to solve */
    PG_ERR_SINGULAR = -5,      /* normal equations not positive definite           */
    PG_ERR_NONFINITE = -6,     /* non-finite update                                 */
    PG_ERR_HIP = -7            /* a HIP runtime call failed                         */
} pg_status;

/* Solvers of the Gauss-Newton step (all exact up to rounding):
 * AUTO picks LDL (block LDL^T with 4x4 pivot blocks on one wavefront, the
 * system held in registers, rank-4 updates on the FP64 matrix cores) when the
 * system has at most 60 unknowns (10 free nodes), else Gauss-Jordan (3x3 pivot
 * blocks, rank-3 updates on the matrix cores, one workgroup per graph) up to
 * 126 unknowns (21 free nodes), else Cholesky; PCG is the Jacobi-preconditioned
 * conjugate gradient the paper names (Sec. IV-D) on the assembled normal
 * equations.  PCG_MATRIX_FREE is that PCG without forming the normal
 * equations: J^T W J p is applied from per-pair Gram blocks of the
 * association pass and the feature blocks (up to 14 keyframes); it stops at
 * |r| <= pcg_rel_tol |b|.  Choosing LDL for a graph that may hold more than 10
 * free nodes, or PCG_MATRIX_FREE with max_frames above 14, fails
 * (PG_ERR_CAPACITY at create). */
enum { PG_SOLVER_AUTO = 0, PG_SOLVER_PCG = 1, PG_SOLVER_CHOLESKY = 2, PG_SOLVER_GAUSS_JORDAN = 3,
       PG_SOLVER_LDL = 4, PG_SOLVER_PCG_MATRIX_FREE = 5 };
enum { PG_WEIGHT_HUBER = 0, PG_WEIGHT_LEARNED = 1 };
enum { PG_PREC_FP32 = 0, PG_PREC_BF16X3 = 1 };

#define PG_MAX_FRAMES_LIMIT 32 /* upper bound of pg_config.max_frames */
#define PG_MAX_ITERS 32        /* upper bound of pg_config.gn_iters   */

/* One pinhole camera per graph (pi and pi_D^-1 of Eq. 3). */
typedef struct {
    int width, height;          /* pixels, 3..8192 each                 */
    double fx, fy, cx, cy;      /* focal lengths > 0 and principal point */
} pg_camera;

/* Method parameters and execution options.  Fill with pg_config_default(). */
typedef struct {
    int max_frames;             /* node capacity, 2..PG_MAX_FRAMES_LIMIT (default 16)       */
    int gn_iters;               /* Gauss-Newton iterations per optimize (default 7)          */
    double lambda_f, lambda_g;  /* Eq. (1) weights of the feature / dense terms (1, 1)       */
    double huber_f_m;           /* Huber threshold of the feature term, metres (0.005)      */
    double huber_g_m;           /* Huber threshold of the dense term, metres (0.005)        */
    double gate_dist_m;         /* dense association distance gate, metres (0.01)           */
    double gate_normal_rad;     /* dense association normal-angle gate, radians (30 deg)    */
    int solver;                 /* PG_SOLVER_AUTO (default), _PCG, _CHOLESKY, _GAUSS_JORDAN, _LDL, _PCG_MATRIX_FREE */
    int pcg_max_iters;          /* PCG iteration cap (default 500)                           */
    double pcg_rel_tol;         /* PCG stop: |r| <= tol |b| (default 1e-12)                  */
    int weighting;              /* PG_WEIGHT_HUBER (default) or PG_WEIGHT_LEARNED            */
    int precision;              /* PG_PREC_FP32 (default) or PG_PREC_BF16X3                  */
    int use_graph;              /* 1 = replay the iteration loop as a captured hipGraph (0)  */
    int timing;                 /* 1 = HIP events around each kernel, launched directly (0)  */
    int tile_pixels;            /* source pixels per association work item (rounded up to a multiple
                                   of 256, at most 2048); 0 = the tile table's, else 1024 */
    double prune_frac;          /* learned weighting: fraction of source pixels dropped (0.25) */
    int persistent;             /* 1 = persistent association blocks drain the work table through
                                   atomic counters (0: one block per work item); same results */
} pg_config;

/* Per-optimize statistics. */
typedef struct {
    int iters_done;                          /* completed Gauss-Newton iterations          */
    double energy_f[PG_MAX_ITERS];           /* lambda_f * sum of Eq. (2) over ordered pairs */
    double energy_g[PG_MAX_ITERS];           /* lambda_g * sum of Eq. (3) over ordered pairs */
    long long n_valid_g[PG_MAX_ITERS];       /* gated-in dense residuals                   */
    long long n_valid_f[PG_MAX_ITERS];       /* valid feature matches (each counted once)  */
    int status_bits;                         /* bit0 singular, bit1 non-finite             */
    long long src_pixels;                    /* sum over ordered pairs of valid source pixels */
    int n_assoc_launches;                    /* association kernel launches (timing = 1)   */
    float ms_assoc, ms_feature, ms_reduce, ms_solve, ms_total; /* kernel time (timing = 1) */
    long long n_target_reads[PG_MAX_ITERS];  /* dense association: target pixels read   */
    int pcg_iters[PG_MAX_ITERS];             /* PCG iterations per Gauss-Newton iteration (PCG solvers; else 0) */
} pg_stats;

/* Defaults listed in pg_config. */
void pg_config_default(pg_config *cfg);

/* Create a graph on the current HIP device.  hip_stream: a hipStream_t or NULL.
 * Errors: PG_ERR_INVALID_ARG (cfg/camera out of range), PG_ERR_NO_DEVICE,
 * PG_ERR_OUT_OF_MEMORY, PG_ERR_CAPACITY (max_frames too large to solve in one
 * workgroup on this device).  *out is NULL on error. */
pg_status pose_graph_create(const pg_config *cfg, const pg_camera *cam, void *hip_stream,
                            pg_graph **out);

/* Add a node: depth (H*W floats, metres) and mask (H*W bytes) of one frame,
 * row-major; its initial pose; fixed != 0 holds the pose constant (the first
 * keyframe I_0 is the fixed reference of Sec. IV-D).  Preprocesses the frame
 * on the GPU (validity, back-projection, normals, packed layout and the list
 * of valid source pixels).  *out_id receives the node id 0, 1, ...
 * Errors: PG_ERR_INVALID_ARG, PG_ERR_CAPACITY (max_frames reached). */
pg_status pose_graph_add_frame(pg_graph *g, const float *depth_m, const uint8_t *mask,
                               const double T_obj_to_cam[16], int fixed, int *out_id);

/* Feature correspondences C_ij between nodes i and j (Eq. 2): n pixel pairs,
 * uv_i and uv_j hold 2n floats (u, v).  Stored once per unordered pair (i and j
 * are swapped when i > j); a later call for the same pair replaces the set,
 * which is otherwise reused by every optimize (Sec. IV-D).  n = 0 removes it.
 * Each match's 3-D points are the back-projections of the nearest pixels; a
 * match whose pixel is outside the image or has no depth/mask is skipped.
 * Errors: PG_ERR_INVALID_ARG. */
pg_status pose_graph_add_matches(pg_graph *g, int id_i, int id_j, const float *uv_i,
                                 const float *uv_j, int n);

/* Set / read a node pose (host memory, 16 doubles). */
pg_status pose_graph_set_pose(pg_graph *g, int id, const double T[16]);
pg_status pose_graph_get_pose(const pg_graph *g, int id, double T_out[16]);

/* Set all n = pose_graph_num_frames(g) poses at once (16 n doubles, host). */
pg_status pose_graph_set_poses(pg_graph *g, int n, const double *T);

/* Run cfg.gn_iters iterations: per iteration, dense association and
 * residuals of every ordered pair, feature residuals, the fused reduction into
 * the 6N x 6N normal equations (J^T W J) delta = -J^T W r, the solve over the
 * free nodes and the update T <- Exp(delta) T.  Poses stay in the graph (the
 * memory-pool write-back of Sec. IV-D) and are readable with get_pose.
 * Synchronous.  On PG_ERR_SINGULAR / PG_ERR_NONFINITE the poses are those of
 * the last completed iteration and stats->iters_done says which.
 * stats may be NULL. */
pg_status pose_graph_optimize(pg_graph *g, pg_stats *stats);

/* Optimise n_graphs independent graphs in one batched schedule (one launch per
 * phase for all graphs; uneven node counts and resolutions allowed).  All
 * graphs must share one device and one stream.  stats: NULL or n_graphs
 * entries.  Returns the first non-OK per-graph status. */
pg_status pose_graph_optimize_batch(pg_graph *const *graphs, int n_graphs, pg_stats *stats);

/* Normal equations at the current poses without updating them: H (6N*6N,
 * row-major, all nodes including fixed ones) and g = J^T W r (6N), as doubles
 * in host memory.  stats (nullable) receives energies and counts in entry 0.
 * The same kernels as optimize. */
pg_status pose_graph_linearize(pg_graph *g, double *H, double *grad, pg_stats *stats);

/* Test inspection of the dense association of ordered pair (i, j) at the
 * current poses: for every pixel x of frame i (H*W entries, host memory),
 * target[x] = associated pixel of frame j, or a negative code (-1 not a valid
 * source, -2 behind the camera, -3 outside the image, -4 invalid target,
 * -5 distance gate, -6 normal gate); r[x] = point-to-plane residual (0 where
 * rejected); uv[2x..2x+1] = continuous projection (NaN where not computed).
 * Any output may be NULL. */
pg_status pose_graph_associate(pg_graph *g, int i, int j, int32_t *target, float *r,
                               float *uv);

/* Test inspection of a preprocessed frame: packed map (4*H*W floats, host:
 * nx, ny, nz, z per pixel, z = 0 where the pixel is not a valid source/target)
 * and the number of valid source pixels.  Either output may be NULL. */
pg_status pose_graph_frame_info(pg_graph *g, int id, float *map, int *n_valid);

/* Learned correspondence weighting (an extension of the Huber weighting of
 * Sec. IV-D; the paper itself weights every residual by the M-estimator
 * only): parameters of a 6-32-32-1 perceptron (ReLU hidden layers, sigmoid
 * output) as fp16, layout W1[32x6] b1[32] W2[32x32] b2[32] W3[1x32] b3[1]
 * (row-major, 1313 values).  The network is evaluated "in FP16": these
 * binary16 parameters, and every layer's input (the features and both hidden
 * layers' activations) rounded to binary16 (nearest, ties to even), with each
 * layer's products summed in FP32 (the hidden layers on the fp16 matrix
 * cores) and the logistic in FP32.  With
 * cfg.weighting == PG_WEIGHT_LEARNED every gated-in dense residual's IRLS
 * weight and energy are multiplied by the network output sigma(f) of its
 * features f (pose_graph_pair_features), and, when cfg.prune_frac > 0, each
 * optimize first drops per frame the floor(prune_frac * V) of its V source
 * pixels with the lowest score (pose_graph_prune), ties by position.
 * Errors: PG_ERR_INVALID_ARG when n_bytes != 2626. */
pg_status pose_graph_set_mlp(pg_graph *g, const void *fp16_params, size_t n_bytes);

/* Features of the dense association of ordered pair (i, j) at the current
 * poses, as the learned weighting sees them at Gauss-Newton iteration
 * 'iteration' (0-based): for each pixel x of frame i with a gated-in target,
 * features[6x..6x+5] = { r / huber_g_m, normal angle / 30 deg, source depth
 * / 0.8 m, |(u, v) - (cx, cy)| / half image diagonal, |A q - p| /
 * gate_dist_m, iteration / max(gn_iters - 1, 1) }, zeros elsewhere;
 * sigma[x] = network output (0 where rejected; needs pose_graph_set_mlp);
 * target[x] as in pose_graph_associate.  Outputs are host or device memory
 * (detected), H*W entries (6*H*W floats for features); any may be NULL.
 * Errors: PG_ERR_INVALID_ARG. */
pg_status pose_graph_pair_features(pg_graph *g, int i, int j, int iteration, float *features,
                                   float *sigma, int32_t *target);

/* Tuned association tiles (project addition: the tile autotuner's table).
 * entries: n_entries (0..256) records of 5 ints {width, height, min_frames,
 * max_frames, tile_pixels} in host memory, copied; tile_pixels a multiple of
 * 256 in 256..2048.  A graph whose cfg.tile_pixels is 0 takes the tile of the
 * first record matching its resolution and node count (else 1024) when its
 * schedule is next built; each graph of a batch keeps its own tile.  Replaces
 * the previous table (n_entries 0 clears it); process-wide, thread-safe.
 * Errors: PG_ERR_INVALID_ARG (message in pose_graph_last_error(NULL)). */
pg_status pg_set_tile_table(const int *entries, int n_entries);

/* Timing of the dense association kernel alone at the current poses (for
 * roofline figures): after one untimed launch, reps (1..10000) launches of
 * iteration 0 back to back on the graph's stream between two HIP events;
 * *ms_per_launch = elapsed / reps.  With learned weighting the pruning pass
 * runs first, untimed.  Leaves the poses unchanged.  Errors:
 * PG_ERR_INVALID_ARG. */
pg_status pose_graph_time_assoc(pg_graph *g, int reps, double *ms_per_launch);

/* Pruning pass of the learned weighting at the current poses (the pass an
 * optimize runs on its starting poses): score[f*H*W + x] = the largest network
 * output over the target frames source pixel x of frame f is gated in with
 * (iteration 0), 0 if none, -1 if x is not a valid source pixel;
 * keep[f*H*W + x] = 1 for the source pixels kept.  Host memory, N*H*W entries
 * each; either may be NULL.  Errors: PG_ERR_INVALID_ARG unless
 * cfg.weighting == PG_WEIGHT_LEARNED and cfg.prune_frac > 0. */
pg_status pose_graph_prune(pg_graph *g, float *score, uint8_t *keep);

/* Number of nodes. */
int pose_graph_num_frames(const pg_graph *g);

/* Message of the last failed call on g (or of the last failed create when g
 * is NULL).  Valid until the next call on the same handle. */
const char *pose_graph_last_error(const pg_graph *g);

/* Release the graph and its device memory.  NULL-safe. */
void pose_graph_destroy(pg_graph *g);

/* ------------------------------------------------------------------------
 * Trainer of the learned weighting network: FP32 master parameters, Adam
 * moments and an fp16 copy in device memory.  Loss: mean binary cross-entropy
 * of sigmoid(network(x)) against labels in {0, 1}; gradients are summed in a
 * fixed order (FP32 within 64-sample blocks, FP64 across blocks), so results
 * are reproducible.  Batches are device memory: x is n*6 floats (row-major
 * feature vectors as pose_graph_pair_features writes them), labels n floats.
 * All work is ordered on the stream given at creation. */
typedef struct pg_mlp pg_mlp; /* opaque, library-owned */

/* max_samples: largest batch (1..2^26).  Parameters start at zero.
 * Errors: PG_ERR_INVALID_ARG, PG_ERR_NO_DEVICE, PG_ERR_OUT_OF_MEMORY. */
pg_status pg_mlp_create(int max_samples, void *hip_stream, pg_mlp **out);
void pg_mlp_destroy(pg_mlp *t);

/* Set the 1313 FP32 parameters (host or device memory, layout as in
 * pose_graph_set_mlp) and reset the Adam state. */
pg_status pg_mlp_set_params(pg_mlp *t, const float *params);

/* Read the FP32 parameters and/or their fp16 copy (host memory; either may
 * be NULL). */
pg_status pg_mlp_get_params(pg_mlp *t, float *params_out, void *fp16_out);

/* Mean loss and its gradient (1313 doubles; may be NULL) at the current
 * parameters over a batch, in host memory.  Errors: PG_ERR_INVALID_ARG (n out
 * of range, host batch). */
pg_status pg_mlp_loss_grad(pg_mlp *t, const float *x, const float *labels, int n, double *loss_out,
                           double *grad_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr on the batch's mean-loss gradient; loss_out (host, may be
 * NULL) receives the batch loss before the step. */
pg_status pg_mlp_adam_step(pg_mlp *t, const float *x, const float *labels, int n, double lr,
                           double *loss_out);

/* y[s] = sigmoid(network(x[s])) at the FP32 parameters; x and y device memory. */
pg_status pg_mlp_forward(pg_mlp *t, const float *x, int n, float *y);

/* Message of the last failed call on t (of the last failed create when NULL). */
const char *pg_mlp_last_error(const pg_mlp *t);

#ifdef __cplusplus
}
#endif
#endif /* POSEGRAPH_H */
