/*
 * FP64 CPU oracle for BundleTrack's online pose-graph optimisation
 * (Wen & Bekris, IROS 2021, Sec. IV-D).  TEST INFRASTRUCTURE ONLY: the plain,
 * slow, obviously-correct reference the GPU library is checked against.  It
 * shares no code with the GPU library.
 *
 * What it computes, in the paper's order:
 *   S0  per frame: validity (mask, finite positive depth), back-projected
 *       vertex map p = pi_D^-1 (Sec. IV-D, after Eq. 3), normal map n_i(.)
 *       (central differences; the paper does not say how normals are made);
 *   S1  per ordered pair (i, j), j != i (the double sum of Eq. 1):
 *       A = T_i T_j^-1 and B = T_j T_i^-1 (the two transforms of Eq. 3);
 *   S2  dense projective association of every valid pixel of frame i into
 *       frame j, gated by point distance and normal angle (text after Eq. 3);
 *   S3  point-to-plane residual of Eq. 3, its Jacobian, Huber IRLS weight
 *       (rho of Eq. 2/3 is the Huber loss; W in the Gauss-Newton step);
 *   S4  feature residual of Eq. 2 and its Jacobian for every match;
 *   S5  normal equations J^T W J and J^T W r summed in a fixed order;
 *   S6  the first keyframe's pose held constant (the gauge of Sec. IV-D),
 *       Gauss-Newton step solved by Cholesky (the converged PCG solution);
 *   S7  update in the tangent space, T <- Exp(delta) T.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ utils */

static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

/* nearest pixel, ties to the upper pixel: floor(x + 1/2) computed exactly */
static double round_half_up(double x)
{
    double f = floor(x);
    return (x - f >= 0.5) ? f + 1.0 : f;
}

static void rigid_inverse(const double *T, double *Ti)
{
    /* [R t; 0 1]^-1 = [R^T  -R^T t; 0 1] */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Ti[4 * r + c] = T[4 * c + r];
    for (int r = 0; r < 3; ++r)
        Ti[4 * r + 3] = -(Ti[4 * r + 0] * T[3] + Ti[4 * r + 1] * T[7] + Ti[4 * r + 2] * T[11]);
    Ti[12] = Ti[13] = Ti[14] = 0.0;
    Ti[15] = 1.0;
}

static void mat4_mul(const double *A, const double *B, double *C)
{
    double tmp[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k)
                s += A[4 * r + k] * B[4 * k + c];
            tmp[4 * r + c] = s;
        }
    memcpy(C, tmp, sizeof(tmp));
}

static void apply_T(const double *T, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r)
        y[r] = T[4 * r] * x[0] + T[4 * r + 1] * x[1] + T[4 * r + 2] * x[2] + T[4 * r + 3];
}

static void apply_R(const double *T, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r)
        y[r] = T[4 * r] * x[0] + T[4 * r + 1] * x[1] + T[4 * r + 2] * x[2];
}

static void apply_Rt(const double *T, const double *x, double *y)
{
    for (int r = 0; r < 3; ++r)
        y[r] = T[r] * x[0] + T[4 + r] * x[1] + T[8 + r] * x[2];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------ Huber */

double orc_huber_rho(double s, double delta)
{
    return (s <= delta) ? 0.5 * s * s : delta * (s - 0.5 * delta);
}

double orc_huber_weight(double s, double delta)
{
    /* rho'(s)/s: the IRLS weight of the diagonal matrix W */
    return (s <= delta) ? 1.0 : delta / s;
}

/* ------------------------------------------------------------------ SE(3) */

void orc_se3_exp(const double *xi, double *T)
{
    const double *v = xi, *w = xi + 3;
    double th2 = dot3(w, w), th = sqrt(th2);
    double A, B, C; /* sin(t)/t, (1-cos t)/t^2, (t - sin t)/t^3 */
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k)
                s += K[3 * r + k] * K[3 * k + c];
            K2[3 * r + c] = s;
        }
    double R[9], V[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double I = (r == c) ? 1.0 : 0.0;
            R[3 * r + c] = I + A * K[3 * r + c] + B * K2[3 * r + c];
            V[3 * r + c] = I + B * K[3 * r + c] + C * K2[3 * r + c];
        }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            T[4 * r + c] = R[3 * r + c];
        T[4 * r + 3] = V[3 * r] * v[0] + V[3 * r + 1] * v[1] + V[3 * r + 2] * v[2];
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

/* --------------------------------------------------------- S0: per frame */

int orc_preprocess_frame(const orc_problem *pb, int f, double *vertex, double *normal,
                         unsigned char *valid)
{
    if (!pb || f < 0 || f >= pb->n_frames)
        return ORC_ERR_ARG;
    const int W = pb->width, H = pb->height;
    const float *D = pb->depth + (size_t)f * W * H;
    const unsigned char *M = pb->mask + (size_t)f * W * H;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t x = (size_t)v * W + u;
            double z = (double)D[x];
            int ok = (M[x] != 0) && isfinite(z) && z > 0.0;
            valid[x] = ok ? 1 : 0;
            /* pi_D^-1: back-projection through the pinhole at the pixel centre */
            vertex[3 * x + 0] = ok ? z * ((double)u - pb->cx) / pb->fx : 0.0;
            vertex[3 * x + 1] = ok ? z * ((double)v - pb->cy) / pb->fy : 0.0;
            vertex[3 * x + 2] = ok ? z : 0.0;
        }
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t x = (size_t)v * W + u;
            normal[3 * x] = normal[3 * x + 1] = normal[3 * x + 2] = 0.0;
            if (!valid[x] || u == 0 || v == 0 || u == W - 1 || v == H - 1)
                continue;
            size_t xl = x - 1, xr = x + 1, xu = x - W, xd = x + W;
            if (!valid[xl] || !valid[xr] || !valid[xu] || !valid[xd])
                continue;
            double du[3], dv[3], n[3];
            for (int k = 0; k < 3; ++k) {
                du[k] = vertex[3 * xr + k] - vertex[3 * xl + k];
                dv[k] = vertex[3 * xd + k] - vertex[3 * xu + k];
            }
            cross3(du, dv, n);
            double len = sqrt(dot3(n, n));
            if (!(len > 0.0))
                continue;
            for (int k = 0; k < 3; ++k)
                n[k] /= len;
            if (dot3(n, vertex + 3 * x) > 0.0) /* face the camera */
                for (int k = 0; k < 3; ++k)
                    n[k] = -n[k];
            for (int k = 0; k < 3; ++k)
                normal[3 * x + k] = n[k];
            valid[x] |= 2;
        }
    return ORC_OK;
}

/* ------------------------------------------------------- frame cache */

typedef struct {
    double *vertex, *normal;
    unsigned char *valid;
} frame_maps;

static frame_maps *build_frames(const orc_problem *pb)
{
    size_t hw = (size_t)pb->width * pb->height;
    frame_maps *fm = (frame_maps *)calloc((size_t)pb->n_frames, sizeof(frame_maps));
    if (!fm)
        return NULL;
    for (int f = 0; f < pb->n_frames; ++f) {
        fm[f].vertex = (double *)malloc(3 * hw * sizeof(double));
        fm[f].normal = (double *)malloc(3 * hw * sizeof(double));
        fm[f].valid = (unsigned char *)malloc(hw);
        orc_preprocess_frame(pb, f, fm[f].vertex, fm[f].normal, fm[f].valid);
    }
    return fm;
}

static void free_frames(const orc_problem *pb, frame_maps *fm)
{
    if (!fm)
        return;
    for (int f = 0; f < pb->n_frames; ++f) {
        free(fm[f].vertex);
        free(fm[f].normal);
        free(fm[f].valid);
    }
    free(fm);
}

/* --------------------------------------------- per-pair partial normal eqs */

static double mlp_sigmoid_of(const double *P, const double *f);
static void mlp_features(const orc_problem *pb, const frame_maps *fm, int i, size_t x, double r,
                         double dist, double cosang, int iteration, double *f);

typedef struct {
    int i, j;                 /* node ids of the 12 columns: [i (6) | j (6)] */
    double H[144], g[12];
    double Habs[144], gabs[12];
    double energy;
    long long count;
} pair_part;

static void add_row(pair_part *pp, const double *row, double w, double res)
{
    /* H += w row row^T, g += w res row */
    for (int a = 0; a < 12; ++a) {
        for (int b = 0; b < 12; ++b) {
            double c = w * (row[a] * row[b]); /* symmetric in a, b */
            pp->H[12 * a + b] += c;
            pp->Habs[12 * a + b] += fabs(c);
        }
        double c = w * res * row[a];
        pp->g[a] += c;
        pp->gabs[a] += fabs(c);
    }
}

/* One dense association step (S2) of source pixel x of frame i into frame j.
 * Returns the target pixel index (>= 0) or a negative rejection code, and the
 * quantities the decision used. */
static int associate_pixel(const orc_problem *pb, const frame_maps *fm, int i, int j,
                           const double *A, const double *B, size_t x, double *s_out,
                           double *r_out, double *proj, double *gate)
{
    const int W = pb->width, H = pb->height;
    if ((fm[i].valid[x] & 3) != 3)
        return -1;
    const double *p = fm[i].vertex + 3 * x;
    const double *n = fm[i].normal + 3 * x;
    double pp[3];
    apply_T(B, p, pp);              /* T_j T_i^-1 p */
    if (!(pp[2] > 0.0))
        return -2;
    double uf = pb->fx * pp[0] / pp[2] + pb->cx; /* pi(.) */
    double vf = pb->fy * pp[1] / pp[2] + pb->cy;
    if (proj) {
        proj[0] = uf;
        proj[1] = vf;
    }
    double ui = round_half_up(uf), vi = round_half_up(vf);
    if (!(ui >= 0.0 && ui < (double)W && vi >= 0.0 && vi < (double)H))
        return -3;
    size_t y = (size_t)vi * W + (size_t)ui;
    if ((fm[j].valid[y] & 3) != 3)
        return -4;
    const double *q = fm[j].vertex + 3 * y;     /* pi_D^-1 of frame j */
    const double *nq = fm[j].normal + 3 * y;
    double s[3], d[3], Rnq[3];
    apply_T(A, q, s);                /* T_i T_j^-1 pi_D^-1(.) */
    for (int k = 0; k < 3; ++k)
        d[k] = s[k] - p[k];
    double dist = sqrt(dot3(d, d));
    apply_R(A, nq, Rnq);
    double cosang = dot3(n, Rnq);
    if (gate) {
        gate[0] = dist;
        gate[1] = cosang;
    }
    if (!(dist < pb->gate_dist))
        return -5;
    if (!(cosang > cos(pb->gate_angle)))
        return -6;
    if (s_out)
        memcpy(s_out, s, sizeof(s));
    if (r_out)
        *r_out = dot3(n, d);         /* n_i(x) . (s - p) */
    return (int)y;
}

/* Jacobian row of r = n.(A q - p) w.r.t. left perturbations of T_i and T_j. */
static void dense_jacobian(const double *A, const double *n, const double *s, const double *q,
                           double *row)
{
    double sxn[3], Rtn[3], qxRtn[3];
    cross3(s, n, sxn);
    apply_Rt(A, n, Rtn);
    cross3(q, Rtn, qxRtn);
    for (int k = 0; k < 3; ++k) {
        row[k] = n[k];            /* d r / d v_i */
        row[3 + k] = sxn[k];      /* d r / d w_i */
        row[6 + k] = -Rtn[k];     /* d r / d v_j */
        row[9 + k] = -qxRtn[k];   /* d r / d w_j */
    }
}

static void pair_transforms(const double *poses, int i, int j, double *A, double *B)
{
    double Ti_inv[16], Tj_inv[16];
    rigid_inverse(poses + 16 * i, Ti_inv);
    rigid_inverse(poses + 16 * j, Tj_inv);
    mat4_mul(poses + 16 * i, Tj_inv, A);   /* frame-j camera -> frame-i camera */
    mat4_mul(poses + 16 * j, Ti_inv, B);   /* frame-i camera -> frame-j camera */
}

/* Dense term of one ordered pair.  With 'given' (H*W target indices, negative
 * = no residual) the association decisions are taken from outside instead of
 * S2, and the residuals, Jacobians and weights are evaluated for them. */
static void dense_pair(const orc_problem *pb, const frame_maps *fm, const double *poses,
                       const int *given, const unsigned char *keep, int iteration, pair_part *pp)
{
    const int i = pp->i, j = pp->j;
    double A[16], B[16];
    pair_transforms(poses, i, j, A, B);
    const size_t hw = (size_t)pb->width * pb->height;
    for (size_t x = 0; x < hw; ++x) {   /* row-major source order */
        if (keep && !keep[(size_t)i * hw + x])
            continue;
        double s[3], r, gate[2];
        int y;
        if (given) {
            y = given[x];
            if (y < 0)
                continue;
            const double *p = fm[i].vertex + 3 * x;
            double d[3], Rnq[3];
            apply_T(A, fm[j].vertex + 3 * (size_t)y, s);
            for (int k = 0; k < 3; ++k)
                d[k] = s[k] - p[k];
            r = dot3(fm[i].normal + 3 * x, d);
            apply_R(A, fm[j].normal + 3 * (size_t)y, Rnq);
            gate[0] = sqrt(dot3(d, d));
            gate[1] = dot3(fm[i].normal + 3 * x, Rnq);
        } else {
            y = associate_pixel(pb, fm, i, j, A, B, x, s, &r, NULL, gate);
            if (y < 0)
                continue;
        }
        const double *n = fm[i].normal + 3 * x;
        const double *q = fm[j].vertex + 3 * (size_t)y;
        double row[12];
        dense_jacobian(A, n, s, q, row);
        double ar = fabs(r);
        double sig = 1.0;   /* learned factor of the IRLS weight */
        if (pb->mlp) {
            double f[6];
            mlp_features(pb, fm, i, x, r, gate[0], gate[1], iteration, f);
            sig = mlp_sigmoid_of(pb->mlp, f);
        }
        double w = pb->lambda_g * sig * orc_huber_weight(ar, pb->huber_g);
        add_row(pp, row, w, r);
        pp->energy += pb->lambda_g * sig * orc_huber_rho(ar, pb->huber_g);
        pp->count += 1;
    }
}

/* Match endpoint: back-projection of the nearest pixel, if it has depth. */
static int match_point(const orc_problem *pb, const frame_maps *fm, int f, const float *uv,
                       double *p)
{
    double u = round_half_up((double)uv[0]), v = round_half_up((double)uv[1]);
    if (!(u >= 0.0 && u < pb->width && v >= 0.0 && v < pb->height))
        return 0;
    size_t x = (size_t)v * pb->width + (size_t)u;
    if (!(fm[f].valid[x] & 1))
        return 0;
    memcpy(p, fm[f].vertex + 3 * x, 3 * sizeof(double));
    return 1;
}

/* e = T_i^-1 p_m - T_j^-1 p_n (Eq. 2) and its 3x12 Jacobian. */
static void feature_eval(const double *Ti, const double *Tj, const double *pm, const double *pn,
                         double *e, double *J)
{
    double Ti_inv[16], Tj_inv[16], a[3], b[3];
    rigid_inverse(Ti, Ti_inv);
    rigid_inverse(Tj, Tj_inv);
    apply_T(Ti_inv, pm, a);
    apply_T(Tj_inv, pn, b);
    for (int k = 0; k < 3; ++k)
        e[k] = a[k] - b[k];
    /* de/dv_i = -R_i^T, de/dw_i = R_i^T [p_m]x ; de/dv_j = R_j^T, de/dw_j = -R_j^T [p_n]x */
    double Pm[9] = {0, -pm[2], pm[1], pm[2], 0, -pm[0], -pm[1], pm[0], 0};
    double Pn[9] = {0, -pn[2], pn[1], pn[2], 0, -pn[0], -pn[1], pn[0], 0};
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            double Rti = Ti[4 * c + r], Rtj = Tj[4 * c + r]; /* (R^T)_{rc} */
            double RtPm = 0.0, RtPn = 0.0;
            for (int k = 0; k < 3; ++k) {
                RtPm += Ti[4 * k + r] * Pm[3 * k + c];
                RtPn += Tj[4 * k + r] * Pn[3 * k + c];
            }
            J[12 * r + c] = -Rti;
            J[12 * r + 3 + c] = RtPm;
            J[12 * r + 6 + c] = Rtj;
            J[12 * r + 9 + c] = -RtPn;
        }
    }
}

static void feature_set(const orc_problem *pb, const frame_maps *fm, const double *poses, int s,
                        pair_part *pp)
{
    const int i = pb->match_i[s], j = pb->match_j[s];
    for (int k = 0; k < pb->match_n[s]; ++k) {
        size_t m = (size_t)pb->match_off[s] + k;
        double pm[3], pn[3];
        if (!match_point(pb, fm, i, pb->uv_i + 2 * m, pm) || !match_point(pb, fm, j, pb->uv_j + 2 * m, pn))
            continue;
        double e[3], J[36];
        feature_eval(poses + 16 * i, poses + 16 * j, pm, pn, e, J);
        double ne = sqrt(dot3(e, e));
        /* E_f(i,j) and E_f(j,i) are the same sum: each match counts twice in Eq. 1 */
        double w = 2.0 * pb->lambda_f * orc_huber_weight(ne, pb->huber_f);
        for (int c = 0; c < 3; ++c)
            add_row(pp, J + 12 * c, w, e[c]);
        pp->energy += 2.0 * pb->lambda_f * orc_huber_rho(ne, pb->huber_f);
        pp->count += 1;
    }
}

static int check_problem(const orc_problem *pb)
{
    if (!pb || pb->n_frames < 1 || pb->width < 3 || pb->height < 3 || !pb->depth || !pb->mask)
        return ORC_ERR_ARG;
    if (!(pb->fx > 0 && pb->fy > 0))
        return ORC_ERR_ARG;
    for (int s = 0; s < pb->n_match_sets; ++s) {
        int i = pb->match_i[s], j = pb->match_j[s];
        if (i < 0 || j < 0 || i >= pb->n_frames || j >= pb->n_frames || i == j)
            return ORC_ERR_ARG;
    }
    return ORC_OK;
}

static int linearize_with(const orc_problem *pb, const frame_maps *fm, const double *poses,
                          const int *given, const unsigned char *keep, int iteration, double *H, double *g,
                          double *H_abs, double *g_abs, orc_lin_stats *st)
{
    const int N = pb->n_frames, n6 = 6 * N;
    const int n_dense = (pb->lambda_g != 0.0) ? N * (N - 1) : 0;
    const int n_feat = (pb->lambda_f != 0.0) ? pb->n_match_sets : 0;
    pair_part *parts = (pair_part *)calloc((size_t)(n_dense + n_feat) + 1, sizeof(pair_part));
    if (!parts)
        return ORC_ERR_ARG;
    /* S1: ordered pairs in lexicographic order, then the match sets in order */
    int k = 0;
    for (int i = 0; i < N && n_dense; ++i)
        for (int j = 0; j < N; ++j)
            if (j != i) {
                parts[k].i = i;
                parts[k].j = j;
                ++k;
            }
    for (int s = 0; s < n_feat; ++s) {
        parts[n_dense + s].i = pb->match_i[s];
        parts[n_dense + s].j = pb->match_j[s];
    }
    const int total = n_dense + n_feat;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
    for (int t = 0; t < total; ++t) {
        if (t < n_dense)                                   /* S2 + S3 */
            dense_pair(pb, fm, poses, given ? given + (size_t)t * pb->width * pb->height : NULL, keep,
                       iteration, &parts[t]);
        else
            feature_set(pb, fm, poses, t - n_dense, &parts[t]); /* S4 */
    }
    /* S5: fixed-order sum of the per-pair partial systems */
    memset(H, 0, sizeof(double) * n6 * n6);
    memset(g, 0, sizeof(double) * n6);
    if (H_abs)
        memset(H_abs, 0, sizeof(double) * n6 * n6);
    if (g_abs)
        memset(g_abs, 0, sizeof(double) * n6);
    double Ef = 0.0, Eg = 0.0;
    long long cf = 0, cg = 0;
    for (int t = 0; t < total; ++t) {
        const pair_part *pp = &parts[t];
        int node[2] = {pp->i, pp->j};
        for (int a = 0; a < 12; ++a) {
            int ra = 6 * node[a / 6] + a % 6;
            for (int b = 0; b < 12; ++b) {
                int cb = 6 * node[b / 6] + b % 6;
                H[(size_t)ra * n6 + cb] += pp->H[12 * a + b];
                if (H_abs)
                    H_abs[(size_t)ra * n6 + cb] += pp->Habs[12 * a + b];
            }
            g[ra] += pp->g[a];
            if (g_abs)
                g_abs[ra] += pp->gabs[a];
        }
        if (t < n_dense) {
            Eg += pp->energy;
            cg += pp->count;
        } else {
            Ef += pp->energy;
            cf += pp->count;
        }
    }
    if (st) {
        st->energy_f = Ef;
        st->energy_g = Eg;
        st->n_valid_f = cf;
        st->n_valid_g = cg;
    }
    free(parts);
    return ORC_OK;
}

int orc_linearize(const orc_problem *pb, const double *poses, double *H, double *g,
                  double *H_abs, double *g_abs, orc_lin_stats *st)
{
    int rc = check_problem(pb);
    if (rc != ORC_OK || !poses || !H || !g)
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    if (!fm)
        return ORC_ERR_ARG;
    rc = linearize_with(pb, fm, poses, NULL, pb->keep, pb->iteration, H, g, H_abs, g_abs, st);
    free_frames(pb, fm);
    return rc;
}

int orc_linearize_given(const orc_problem *pb, const double *poses, const int *targets, double *H,
                        double *g, double *H_abs, double *g_abs, orc_lin_stats *st)
{
    int rc = check_problem(pb);
    if (rc != ORC_OK || !poses || !targets || !H || !g)
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    if (!fm)
        return ORC_ERR_ARG;
    rc = linearize_with(pb, fm, poses, targets, pb->keep, pb->iteration, H, g, H_abs, g_abs, st);
    free_frames(pb, fm);
    return rc;
}

/* ------------------------------------------------------------ S6: solve */

int orc_cholesky_solve(int n, const double *A, const double *b, double *x)
{
    if (n <= 0)
        return ORC_OK;
    double *L = (double *)calloc((size_t)n * n, sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    if (!L || !y) {
        free(L);
        free(y);
        return ORC_ERR_ARG;
    }
    double maxdiag = 0.0;
    for (int i = 0; i < n; ++i)
        if (A[(size_t)i * n + i] > maxdiag)
            maxdiag = A[(size_t)i * n + i];
    int rc = ORC_OK;
    if (!(maxdiag > 0.0))
        rc = ORC_ERR_SINGULAR;
    for (int j = 0; j < n && rc == ORC_OK; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k)
            s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 1e-12 * maxdiag)) {
            rc = ORC_ERR_SINGULAR;
            break;
        }
        double d = sqrt(s);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k)
                t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / d;
        }
    }
    if (rc == ORC_OK) {
        for (int i = 0; i < n; ++i) { /* L y = b */
            double t = b[i];
            for (int k = 0; k < i; ++k)
                t -= L[(size_t)i * n + k] * y[k];
            y[i] = t / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) { /* L^T x = y */
            double t = y[i];
            for (int k = i + 1; k < n; ++k)
                t -= L[(size_t)k * n + i] * x[k];
            x[i] = t / L[(size_t)i * n + i];
        }
    }
    free(L);
    free(y);
    return rc;
}

/* ------------------------------------------------------ S1..S7 iterated */

int orc_optimize(const orc_problem *pb, double *poses, int iters, orc_opt_stats *st)
{
    int rc = check_problem(pb);
    if (rc != ORC_OK || !poses || iters < 0 || iters > ORC_MAX_ITERS)
        return ORC_ERR_ARG;
    const int N = pb->n_frames, n6 = 6 * N;
    int *free_ids = (int *)malloc(sizeof(int) * N);
    int nfree = 0;
    for (int f = 0; f < N; ++f)
        if (!(pb->fixed && pb->fixed[f]))
            free_ids[nfree++] = f;
    const int nf = 6 * nfree;
    double *H = (double *)malloc(sizeof(double) * n6 * n6);
    double *g = (double *)malloc(sizeof(double) * n6);
    double *Hff = (double *)malloc(sizeof(double) * (nf ? nf * nf : 1));
    double *bf = (double *)malloc(sizeof(double) * (nf ? nf : 1));
    double *dx = (double *)malloc(sizeof(double) * (nf ? nf : 1));
    frame_maps *fm = build_frames(pb);
    if (st)
        memset(st, 0, sizeof(*st));
    /* learned weighting: prune the source pixels once, at the initial poses */
    const unsigned char *keep = pb->keep;
    unsigned char *own_keep = NULL;
    if (pb->mlp && !keep && pb->prune_frac > 0.0) {
        const size_t tot = (size_t)N * pb->width * pb->height;
        double *score = (double *)malloc(sizeof(double) * tot);
        own_keep = (unsigned char *)malloc(tot);
        orc_prune_scores(pb, poses, score);
        orc_prune_select(pb, score, pb->prune_frac, own_keep);
        free(score);
        keep = own_keep;
    }
    rc = ORC_OK;
    for (int it = 0; it < iters; ++it) {
        orc_lin_stats ls;
        linearize_with(pb, fm, poses, NULL, keep, it, H, g, NULL, NULL, &ls);
        if (st) {
            st->energy_f[it] = ls.energy_f;
            st->energy_g[it] = ls.energy_g;
            st->n_valid_f[it] = ls.n_valid_f;
            st->n_valid_g[it] = ls.n_valid_g;
        }
        if (nfree) {
            /* S6: drop the fixed nodes, solve H_ff delta = -g_f */
            for (int a = 0; a < nf; ++a) {
                int ra = 6 * free_ids[a / 6] + a % 6;
                for (int b = 0; b < nf; ++b) {
                    int cb = 6 * free_ids[b / 6] + b % 6;
                    Hff[(size_t)a * nf + b] = H[(size_t)ra * n6 + cb];
                }
                bf[a] = -g[ra];
            }
            if (orc_cholesky_solve(nf, Hff, bf, dx) != ORC_OK) {
                rc = ORC_ERR_SINGULAR;
                break;
            }
            /* S7: T_i <- Exp(delta_i) T_i */
            for (int a = 0; a < nfree; ++a) {
                double E[16];
                orc_se3_exp(dx + 6 * a, E);
                mat4_mul(E, poses + 16 * free_ids[a], poses + 16 * free_ids[a]);
            }
        }
        if (st)
            st->iters_done = it + 1;
    }
    free_frames(pb, fm);
    free(own_keep);
    free(free_ids);
    free(H);
    free(g);
    free(Hff);
    free(bf);
    free(dx);
    return rc;
}

/* ------------------------------------------------ inspection entry points */

int orc_associate(const orc_problem *pb, const double *poses, int i, int j, int *target,
                  double *r, double *proj, double *gate)
{
    if (check_problem(pb) != ORC_OK || !poses || i < 0 || j < 0 || i >= pb->n_frames ||
        j >= pb->n_frames || i == j)
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    double A[16], B[16];
    pair_transforms(poses, i, j, A, B);
    const size_t hw = (size_t)pb->width * pb->height;
    for (size_t x = 0; x < hw; ++x) {
        double rr = 0.0, pr[2] = {NAN, NAN}, gt[2] = {NAN, NAN};
        int y = associate_pixel(pb, fm, i, j, A, B, x, NULL, &rr, pr, gt);
        if (target)
            target[x] = y;
        if (r)
            r[x] = (y >= 0) ? rr : 0.0;
        if (proj) {
            proj[2 * x] = pr[0];
            proj[2 * x + 1] = pr[1];
        }
        if (gate) {
            gate[2 * x] = gt[0];
            gate[2 * x + 1] = gt[1];
        }
    }
    free_frames(pb, fm);
    return ORC_OK;
}

int orc_dense_frozen(const orc_problem *pb, const double *poses, int i, int j, int n,
                     const int *src, const int *tgt, double *r, double *J)
{
    if (check_problem(pb) != ORC_OK || !poses || i == j)
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    double A[16], B[16];
    pair_transforms(poses, i, j, A, B);
    for (int k = 0; k < n; ++k) {
        const double *p = fm[i].vertex + 3 * (size_t)src[k];
        const double *nn = fm[i].normal + 3 * (size_t)src[k];
        const double *q = fm[j].vertex + 3 * (size_t)tgt[k];
        double s[3], d[3];
        apply_T(A, q, s);
        for (int c = 0; c < 3; ++c)
            d[c] = s[c] - p[c];
        r[k] = dot3(nn, d);
        if (J)
            dense_jacobian(A, nn, s, q, J + 12 * (size_t)k);
    }
    free_frames(pb, fm);
    return ORC_OK;
}

int orc_feature_eval(const orc_problem *pb, const double *poses, int s, int k, double *e,
                     double *J)
{
    if (check_problem(pb) != ORC_OK || s < 0 || s >= pb->n_match_sets || k < 0 ||
        k >= pb->match_n[s])
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    const int i = pb->match_i[s], j = pb->match_j[s];
    size_t m = (size_t)pb->match_off[s] + k;
    double pm[3], pn[3], Jl[36];
    int ok = match_point(pb, fm, i, pb->uv_i + 2 * m, pm) && match_point(pb, fm, j, pb->uv_j + 2 * m, pn);
    if (ok) {
        feature_eval(poses + 16 * i, poses + 16 * j, pm, pn, e, Jl);
        if (J)
            memcpy(J, Jl, sizeof(Jl));
    }
    free_frames(pb, fm);
    return ok;
}

/* ---------------------------------------------- learned weighting network */

/* parameter offsets: W1 (32x6), b1, W2 (32x32), b2, W3 (1x32), b3 */
#define MLP_W1 0
#define MLP_B1 (MLP_W1 + ORC_MLP_HID * ORC_MLP_IN)
#define MLP_W2 (MLP_B1 + ORC_MLP_HID)
#define MLP_B2 (MLP_W2 + ORC_MLP_HID * ORC_MLP_HID)
#define MLP_W3 (MLP_B2 + ORC_MLP_HID)
#define MLP_B3 (MLP_W3 + ORC_MLP_HID)

static double sigmoid(double t) { return 1.0 / (1.0 + exp(-t)); }

/* one input: hidden pre-activations a1, a2, activations h1, h2, logit */
static double mlp_eval(const double *P, const double *x, double *a1, double *h1, double *a2, double *h2)
{
    for (int o = 0; o < ORC_MLP_HID; ++o) {
        double s = P[MLP_B1 + o];
        for (int k = 0; k < ORC_MLP_IN; ++k)
            s += P[MLP_W1 + ORC_MLP_IN * o + k] * x[k];
        a1[o] = s;
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < ORC_MLP_HID; ++o) {
        double s = P[MLP_B2 + o];
        for (int k = 0; k < ORC_MLP_HID; ++k)
            s += P[MLP_W2 + ORC_MLP_HID * o + k] * h1[k];
        a2[o] = s;
        h2[o] = s > 0.0 ? s : 0.0;
    }
    double z = P[MLP_B3];
    for (int k = 0; k < ORC_MLP_HID; ++k)
        z += P[MLP_W3 + k] * h2[k];
    return z;
}

void orc_mlp_forward(const double *params, int n, const double *x, double *y)
{
    double a1[ORC_MLP_HID], h1[ORC_MLP_HID], a2[ORC_MLP_HID], h2[ORC_MLP_HID];
    for (int i = 0; i < n; ++i)
        y[i] = sigmoid(mlp_eval(params, x + ORC_MLP_IN * (size_t)i, a1, h1, a2, h2));
}

double orc_mlp_bce(const double *params, int n, const double *x, const double *labels, double *grad)
{
    double a1[ORC_MLP_HID], h1[ORC_MLP_HID], a2[ORC_MLP_HID], h2[ORC_MLP_HID];
    double d1[ORC_MLP_HID], d2[ORC_MLP_HID];
    if (grad)
        memset(grad, 0, sizeof(double) * ORC_MLP_PARAMS);
    double loss = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *xi = x + ORC_MLP_IN * (size_t)i;
        const double z = mlp_eval(params, xi, a1, h1, a2, h2);
        const double t = labels[i];
        /* -[t log s(z) + (1 - t) log(1 - s(z))] = log(1 + e^z) - t z, evaluated stably */
        loss += (z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z))) - t * z;
        if (!grad)
            continue;
        const double dz = (sigmoid(z) - t) / n;   /* d loss / d z (mean over the batch) */
        grad[MLP_B3] += dz;
        for (int k = 0; k < ORC_MLP_HID; ++k) {
            grad[MLP_W3 + k] += dz * h2[k];
            d2[k] = (a2[k] > 0.0) ? dz * params[MLP_W3 + k] : 0.0;
        }
        for (int o = 0; o < ORC_MLP_HID; ++o) {
            grad[MLP_B2 + o] += d2[o];
            for (int k = 0; k < ORC_MLP_HID; ++k)
                grad[MLP_W2 + ORC_MLP_HID * o + k] += d2[o] * h1[k];
        }
        for (int k = 0; k < ORC_MLP_HID; ++k) {
            double s = 0.0;
            for (int o = 0; o < ORC_MLP_HID; ++o)
                s += params[MLP_W2 + ORC_MLP_HID * o + k] * d2[o];
            d1[k] = (a1[k] > 0.0) ? s : 0.0;
        }
        for (int o = 0; o < ORC_MLP_HID; ++o) {
            grad[MLP_B1 + o] += d1[o];
            for (int k = 0; k < ORC_MLP_IN; ++k)
                grad[MLP_W1 + ORC_MLP_IN * o + k] += d1[o] * xi[k];
        }
    }
    return loss / n;
}

double orc_round_half(double x)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e;
    frexp(fabs(x), &e);   /* |x| = m 2^e, m in [0.5, 1) */
    /* binary16: 11 significant bits for normal values (|x| >= 2^-14, i.e.
     * e >= -13); below, the fixed quantum 2^-24 of the subnormals */
    const double q = (e >= -13) ? ldexp(1.0, e - 11) : ldexp(1.0, -24);
    const double r = nearbyint(x / q) * q;   /* default rounding: nearest, ties to even */
    if (fabs(r) > 65504.0)
        return x > 0.0 ? INFINITY : -INFINITY;
    return r;
}

/* The network "in FP16" (6-32-32-1): the parameters are binary16 values, and
 * the input of every layer (the features, then each hidden layer's
 * activations) is rounded to binary16 (nearest, ties to even) before it is
 * multiplied; products and sums are exact here (FP64).  s1, s2 (may be NULL)
 * receive the exact pre-activations of the two hidden layers, from the
 * rounded inputs of their layer. */
static double mlp_eval_half_trace(const double *P, const double *f, double *s1, double *s2)
{
    double x[ORC_MLP_IN], h1[ORC_MLP_HID];
    for (int k = 0; k < ORC_MLP_IN; ++k)
        x[k] = orc_round_half(f[k]);
    for (int o = 0; o < ORC_MLP_HID; ++o) {
        double s = P[MLP_B1 + o];
        for (int k = 0; k < ORC_MLP_IN; ++k)
            s += P[MLP_W1 + ORC_MLP_IN * o + k] * x[k];
        if (s1)
            s1[o] = s;
        h1[o] = orc_round_half(s > 0.0 ? s : 0.0);
    }
    double z = P[MLP_B3];
    for (int o = 0; o < ORC_MLP_HID; ++o) {
        double s = P[MLP_B2 + o];
        for (int k = 0; k < ORC_MLP_HID; ++k)
            s += P[MLP_W2 + ORC_MLP_HID * o + k] * h1[k];
        if (s2)
            s2[o] = s;
        z += P[MLP_W3 + o] * orc_round_half(s > 0.0 ? s : 0.0);
    }
    return z;
}

static double mlp_eval_half(const double *P, const double *f)
{
    return mlp_eval_half_trace(P, f, NULL, NULL);
}

void orc_mlp_trace_half(const double *params, int n, const double *x, double *s1, double *s2,
                        double *z)
{
    for (int i = 0; i < n; ++i) {
        const double zi = mlp_eval_half_trace(params, x + ORC_MLP_IN * (size_t)i,
                                              s1 ? s1 + ORC_MLP_HID * (size_t)i : NULL,
                                              s2 ? s2 + ORC_MLP_HID * (size_t)i : NULL);
        if (z)
            z[i] = zi;
    }
}

void orc_mlp_forward_half(const double *params, int n, const double *x, double *y)
{
    for (int i = 0; i < n; ++i)
        y[i] = sigmoid(mlp_eval_half(params, x + ORC_MLP_IN * (size_t)i));
}

static double mlp_sigmoid_of(const double *P, const double *f)
{
    return sigmoid(mlp_eval_half(P, f));
}

static void mlp_features(const orc_problem *pb, const frame_maps *fm, int i, size_t x, double r,
                         double dist, double cosang, int iteration, double *f)
{
    const int W = pb->width, H = pb->height;
    const double u = (double)(x % (size_t)W), v = (double)(x / (size_t)W);
    const double c = cosang > 1.0 ? 1.0 : (cosang < -1.0 ? -1.0 : cosang);
    const int den = pb->mlp_iters > 1 ? pb->mlp_iters - 1 : 1;
    f[0] = r / pb->huber_g;
    f[1] = acos(c) / (3.14159265358979323846 / 6.0);   /* angle in units of 30 degrees */
    f[2] = fm[i].vertex[3 * x + 2] / 0.8;
    f[3] = sqrt((u - pb->cx) * (u - pb->cx) + (v - pb->cy) * (v - pb->cy)) /
           sqrt(0.25 * W * W + 0.25 * H * H);
    f[4] = dist / pb->gate_dist;
    f[5] = (double)iteration / den;
}

int orc_pairs_features(const orc_problem *pb, const double *poses, int n_pairs, const int *pi,
                       const int *pj, int iteration, int *target, double *features)
{
    if (check_problem(pb) != ORC_OK || !poses || n_pairs < 0 || (n_pairs > 0 && (!pi || !pj)))
        return ORC_ERR_ARG;
    for (int q = 0; q < n_pairs; ++q)
        if (pi[q] == pj[q] || pi[q] < 0 || pj[q] < 0 || pi[q] >= pb->n_frames || pj[q] >= pb->n_frames)
            return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    const size_t hw = (size_t)pb->width * pb->height;
    for (int q = 0; q < n_pairs; ++q) {
        const int i = pi[q], j = pj[q];
        double A[16], B[16];
        pair_transforms(poses, i, j, A, B);
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long long xx = 0; xx < (long long)hw; ++xx) {
            const size_t x = (size_t)xx;
            double r = 0.0, gate[2] = {0.0, 0.0};
            int y = associate_pixel(pb, fm, i, j, A, B, x, NULL, &r, NULL, gate);
            if (target)
                target[(size_t)q * hw + x] = y;
            if (!features)
                continue;
            double *f = features + 6 * ((size_t)q * hw + x);
            if (y >= 0)
                mlp_features(pb, fm, i, x, r, gate[0], gate[1], iteration, f);
            else
                f[0] = f[1] = f[2] = f[3] = f[4] = f[5] = 0.0;
        }
    }
    free_frames(pb, fm);
    return ORC_OK;
}

int orc_pair_features(const orc_problem *pb, const double *poses, int i, int j, int iteration,
                      int *target, double *features)
{
    return orc_pairs_features(pb, poses, 1, &i, &j, iteration, target, features);
}

int orc_prune_scores(const orc_problem *pb, const double *poses, double *score)
{
    if (check_problem(pb) != ORC_OK || !pb->mlp || !poses || !score)
        return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    const int N = pb->n_frames;
    const size_t hw = (size_t)pb->width * pb->height;
    for (int i = 0; i < N; ++i) {
        double *sc = score + (size_t)i * hw;
        for (size_t x = 0; x < hw; ++x)
            sc[x] = ((fm[i].valid[x] & 3) == 3) ? 0.0 : -1.0;
#pragma omp parallel for schedule(static) num_threads(g_threads)
        for (long long xx = 0; xx < (long long)hw; ++xx) {
            const size_t x = (size_t)xx;
            if (sc[x] < 0.0)
                continue;
            for (int j = 0; j < N; ++j) {
                if (j == i)
                    continue;
                double A[16], B[16], r = 0.0, gate[2];
                pair_transforms(poses, i, j, A, B);
                if (associate_pixel(pb, fm, i, j, A, B, x, NULL, &r, NULL, gate) < 0)
                    continue;
                double f[6];
                mlp_features(pb, fm, i, x, r, gate[0], gate[1], 0, f);
                const double s = mlp_sigmoid_of(pb->mlp, f);
                if (s > sc[x])
                    sc[x] = s;
            }
        }
    }
    free_frames(pb, fm);
    return ORC_OK;
}

typedef struct {
    double score;
    size_t pos;
} scored_px;

static int cmp_scored(const void *a, const void *b)
{
    const scored_px *p = (const scored_px *)a, *q = (const scored_px *)b;
    if (p->score != q->score)
        return p->score < q->score ? -1 : 1;
    return p->pos < q->pos ? -1 : (p->pos > q->pos ? 1 : 0);
}

int orc_prune_select(const orc_problem *pb, const double *score, double frac, unsigned char *keep)
{
    if (!pb || !score || !keep || frac < 0.0 || frac > 1.0)
        return ORC_ERR_ARG;
    const size_t hw = (size_t)pb->width * pb->height;
    scored_px *buf = (scored_px *)malloc(sizeof(scored_px) * hw);
    for (int f = 0; f < pb->n_frames; ++f) {
        const double *sc = score + (size_t)f * hw;
        unsigned char *kp = keep + (size_t)f * hw;
        size_t V = 0;
        for (size_t x = 0; x < hw; ++x) {
            kp[x] = 0;
            if (sc[x] >= 0.0) {
                buf[V].score = sc[x];
                buf[V].pos = x;
                ++V;
                kp[x] = 1;
            }
        }
        const size_t drop = (size_t)floor(frac * (double)V);
        qsort(buf, V, sizeof(scored_px), cmp_scored);
        for (size_t k = 0; k < drop; ++k)
            kp[buf[k].pos] = 0;
    }
    free(buf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Coarse registration by RANSAC (Sec. IV-B): each hypothesis is the
 * least-squares rigid transform of a sample of three matched keypoint pairs
 * (Arun et al.), scored by the matches it brings within delta of their
 * partner with normals within alpha; the best sampled hypothesis is the
 * registration.  The random samples are an input. */

/* Singular value decomposition of a 3x3 matrix by one-sided Jacobi
 * rotations: M V = W with orthogonal columns; columns of W (and of V) sorted
 * by decreasing norm. */
static void svd3_jacobi(const double *M, double *W, double *V)
{
    memcpy(W, M, 9 * sizeof(double));
    for (int r = 0; r < 9; ++r)
        V[r] = (r % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double a = 0.0, b = 0.0, c = 0.0;   /* |w_p|^2, |w_q|^2, w_p . w_q */
                for (int r = 0; r < 3; ++r) {
                    a += W[3 * r + p] * W[3 * r + p];
                    b += W[3 * r + q] * W[3 * r + q];
                    c += W[3 * r + p] * W[3 * r + q];
                }
                if (c == 0.0 || fabs(c) <= 1e-300)
                    continue;
                const double rel = fabs(c) / sqrt(a * b);
                if (rel > off)
                    off = rel;
                /* rotation that makes columns p and q orthogonal */
                const double zeta = (b - a) / (2.0 * c);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int r = 0; r < 3; ++r) {
                    const double wp = W[3 * r + p], wq = W[3 * r + q];
                    W[3 * r + p] = cs * wp - sn * wq;
                    W[3 * r + q] = sn * wp + cs * wq;
                    const double vp = V[3 * r + p], vq = V[3 * r + q];
                    V[3 * r + p] = cs * vp - sn * vq;
                    V[3 * r + q] = sn * vp + cs * vq;
                }
            }
        if (off <= 1e-15)
            break;
    }
    /* sort the columns by decreasing norm */
    for (int p = 0; p < 2; ++p)
        for (int q = p + 1; q < 3; ++q) {
            double a = 0.0, b = 0.0;
            for (int r = 0; r < 3; ++r) {
                a += W[3 * r + p] * W[3 * r + p];
                b += W[3 * r + q] * W[3 * r + q];
            }
            if (b > a)
                for (int r = 0; r < 3; ++r) {
                    double t = W[3 * r + p];
                    W[3 * r + p] = W[3 * r + q];
                    W[3 * r + q] = t;
                    t = V[3 * r + p];
                    V[3 * r + p] = V[3 * r + q];
                    V[3 * r + q] = t;
                }
        }
}

static double det3(const double *M)
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

int orc_arun(int k, const double *a, const double *b, double *T)
{
    if (k < 3 || !a || !b || !T)
        return ORC_ERR_ARG;
    double ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
    for (int m = 0; m < k; ++m)
        for (int r = 0; r < 3; ++r) {
            ca[r] += a[3 * m + r] / k;
            cb[r] += b[3 * m + r] / k;
        }
    /* cross-covariance S = sum (a - ca)(b - cb)^T; S = U D V^T; the rotation
     * mapping b onto a is R = U diag(1, 1, det(U) det(V)) V^T */
    double S[9] = {0};
    for (int m = 0; m < k; ++m)
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                S[3 * r + c] += (a[3 * m + r] - ca[r]) * (b[3 * m + c] - cb[c]);
    double W[9], V[9], U[9];
    svd3_jacobi(S, W, V);
    double n0 = 0.0, n1 = 0.0;
    for (int r = 0; r < 3; ++r) {
        n0 += W[3 * r] * W[3 * r];
        n1 += W[3 * r + 1] * W[3 * r + 1];
    }
    n0 = sqrt(n0);
    n1 = sqrt(n1);
    if (!(n1 > 1e-12 * n0))
        return ORC_ERR_SINGULAR;   /* collinear points: the rotation about their line is free */
    for (int r = 0; r < 3; ++r) {
        U[3 * r] = W[3 * r] / n0;
        U[3 * r + 1] = W[3 * r + 1] / n1;
    }
    /* third left vector completes a right-handed basis (the third singular
     * value may be zero); the sign choice cancels in R */
    const double u0[3] = {U[0], U[3], U[6]}, u1[3] = {U[1], U[4], U[7]};
    double u2[3];
    cross3(u0, u1, u2);
    for (int r = 0; r < 3; ++r)
        U[3 * r + 2] = u2[r];
    const double d = det3(V) < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            T[4 * r + c] = U[3 * r] * V[3 * c] + U[3 * r + 1] * V[3 * c + 1] + d * U[3 * r + 2] * V[3 * c + 2];
    for (int r = 0; r < 3; ++r)
        T[4 * r + 3] = ca[r] - (T[4 * r] * cb[0] + T[4 * r + 1] * cb[1] + T[4 * r + 2] * cb[2]);
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
    return ORC_OK;
}

/* 3-D point and normal of a keypoint at the nearest pixel; valid when the
 * pixel is inside the image, has depth and mask and a valid normal */
static int keypoint_geometry(const orc_problem *pb, const frame_maps *fm, int f, const float *uv, double *p,
                             double *n)
{
    double u = round_half_up((double)uv[0]), v = round_half_up((double)uv[1]);
    if (!(u >= 0.0 && u < pb->width && v >= 0.0 && v < pb->height))
        return 0;
    size_t x = (size_t)v * pb->width + (size_t)u;
    if ((fm[f].valid[x] & 3) != 3)
        return 0;
    memcpy(p, fm[f].vertex + 3 * x, 3 * sizeof(double));
    memcpy(n, fm[f].normal + 3 * x, 3 * sizeof(double));
    return 1;
}

int orc_ransac_score(int n, const double *a, const double *na, const double *b, const double *nb,
                     const unsigned char *valid, const int *sample, double delta, double alpha,
                     double *T, unsigned char *inlier)
{
    double sa[9], sb[9];
    for (int q = 0; q < 3; ++q) {
        const int m = sample[q];
        if (m < 0 || m >= n || !valid[m])
            return -1;
        for (int r = 0; r < q; ++r)
            if (sample[r] == m)
                return -1;
        memcpy(sa + 3 * q, a + 3 * m, 3 * sizeof(double));
        memcpy(sb + 3 * q, b + 3 * m, 3 * sizeof(double));
    }
    /* a sample whose triangle is (nearly) degenerate in either frame fixes no
     * rotation: area below 1e-8 m^2 (sides of 0.1 mm) */
    for (int s = 0; s < 2; ++s) {
        const double *P = s ? sb : sa;
        double e1[3], e2[3], c[3];
        for (int r = 0; r < 3; ++r) {
            e1[r] = P[3 + r] - P[r];
            e2[r] = P[6 + r] - P[r];
        }
        cross3(e1, e2, c);
        if (!(0.5 * sqrt(dot3(c, c)) >= 1e-8))
            return -1;
    }
    double Th[16];
    if (orc_arun(3, sa, sb, Th) != ORC_OK)
        return -1;
    const double cos_a = cos(alpha);
    int count = 0;
    for (int m = 0; m < n; ++m) {
        int in = 0;
        if (valid[m]) {
            double y[3], rn[3];
            apply_T(Th, b + 3 * m, y);
            apply_R(Th, nb + 3 * m, rn);
            const double d[3] = {y[0] - a[3 * m], y[1] - a[3 * m + 1], y[2] - a[3 * m + 2]};
            in = sqrt(dot3(d, d)) < delta && dot3(rn, na + 3 * m) > cos_a;
        }
        count += in;
        if (inlier)
            inlier[m] = (unsigned char)in;
    }
    if (T)
        memcpy(T, Th, sizeof(Th));
    return count;
}

int orc_ransac_pairs(const orc_problem *pb, int n_pairs, const int *pi, const int *pj, const int *match_off,
                     const float *uv_i, const float *uv_j, int n_hyp, const int *samples, double delta,
                     double alpha, int *best, int *score, double *T, unsigned char *inlier)
{
    if (check_problem(pb) != ORC_OK || n_pairs < 0 || n_hyp < 1 || !match_off || !samples || !best || !T)
        return ORC_ERR_ARG;
    for (int q = 0; q < n_pairs; ++q)
        if (pi[q] < 0 || pj[q] < 0 || pi[q] >= pb->n_frames || pj[q] >= pb->n_frames || pi[q] == pj[q] ||
            match_off[q + 1] < match_off[q])
            return ORC_ERR_ARG;
    frame_maps *fm = build_frames(pb);
    for (int q = 0; q < n_pairs; ++q) {
        const int n = match_off[q + 1] - match_off[q], o = match_off[q];
        double *a = (double *)malloc(sizeof(double) * 12 * (size_t)(n > 0 ? n : 1));
        double *na = a + 3 * n, *b = a + 6 * n, *nb = a + 9 * n;
        unsigned char *valid = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
        for (int m = 0; m < n; ++m)
            valid[m] = (unsigned char)(keypoint_geometry(pb, fm, pi[q], uv_i + 2 * (size_t)(o + m), a + 3 * m,
                                                         na + 3 * m) &&
                                       keypoint_geometry(pb, fm, pj[q], uv_j + 2 * (size_t)(o + m), b + 3 * m,
                                                         nb + 3 * m));
        int bh = -1, bs = -1;
        for (int h = 0; h < n_hyp; ++h) {
            const int s = orc_ransac_score(n, a, na, b, nb, valid, samples + 3 * ((size_t)q * n_hyp + h), delta,
                                           alpha, NULL, NULL);
            if (score)
                score[(size_t)q * n_hyp + h] = s;
            if (s > bs) {
                bs = s;
                bh = h;
            }
        }
        best[q] = bs >= 0 ? bh : -1;
        double *Tq = T + 16 * (size_t)q;
        for (int r = 0; r < 16; ++r)
            Tq[r] = (r % 5 == 0) ? 1.0 : 0.0;
        if (inlier)
            memset(inlier + o, 0, (size_t)n);
        if (bs >= 0)
            orc_ransac_score(n, a, na, b, nb, valid, samples + 3 * ((size_t)q * n_hyp + bh), delta, alpha, Tq,
                             inlier ? inlier + o : NULL);
        free(a);
        free(valid);
    }
    free_frames(pb, fm);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Keypoint matching (Sec. IV-B): nearest neighbours of descriptors in
 * Euclidean distance, kept when mutual and, with ratio < 1, when the nearest
 * is closer than ratio times the second nearest (squared distances exact in
 * FP64 from the FP32 descriptors). */
int orc_match_descriptors(int na, const float *A, int nb, const float *B, int dim, double ratio, int *match,
                          double *d1_out, double *d2_out)
{
    if (na < 0 || nb < 0 || dim < 1 || (na > 0 && (!A || !match)) || (nb > 0 && !B))
        return ORC_ERR_ARG;
    int *best_b = (int *)malloc(sizeof(int) * (size_t)(nb > 0 ? nb : 1));
    double *best_bd = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    for (int b = 0; b < nb; ++b) {
        best_b[b] = -1;
        best_bd[b] = INFINITY;
    }
    int *best_a = (int *)malloc(sizeof(int) * (size_t)(na > 0 ? na : 1));
    double *d1 = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
    double *d2 = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
    for (int a = 0; a < na; ++a) {
        best_a[a] = -1;
        d1[a] = d2[a] = INFINITY;
        for (int b = 0; b < nb; ++b) {
            double d = 0.0;
            for (int k = 0; k < dim; ++k) {
                const double e = (double)A[(size_t)a * dim + k] - (double)B[(size_t)b * dim + k];
                d += e * e;
            }
            /* nearest (lowest index among equals) and second nearest of a */
            if (d < d1[a]) {
                d2[a] = d1[a];
                d1[a] = d;
                best_a[a] = b;
            } else if (d < d2[a]) {
                d2[a] = d;
            }
            /* nearest of b (lowest index among equals) */
            if (d < best_bd[b]) {
                best_bd[b] = d;
                best_b[b] = a;
            }
        }
    }
    for (int a = 0; a < na; ++a) {
        const int b = best_a[a];
        int m = (b >= 0 && best_b[b] == a) ? b : -1;
        if (m >= 0 && ratio < 1.0 && !(d1[a] < ratio * ratio * d2[a]))
            m = -1;
        match[a] = m;
        if (d1_out)
            d1_out[a] = d1[a];
        if (d2_out)
            d2_out[a] = d2[a];
    }
    free(best_b);
    free(best_bd);
    free(best_a);
    free(d1);
    free(d2);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Keyframe memory pool (Sec. IV-C, IV-E): the minimum H-subgraph objective
 * over rotation geodesic distances, solved by the paper's greedy selection,
 * and the novelty rule that admits a frame to the pool. */

double orc_rot_geodesic(const double *Ta, const double *Tb)
{
    /* tr(R_a^T R_b) = sum over entries of R_a .* R_b */
    double tr = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            tr += Ta[4 * r + c] * Tb[4 * r + c];
    double cs = 0.5 * (tr - 1.0);
    if (cs > 1.0)
        cs = 1.0;
    if (cs < -1.0)
        cs = -1.0;
    return acos(cs);
}

int orc_select_keyframes(int n_pool, const double *T_pool, const double *T_cur, int K, int *selected,
                         int *n_selected, double *cost)
{
    if (n_pool < 1 || K < 1 || !T_pool || !T_cur || !selected || !n_selected)
        return ORC_ERR_ARG;
    const int want = K < n_pool ? K : n_pool;
    double *sum = (double *)malloc(sizeof(double) * (size_t)n_pool);
    unsigned char *taken = (unsigned char *)calloc((size_t)n_pool, 1);
    if (!sum || !taken) {
        free(sum);
        free(taken);
        return ORC_ERR_ARG;
    }
    /* the initial frame first; every other keyframe starts with its distance
     * to the current frame and to the initial frame */
    selected[0] = 0;
    taken[0] = 1;
    sum[0] = orc_rot_geodesic(T_pool, T_cur);
    for (int k = 1; k < n_pool; ++k)
        sum[k] = orc_rot_geodesic(T_pool + 16 * (size_t)k, T_cur) +
                 orc_rot_geodesic(T_pool + 16 * (size_t)k, T_pool);
    int n = 1;
    while (n < want) {
        int best = -1;
        for (int k = 0; k < n_pool; ++k)
            if (!taken[k] && (best < 0 || sum[k] < sum[best]))
                best = k;
        selected[n++] = best;
        taken[best] = 1;
        for (int k = 0; k < n_pool; ++k)
            if (!taken[k])
                sum[k] += orc_rot_geodesic(T_pool + 16 * (size_t)k, T_pool + 16 * (size_t)best);
    }
    *n_selected = n;
    if (cost)
        memcpy(cost, sum, sizeof(double) * (size_t)n_pool);
    free(sum);
    free(taken);
    return ORC_OK;
}

int orc_novel_view(int n_pool, const double *T_pool, const double *T_cur, double thresh)
{
    for (int k = 0; k < n_pool; ++k)
        if (!(orc_rot_geodesic(T_pool + 16 * (size_t)k, T_cur) > thresh))
            return 0;
    return 1;
}
