// HIP kernels (gfx950) and C entry points of the front end of BundleTrack
// (Wen & Bekris, IROS 2021), Sec. IV-B: mutual nearest-neighbour matching of
// keypoint descriptors between frames, several frame pairs per launch.
//
//   match_tile_kernel     one block per (pair, 64 rows of A): the rows' dot
//                         products with B, 64 rows of B at a time, on the FP64
//                         matrix cores; squared distances |a|^2 + |b|^2 - 2 a.b
//                         in FP64; per row the nearest and second-nearest
//                         distance (lowest index among equals), per column of
//                         B the nearest of the block's rows (a partial record)
//   match_resolve_kernel  one block per pair: each row of B's nearest row of A
//                         from the partial records, then the mutual and ratio
//                         tests per row of A
//
// and the coarse registration by RANSAC of Sec. IV-B over the frames a pose
// graph holds:
//
//   ransac_hyp_kernel     one wavefront per (pair, 64 hypotheses): the pair's
//                         matched keypoints (3-D point and normal at the
//                         nearest pixel of each frame) in LDS, one hypothesis
//                         per lane: the least-squares rigid transform of its
//                         three matches (Arun et al.; SVD by one-sided Jacobi
//                         rotations) and its inlier count
//   ransac_best_kernel    one block per pair: the best hypothesis (most
//                         inliers, lowest index among equals), its transform
//                         and inlier flags
#include "pg_frontend.h"
#include "pg_device.hpp"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

namespace pg {
namespace {

constexpr int kMatchRows = 64;   // rows of A per block and rows of B per step
constexpr int kMatchThreads = 256;

struct MatchPart {   // nearest row of A (local index) to one row of B within one block's rows
    double d;
    int a;
    int pad;
};

struct MatchRow {    // per row of A: nearest and second-nearest distance, nearest row of B
    double d1, d2;
    int i1;
    int pad;
};

struct MatchArgs {
    const float* desc;
    int n_pairs;
    double ratio;
    int* match;
    double* d1;
    double* d2;
    MatchPart* part;
    MatchRow* rows;
    int a0[PG_MATCH_MAX_PAIRS], na[PG_MATCH_MAX_PAIRS];   // first row and rows of set A
    int b0[PG_MATCH_MAX_PAIRS], nb[PG_MATCH_MAX_PAIRS];   // of set B
    int out0[PG_MATCH_MAX_PAIRS];                          // first output row of the pair
    int part0[PG_MATCH_MAX_PAIRS];                         // first partial record of the pair
    int tile0[PG_MATCH_MAX_PAIRS + 1];                     // first block of the pair
};
static_assert(sizeof(MatchArgs) <= 4096, "kernel arguments");

typedef double mt_d4 __attribute__((ext_vector_type(4)));

// (d, i) before (e, j): smaller distance, then lower index
__device__ __forceinline__ bool lex_less(double d, int i, double e, int j)
{
    return d < e || (d == e && i < j);
}

// Merge two (nearest, second nearest, index of nearest) states of one row.
__device__ __forceinline__ void merge_best(double& x1, double& x2, int& xi, double y1, double y2, int yi)
{
    if (lex_less(y1, yi, x1, xi)) {
        const double t1 = x1;
        x1 = y1;
        x2 = fmin(y2, t1);
        xi = yi;
    } else {
        x2 = fmin(x2, y1);
    }
}

// One block of 256 threads: rows arow0 .. arow0 + 63 of set A against all of
// set B.  Wave w holds the matrix cores' A operand of rows 16 w .. 16 w + 15
// in registers (lane l: row l % 16, the k-quarter l / 16 of the descriptor, so
// one 16 x 16 x 4 product per step covers k = q DIM/4 + j for the four
// quarters q); a 64-row tile of B is staged in LDS and each wave multiplies
// its 16 rows with the tile's four 16-row column blocks: lane l of block t
// holds the dot products of rows 16 w + 4 v + l / 16 with column 16 t + l % 16.
template <int DIM>
__global__ __launch_bounds__(kMatchThreads) void match_tile_kernel(MatchArgs args)
{
    constexpr int KQ = DIM / 4;      // descriptor entries per quarter
    constexpr int STR = DIM + 4;     // LDS row stride (floats): rows spread over the banks
    static_assert(DIM % 16 == 0 && DIM <= 256, "descriptor length");
    extern __shared__ float sB[];    // kMatchRows x STR
    __shared__ double sna[kMatchRows], snb[kMatchRows];
    __shared__ double cmin_d[4][kMatchRows];
    __shared__ int cmin_a[4][kMatchRows];
    const int blk = blockIdx.x;
    int q = 0;
    while (q + 1 < args.n_pairs && args.tile0[q + 1] <= blk)
        ++q;
    const int at = blk - args.tile0[q];
    const int arow0 = at * kMatchRows;
    const int na = args.na[q], nb = args.nb[q];
    const float* __restrict__ A = args.desc + (size_t)args.a0[q] * DIM;
    const float* __restrict__ B = args.desc + (size_t)args.b0[q] * DIM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;

    // A operand rows in registers (rows past the set read row 0 and are masked)
    float areg[KQ];
    {
        const int r = arow0 + 16 * wave + c;
        const float* src = A + (size_t)(r < na ? r : 0) * DIM + KQ * g;
#pragma unroll
        for (int k = 0; k < KQ; k += 4) {
            const float4 v = *(const float4*)(src + k);
            areg[k] = v.x;
            areg[k + 1] = v.y;
            areg[k + 2] = v.z;
            areg[k + 3] = v.w;
        }
    }
    // squared norms of the block's rows (FP64, four threads per row)
    {
        const int r = tid >> 2, part = tid & 3;
        const int ra = arow0 + r < na ? arow0 + r : 0;
        double s = 0.0;
        for (int k = part * KQ; k < (part + 1) * KQ; ++k) {
            const double x = A[(size_t)ra * DIM + k];
            s = fma(x, x, s);
        }
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        if (part == 0)
            sna[r] = s;
    }
    // running nearest / second nearest of the lane's rows 16 w + 4 v + g
    double d1[4], d2[4];
    int i1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        d1[v] = d2[v] = INFINITY;
        i1[v] = -1;
    }
    for (int b0 = 0; b0 < nb; b0 += kMatchRows) {
        __syncthreads();   // the previous tile's LDS reads are done
        for (int e = tid; e < kMatchRows * (DIM / 4); e += kMatchThreads) {
            const int r = e / (DIM / 4), k4 = e - r * (DIM / 4);
            const float4 v = (b0 + r < nb) ? *(const float4*)(B + (size_t)(b0 + r) * DIM + 4 * k4)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
            *(float4*)(sB + r * STR + 4 * k4) = v;
        }
        __syncthreads();
        {
            const int r = tid >> 2, part = tid & 3;
            double s = 0.0;
            for (int k = part * KQ; k < (part + 1) * KQ; ++k) {
                const double x = sB[r * STR + k];
                s = fma(x, x, s);
            }
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            if (part == 0)
                snb[r] = s;
        }
        mt_d4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = mt_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < KQ; j += 4) {
            float4 bq[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                bq[t] = *(const float4*)(sB + (16 * t + c) * STR + KQ * g + j);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const double av = (double)areg[j + jj];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float bv = (jj == 0) ? bq[t].x : (jj == 1) ? bq[t].y : (jj == 2) ? bq[t].z : bq[t].w;
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)bv, acc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // snb complete
        // distances; the lane's rows and columns
        double cd[4];
        int ca[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            cd[t] = INFINITY;
            ca[t] = 0x7fffffff;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ra = 16 * wave + 4 * v + g;
            const bool aok = arow0 + ra < na;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = b0 + 16 * t + c;
                const double d = (aok && b < nb) ? sna[ra] + snb[16 * t + c] - 2.0 * acc[t][v] : INFINITY;
                if (lex_less(d, b, d1[v], i1[v])) {
                    d2[v] = d1[v];
                    d1[v] = d;
                    i1[v] = b;
                } else if (d < d2[v]) {
                    d2[v] = d;
                }
                if (aok && lex_less(d, arow0 + ra, cd[t], ca[t])) {
                    cd[t] = d;
                    ca[t] = arow0 + ra;
                }
            }
        }
        // column minima over the wave's 16 rows (lanes of one column: xor 16, 32),
        // then over the four waves
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
                const double od = __shfl_xor(cd[t], o);
                const int oa = __shfl_xor(ca[t], o);
                if (lex_less(od, oa, cd[t], ca[t])) {
                    cd[t] = od;
                    ca[t] = oa;
                }
            }
            if (g == 0) {
                cmin_d[wave][16 * t + c] = cd[t];
                cmin_a[wave][16 * t + c] = ca[t];
            }
        }
        __syncthreads();
        if (tid < kMatchRows && b0 + tid < nb) {
            double bd = cmin_d[0][tid];
            int ba = cmin_a[0][tid];
            for (int w = 1; w < 4; ++w)
                if (lex_less(cmin_d[w][tid], cmin_a[w][tid], bd, ba)) {
                    bd = cmin_d[w][tid];
                    ba = cmin_a[w][tid];
                }
            MatchPart p;
            p.d = bd;
            p.a = ba;
            p.pad = 0;
            args.part[args.part0[q] + (size_t)at * nb + b0 + tid] = p;
        }
    }
    // per row: merge the 16 lanes of its columns (xor 1, 2, 4, 8)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const double y1 = __shfl_xor(d1[v], o), y2 = __shfl_xor(d2[v], o);
            const int yi = __shfl_xor(i1[v], o);
            merge_best(d1[v], d2[v], i1[v], y1, y2, yi);
        }
        const int ra = arow0 + 16 * wave + 4 * v + g;
        if (c == 0 && ra < na) {
            MatchRow r;
            r.d1 = d1[v];
            r.d2 = d2[v];
            r.i1 = i1[v];
            r.pad = 0;
            args.rows[args.out0[q] + ra] = r;
        }
    }
}

// One block per pair: nearest row of A of every row of B (lowest index among
// equals) from the partial records, then the mutual and ratio tests.
__global__ __launch_bounds__(kMatchThreads) void match_resolve_kernel(MatchArgs args)
{
    __shared__ int best_of_b[PG_MATCH_MAX_ROWS];
    const int q = blockIdx.x;
    const int na = args.na[q], nb = args.nb[q];
    const int tiles = args.tile0[q + 1] - args.tile0[q];
    for (int b = threadIdx.x; b < nb; b += kMatchThreads) {
        double bd = INFINITY;
        int ba = 0x7fffffff;
        for (int at = 0; at < tiles; ++at) {
            const MatchPart p = args.part[args.part0[q] + (size_t)at * nb + b];
            if (lex_less(p.d, p.a, bd, ba)) {
                bd = p.d;
                ba = p.a;
            }
        }
        best_of_b[b] = (ba == 0x7fffffff) ? -1 : ba;
    }
    __syncthreads();
    const double r2 = args.ratio * args.ratio;
    for (int a = threadIdx.x; a < na; a += kMatchThreads) {
        const MatchRow r = args.rows[args.out0[q] + a];
        int m = (r.i1 >= 0 && best_of_b[r.i1] == a) ? r.i1 : -1;
        if (m >= 0 && args.ratio < 1.0 && !(r.d1 < r2 * r.d2))
            m = -1;
        const int o = args.out0[q] + a;
        args.match[o] = m;
        if (args.d1)
            args.d1[o] = r.d1;
        if (args.d2)
            args.d2[o] = r.d2;
    }
}

// Scratch of the allocation-free entry point: the partial records, then the
// row records, in one fixed array per device.  Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress (scratch_on_device), taken once with that device current.
constexpr size_t kScratchPartBytes = sizeof(MatchPart) * (size_t)PG_MATCH_SCRATCH_PARTIALS;
constexpr size_t kScratchBytes = kScratchPartBytes + sizeof(MatchRow) * (size_t)PG_MATCH_SCRATCH_ROWS;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// ------------------------------------------------------------ RANSAC

constexpr int kRansacHyp = 64;   // hypotheses per wavefront block

struct RansacArgs {
    const float4* maps;     // n_frames x H x W packed {normal, z}; z = 0: no valid point
    int W, H;
    double fx, fy, cx, cy;
    const int4* pairs;      // per pair: frame i, frame j, first match, match count
    const float* uv_i;      // per match: (u, v) in frame i
    const float* uv_j;      // per match: (u, v) in frame j
    const int* samples;     // per pair and hypothesis: three match indices
    int n_hyp, hyp_blocks;
    double delta, cos_alpha;
    int* score;             // per pair and hypothesis; -1: unusable sample
    double* T;              // per pair and hypothesis: [R | t] (12)
    int* best;              // per pair
    double* T_best;         // per pair: 16, row-major
    unsigned char* inlier;  // per match
};

// 3-D point (pi_D^-1 at the nearest pixel, ties up) and normal of a keypoint;
// false outside the image or where the frame has no valid point
__device__ bool keypoint_point(const RansacArgs& a, int f, float uf, float vf, double* p, double* nrm)
{
    const double x = (double)uf, y = (double)vf;
    double u = floor(x), v = floor(y);
    u += (x - u >= 0.5) ? 1.0 : 0.0;
    v += (y - v >= 0.5) ? 1.0 : 0.0;
    if (!(u >= 0.0 && u < (double)a.W && v >= 0.0 && v < (double)a.H))
        return false;
    const float4 e = a.maps[(size_t)f * a.W * a.H + (size_t)v * a.W + (size_t)u];
    if (!(e.w > 0.0f))
        return false;
    const double z = e.w;
    p[0] = (z * (u - a.cx)) / a.fx;
    p[1] = (z * (v - a.cy)) / a.fy;
    p[2] = z;
    nrm[0] = e.x;
    nrm[1] = e.y;
    nrm[2] = e.z;
    return true;
}

// Rotation and translation minimising sum |R b_k + t - a_k|^2 over three
// point pairs (Arun et al.): S = sum (a_k - ca)(b_k - cb)^T = U D V^T,
// R = U diag(1, 1, det V) V^T with U's third column the cross product of its
// first two (right-handed; the third singular value of three points is 0),
// t = ca - R cb.  The SVD by one-sided Jacobi rotations: columns p, q of
// W = S V are rotated until orthogonal, then sorted by decreasing length.
// False for collinear points (second singular value below 1e-12 of the first).
__device__ bool arun3(const double (&A)[9], const double (&B)[9], double (&T)[12])
{
    double ca[3], cb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        ca[r] = (A[r] + A[3 + r] + A[6 + r]) / 3.0;
        cb[r] = (B[r] + B[3 + r] + B[6 + r]) / 3.0;
    }
    double W[9], V[9];   // row-major 3 x 3
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                s = fma(A[3 * k + r] - ca[r], B[3 * k + c] - cb[c], s);
            W[3 * r + c] = s;
            V[3 * r + c] = (r == c) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool turned = false;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = (pq == 2) ? 1 : 0, q = (pq == 0) ? 1 : 2;
            double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                al = fma(W[3 * r + p], W[3 * r + p], al);
                be = fma(W[3 * r + q], W[3 * r + q], be);
                ga = fma(W[3 * r + p], W[3 * r + q], ga);
            }
            if (!(fabs(ga) > 1e-15 * sqrt(al * be)))
                continue;
            turned = true;
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double wp = W[3 * r + p], wq = W[3 * r + q];
                W[3 * r + p] = cs * wp - sn * wq;
                W[3 * r + q] = sn * wp + cs * wq;
                const double vp = V[3 * r + p], vq = V[3 * r + q];
                V[3 * r + p] = cs * vp - sn * vq;
                V[3 * r + q] = sn * vp + cs * vq;
            }
        }
        if (!turned)
            break;
    }
    double nn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        nn[c] = W[c] * W[c] + W[3 + c] * W[3 + c] + W[6 + c] * W[6 + c];
    // the two longest columns, in order (the third is not needed)
    int c0 = 0, c1 = 1, c2 = 2;
    if (nn[c1] > nn[c0]) { const int x = c0; c0 = c1; c1 = x; }
    if (nn[c2] > nn[c0]) { const int x = c0; c0 = c2; c2 = x; }
    if (nn[c2] > nn[c1]) { const int x = c1; c1 = c2; c2 = x; }
    const double n0 = sqrt(nn[c0]), n1 = sqrt(nn[c1]);
    if (!(n1 > 1e-12 * n0))
        return false;
    double u0[3], u1[3], u2[3], v0[3], v1[3], v2[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        u0[r] = W[3 * r + c0] / n0;
        u1[r] = W[3 * r + c1] / n1;
        v0[r] = V[3 * r + c0];
        v1[r] = V[3 * r + c1];
        v2[r] = V[3 * r + c2];
    }
    u2[0] = u0[1] * u1[2] - u0[2] * u1[1];
    u2[1] = u0[2] * u1[0] - u0[0] * u1[2];
    u2[2] = u0[0] * u1[1] - u0[1] * u1[0];
    // det of V with its columns in sorted order
    const double detv = v0[0] * (v1[1] * v2[2] - v1[2] * v2[1]) - v1[0] * (v0[1] * v2[2] - v0[2] * v2[1]) +
                        v2[0] * (v0[1] * v1[2] - v0[2] * v1[1]);
    const double d = detv < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            T[4 * r + c] = u0[r] * v0[c] + u1[r] * v1[c] + d * u2[r] * v2[c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        T[4 * r + 3] = ca[r] - (T[4 * r] * cb[0] + T[4 * r + 1] * cb[1] + T[4 * r + 2] * cb[2]);
    return true;
}

// inlier test of one match under [R | t]: |R b + t - a| < delta and
// (R n_b) . n_a > cos alpha
__device__ __forceinline__ bool ransac_inlier(const double (&T)[12], const double* a, const double* na,
                                              const double* b, const double* nb, double delta, double cos_alpha)
{
    double d2 = 0.0, c = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double y = T[4 * r] * b[0] + T[4 * r + 1] * b[1] + T[4 * r + 2] * b[2] + T[4 * r + 3] - a[r];
        const double rn = T[4 * r] * nb[0] + T[4 * r + 1] * nb[1] + T[4 * r + 2] * nb[2];
        d2 = fma(y, y, d2);
        c = fma(rn, na[r], c);
    }
    return sqrt(d2) < delta && c > cos_alpha;
}

__global__ __launch_bounds__(kRansacHyp) void ransac_hyp_kernel(RansacArgs args)
{
    __shared__ double sg[12 * PG_RANSAC_MAX_MATCHES];   // per match: a, n_a, b, n_b
    __shared__ unsigned char sv[PG_RANSAC_MAX_MATCHES];
    const int q = blockIdx.x / args.hyp_blocks;
    const int hb = blockIdx.x - q * args.hyp_blocks;
    const int4 pr = args.pairs[q];
    const int n = pr.w;
    for (int m = threadIdx.x; m < n; m += kRansacHyp) {
        const int k = pr.z + m;
        double* g = sg + 12 * m;
        const bool ok = keypoint_point(args, pr.x, args.uv_i[2 * k], args.uv_i[2 * k + 1], g, g + 3) &&
                        keypoint_point(args, pr.y, args.uv_j[2 * k], args.uv_j[2 * k + 1], g + 6, g + 9);
        sv[m] = ok ? 1 : 0;
    }
    __syncthreads();
    const int h = hb * kRansacHyp + threadIdx.x;
    if (h >= args.n_hyp)
        return;
    const size_t o = (size_t)q * args.n_hyp + h;
    int s[3];
    bool usable = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s[k] = args.samples[3 * o + k];
        usable = usable && s[k] >= 0 && s[k] < n;
    }
    usable = usable && s[0] != s[1] && s[0] != s[2] && s[1] != s[2];
    double A[9], B[9], T[12];
    if (usable) {
        usable = sv[s[0]] && sv[s[1]] && sv[s[2]];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                A[3 * k + r] = sg[12 * s[k] + r];
                B[3 * k + r] = sg[12 * s[k] + 6 + r];
            }
    }
    // a triangle of area below 1e-8 m^2 in either frame fixes no rotation
    if (usable) {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double* P = f ? B : A;
            const double e1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
            const double e2[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
            const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                         cz = e1[0] * e2[1] - e1[1] * e2[0];
            usable = usable && (0.5 * sqrt(cx * cx + cy * cy + cz * cz) >= 1e-8);
        }
    }
    if (usable)
        usable = arun3(A, B, T);
    int count = -1;
    if (usable) {
        count = 0;
        for (int m = 0; m < n; ++m)
            count += (sv[m] && ransac_inlier(T, sg + 12 * m, sg + 12 * m + 3, sg + 12 * m + 6, sg + 12 * m + 9,
                                             args.delta, args.cos_alpha))
                         ? 1
                         : 0;
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k)
            T[k] = 0.0;
    }
    args.score[o] = count;
#pragma unroll
    for (int k = 0; k < 12; ++k)
        args.T[12 * o + k] = T[k];
}

__global__ __launch_bounds__(256) void ransac_best_kernel(RansacArgs args)
{
    __shared__ int ws[4], wh[4];
    __shared__ double sT[12];
    __shared__ int sbest;
    const int q = blockIdx.x;
    const int4 pr = args.pairs[q];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // most inliers, lowest index among equals
    int bs = -1, bh = 0x7fffffff;
    for (int h = tid; h < args.n_hyp; h += 256) {
        const int sc = args.score[(size_t)q * args.n_hyp + h];
        if (sc > bs) {
            bs = sc;
            bh = h;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int os = __shfl_xor(bs, o), oh = __shfl_xor(bh, o);
        if (os > bs || (os == bs && oh < bh)) {
            bs = os;
            bh = oh;
        }
    }
    if (lane == 0) {
        ws[wave] = bs;
        wh[wave] = bh;
    }
    __syncthreads();
    if (tid == 0) {
        int s = ws[0], hh = wh[0];
        for (int w = 1; w < 4; ++w)
            if (ws[w] > s || (ws[w] == s && wh[w] < hh)) {
                s = ws[w];
                hh = wh[w];
            }
        sbest = (s >= 0) ? hh : -1;
        args.best[q] = sbest;
    }
    __syncthreads();
    const int b = sbest;
    if (tid < 12)
        sT[tid] = (b >= 0) ? args.T[12 * ((size_t)q * args.n_hyp + b) + tid] : ((tid % 5 == 0) ? 1.0 : 0.0);
    __syncthreads();
    if (tid < 16)
        args.T_best[16 * q + tid] = (tid < 12) ? sT[tid] : (tid == 15 ? 1.0 : 0.0);
    double T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        T[k] = sT[k];
    for (int m = tid; m < pr.w; m += 256) {
        const int k = pr.z + m;
        double g[12];
        bool in = false;
        if (b >= 0 && keypoint_point(args, pr.x, args.uv_i[2 * k], args.uv_i[2 * k + 1], g, g + 3) &&
            keypoint_point(args, pr.y, args.uv_j[2 * k], args.uv_j[2 * k + 1], g + 6, g + 9))
            in = ransac_inlier(T, g, g + 3, g + 6, g + 9, args.delta, args.cos_alpha);
        args.inlier[k] = in ? 1 : 0;
    }
}

// ------------------------------------------------------------ keyframe pool

constexpr int kPoolThreads = 256;
constexpr int kPoolPer = PG_POOL_MAX / kPoolThreads;   // keyframes per thread

// rotation geodesic distance between pose a (global) and pose b (LDS)
__device__ __forceinline__ double pool_geodesic(const double* __restrict__ a, const double* b)
{
    double tr = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            tr = fma(a[4 * r + c], b[4 * r + c], tr);
    return acos(fmin(1.0, fmax(-1.0, 0.5 * (tr - 1.0))));
}

// One block: thread t owns keyframes t + 256 m; per greedy step a block-wide
// argmin of (sum, index) over the keyframes not yet taken, then every sum
// grows by its distance to the new keyframe.  Pool entry 16 n_pool .. 16
// n_pool + 15 holds the current frame's pose.
__global__ __launch_bounds__(kPoolThreads) void keyframe_select_kernel(const double* __restrict__ T, int n_pool, int K,
                                                                       double novel_rad, int* out)
{
    __shared__ double piv[16];
    __shared__ double cur[16];
    __shared__ double wd[kPoolThreads / 64];
    __shared__ int wk[kPoolThreads / 64];
    __shared__ int spick;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 16) {
        cur[tid] = T[16 * (size_t)n_pool + tid];
        piv[tid] = T[tid];   // keyframe 0, selected first
    }
    __syncthreads();
    double sum[kPoolPer];
    bool taken[kPoolPer];
    double dmin = INFINITY;
#pragma unroll
    for (int m = 0; m < kPoolPer; ++m) {
        const int k = tid + kPoolThreads * m;
        taken[m] = (k == 0) || k >= n_pool;
        sum[m] = INFINITY;
        if (k < n_pool) {
            const double dc = pool_geodesic(T + 16 * (size_t)k, cur);
            dmin = fmin(dmin, dc);
            sum[m] = dc + (k == 0 ? 0.0 : pool_geodesic(T + 16 * (size_t)k, piv));
        }
    }
    // novelty: the nearest keyframe's distance, over the block
    for (int o = 32; o > 0; o >>= 1)
        dmin = fmin(dmin, __shfl_xor(dmin, o));
    if (lane == 0)
        wd[wave] = dmin;
    __syncthreads();
    if (tid == 0) {
        double d = wd[0];
        for (int w = 1; w < kPoolThreads / 64; ++w)
            d = fmin(d, wd[w]);
        out[0] = d > novel_rad ? 1 : 0;
        out[2] = 0;   // selected[0]
    }
    // cost of keyframe 0 as it was when chosen: its distance to the current frame
    double* cost = (double*)(out + 2 + PG_POOL_MAX);
    if (tid == 0)
        cost[0] = sum[0];
    const int want = K < n_pool ? K : n_pool;
    for (int n = 1; n < want; ++n) {
        double bd = INFINITY;
        int bk = 0x7fffffff;
#pragma unroll
        for (int m = 0; m < kPoolPer; ++m) {
            const int k = tid + kPoolThreads * m;
            if (!taken[m] && (sum[m] < bd || (sum[m] == bd && k < bk))) {
                bd = sum[m];
                bk = k;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o);
            const int ok = __shfl_xor(bk, o);
            if (od < bd || (od == bd && ok < bk)) {
                bd = od;
                bk = ok;
            }
        }
        __syncthreads();   // the previous step's pivot reads are done
        if (lane == 0) {
            wd[wave] = bd;
            wk[wave] = bk;
        }
        __syncthreads();
        if (tid == 0) {
            double d = wd[0];
            int k = wk[0];
            for (int w = 1; w < kPoolThreads / 64; ++w)
                if (wd[w] < d || (wd[w] == d && wk[w] < k)) {
                    d = wd[w];
                    k = wk[w];
                }
            spick = k;
            out[2 + n] = k;
        }
        __syncthreads();
        const int pick = spick;
        if (tid < 16)
            piv[tid] = T[16 * (size_t)pick + tid];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kPoolPer; ++m) {
            const int k = tid + kPoolThreads * m;
            if (k == pick) {
                taken[m] = true;
                cost[k] = sum[m];
            } else if (!taken[m]) {
                sum[m] += pool_geodesic(T + 16 * (size_t)k, piv);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < kPoolPer; ++m) {
        const int k = tid + kPoolThreads * m;
        if (k < n_pool && !taken[m])
            cost[k] = sum[m];
    }
    if (tid == 0)
        out[1] = want;
}

thread_local std::string g_frontend_error;

pg_status ffail(pg_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_frontend_error = buf;
    return s;
}

bool on_device(const void* p)
{
    if (!p)
        return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

// Argument checks and the pair tables; the partial and row counts the call needs.
pg_status match_setup(const float* desc, const int* set_off, int n_sets, int dim, const int* pair_a,
                      const int* pair_b, int n_pairs, double ratio, int* match, double* d1, double* d2,
                      MatchArgs& a, size_t& n_part, size_t& n_rows, int& n_blocks)
{
    g_frontend_error.clear();
    if (n_pairs < 1 || n_pairs > PG_MATCH_MAX_PAIRS)
        return n_pairs < 1 ? ffail(PG_ERR_INVALID_ARG, "n_pairs %d < 1", n_pairs)
                           : ffail(PG_ERR_CAPACITY, "n_pairs %d exceeds %d", n_pairs, PG_MATCH_MAX_PAIRS);
    if (dim != 32 && dim != 64 && dim != 128 && dim != 256)
        return ffail(PG_ERR_INVALID_ARG, "descriptor length %d is not 32, 64, 128 or 256", dim);
    if (n_sets < 1 || !set_off || !pair_a || !pair_b)
        return ffail(PG_ERR_INVALID_ARG, "set offsets and pair arrays are required");
    if (!(ratio > 0.0) || !isfinite(ratio))
        return ffail(PG_ERR_INVALID_ARG, "ratio must be positive and finite");
    for (int s = 0; s < n_sets; ++s) {
        if (set_off[s] < 0 || set_off[s + 1] < set_off[s])
            return ffail(PG_ERR_INVALID_ARG, "set offsets must be non-negative and non-decreasing");
        if (set_off[s + 1] - set_off[s] > PG_MATCH_MAX_ROWS)
            return ffail(PG_ERR_CAPACITY, "set %d has %d rows, more than %d", s, set_off[s + 1] - set_off[s],
                         PG_MATCH_MAX_ROWS);
    }
    if (!on_device(desc) || !on_device(match) || (d1 && !on_device(d1)) || (d2 && !on_device(d2)))
        return ffail(PG_ERR_INVALID_ARG, "descriptors and outputs must be device memory");
    if (((uintptr_t)desc & 15) != 0)
        return ffail(PG_ERR_INVALID_ARG, "descriptors must be 16-byte aligned");
    a = MatchArgs{};
    a.desc = desc;
    a.n_pairs = n_pairs;
    a.ratio = ratio;
    a.match = match;
    a.d1 = d1;
    a.d2 = d2;
    n_part = 0;
    n_rows = 0;
    n_blocks = 0;
    for (int q = 0; q < n_pairs; ++q) {
        const int sa = pair_a[q], sb = pair_b[q];
        if (sa < 0 || sb < 0 || sa >= n_sets || sb >= n_sets)
            return ffail(PG_ERR_INVALID_ARG, "pair %d names set %d / %d of %d", q, sa, sb, n_sets);
        a.a0[q] = set_off[sa];
        a.na[q] = set_off[sa + 1] - set_off[sa];
        a.b0[q] = set_off[sb];
        a.nb[q] = set_off[sb + 1] - set_off[sb];
        a.out0[q] = (int)n_rows;
        a.part0[q] = (int)n_part;
        a.tile0[q] = n_blocks;
        const int tiles = (a.na[q] + kMatchRows - 1) / kMatchRows;
        n_blocks += tiles;
        n_rows += (size_t)a.na[q];
        n_part += (size_t)tiles * (size_t)a.nb[q];
        if (n_part > (size_t)1 << 30)
            return ffail(PG_ERR_CAPACITY, "too many partial records");
    }
    a.tile0[n_pairs] = n_blocks;
    return PG_OK;
}

template <int DIM>
hipError_t launch_match_dim(const MatchArgs& a, int n_blocks, hipStream_t st)
{
    const size_t lds = sizeof(float) * kMatchRows * (DIM + 4);
    static bool attr_set = false;
    if (!attr_set && lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)match_tile_kernel<DIM>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    if (n_blocks > 0)
        match_tile_kernel<DIM><<<n_blocks, kMatchThreads, lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_match(const MatchArgs& a, int dim, int n_blocks, hipStream_t st)
{
    hipError_t e;
    switch (dim) {
    case 32: e = launch_match_dim<32>(a, n_blocks, st); break;
    case 64: e = launch_match_dim<64>(a, n_blocks, st); break;
    case 128: e = launch_match_dim<128>(a, n_blocks, st); break;
    default: e = launch_match_dim<256>(a, n_blocks, st); break;
    }
    if (e != hipSuccess)
        return e;
    match_resolve_kernel<<<a.n_pairs, kMatchThreads, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace

// RANSAC over the pairs of a graph's frames (arrays in device memory; the
// counts were checked by the caller)
hipError_t launch_ransac(const float4* maps, int W, int H, double fx, double fy, double cx, double cy,
                         const int4* pairs, int n_pairs, const float* uv_i, const float* uv_j, const int* samples,
                         int n_hyp, double delta, double cos_alpha, int* score, double* T, int* best, double* T_best,
                         unsigned char* inlier, hipStream_t st)
{
    RansacArgs a;
    a.maps = maps;
    a.W = W;
    a.H = H;
    a.fx = fx;
    a.fy = fy;
    a.cx = cx;
    a.cy = cy;
    a.pairs = pairs;
    a.uv_i = uv_i;
    a.uv_j = uv_j;
    a.samples = samples;
    a.n_hyp = n_hyp;
    a.hyp_blocks = (n_hyp + kRansacHyp - 1) / kRansacHyp;
    a.delta = delta;
    a.cos_alpha = cos_alpha;
    a.score = score;
    a.T = T;
    a.best = best;
    a.T_best = T_best;
    a.inlier = inlier;
    if (n_pairs <= 0)
        return hipSuccess;
    ransac_hyp_kernel<<<n_pairs * a.hyp_blocks, kRansacHyp, 0, st>>>(a);
    ransac_best_kernel<<<n_pairs, 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace pg

using namespace pg;

extern "C" {

pg_status pg_match_descriptors(const float* desc, const int* set_off, int n_sets, int dim, const int* pair_a,
                               const int* pair_b, int n_pairs, double ratio, int* match, double* d1, double* d2,
                               void* hip_stream)
{
    MatchArgs a;
    size_t n_part = 0, n_rows = 0;
    int n_blocks = 0;
    pg_status s = match_setup(desc, set_off, n_sets, dim, pair_a, pair_b, n_pairs, ratio, match, d1, d2, a, n_part,
                              n_rows, n_blocks);
    if (s != PG_OK)
        return s;
    hipStream_t st = (hipStream_t)hip_stream;
    void* mem = nullptr;
    const size_t bytes = sizeof(MatchPart) * (n_part ? n_part : 1) + sizeof(MatchRow) * (n_rows ? n_rows : 1);
    hipError_t e = hipMallocAsync(&mem, bytes, st);
    if (e != hipSuccess)
        return ffail(e == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP, "hipMallocAsync: %s",
                     hipGetErrorString(e));
    a.part = (MatchPart*)mem;
    a.rows = (MatchRow*)((char*)mem + sizeof(MatchPart) * (n_part ? n_part : 1));
    e = launch_match(a, dim, n_blocks, st);
    const hipError_t ef = hipFreeAsync(mem, st);
    if (e != hipSuccess)
        return ffail(PG_ERR_HIP, "match launch: %s", hipGetErrorString(e));
    if (ef != hipSuccess)
        return ffail(PG_ERR_HIP, "hipFreeAsync: %s", hipGetErrorString(ef));
    return PG_OK;
}

pg_status pg_match_descriptors_noalloc(const float* desc, const int* set_off, int n_sets, int dim,
                                       const int* pair_a, const int* pair_b, int n_pairs, double ratio, int* match,
                                       double* d1, double* d2, void* hip_stream)
{
    MatchArgs a;
    size_t n_part = 0, n_rows = 0;
    int n_blocks = 0;
    pg_status s = match_setup(desc, set_off, n_sets, dim, pair_a, pair_b, n_pairs, ratio, match, d1, d2, a, n_part,
                              n_rows, n_blocks);
    if (s != PG_OK)
        return s;
    if (n_part > (size_t)PG_MATCH_SCRATCH_PARTIALS || n_rows > (size_t)PG_MATCH_SCRATCH_ROWS)
        return ffail(PG_ERR_CAPACITY, "%zu partial records / %zu rows exceed the fixed scratch (%d / %d)", n_part,
                     n_rows, PG_MATCH_SCRATCH_PARTIALS, PG_MATCH_SCRATCH_ROWS);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return ffail(PG_ERR_NO_DEVICE, "no current device");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return ffail(PG_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        base = g_scratch_ptr[dev];
    }
    a.part = (MatchPart*)base;
    a.rows = (MatchRow*)((char*)base + kScratchPartBytes);
    e = launch_match(a, dim, n_blocks, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return ffail(PG_ERR_HIP, "match launch: %s", hipGetErrorString(e));
    return PG_OK;
}

pg_status pg_select_keyframes(const double* T_pool, int n_pool, const double* T_cur, int K, double novel_rad,
                              int* selected, int* n_selected, int* novel, double* cost, void* hip_stream)
{
    g_frontend_error.clear();
    if (!T_pool || !T_cur || !selected || !n_selected || n_pool < 1 || K < 1 || !(novel_rad >= 0.0))
        return ffail(PG_ERR_INVALID_ARG, "pool, current pose, outputs, n_pool >= 1, K >= 1 and novel_rad >= 0 "
                                         "are required");
    if (n_pool > PG_POOL_MAX)
        return ffail(PG_ERR_CAPACITY, "pool of %d keyframes exceeds %d", n_pool, PG_POOL_MAX);
    hipStream_t st = (hipStream_t)hip_stream;
    // device block: the pool and the current pose, then the results (novel,
    // count, PG_POOL_MAX indices, PG_POOL_MAX costs)
    const size_t tb = sizeof(double) * 16 * ((size_t)n_pool + 1);
    const size_t rb = sizeof(int) * (2 + PG_POOL_MAX) + sizeof(double) * PG_POOL_MAX;
    void* mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, tb + rb, st);
    if (e != hipSuccess)
        return ffail(e == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP, "hipMallocAsync: %s",
                     hipGetErrorString(e));
    double* dT = (double*)mem;
    int* dout = (int*)((char*)mem + tb);
    e = hipMemcpyAsync(dT, T_pool, sizeof(double) * 16 * n_pool,
                       on_device(T_pool) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dT + 16 * (size_t)n_pool, T_cur, sizeof(double) * 16,
                           on_device(T_cur) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        keyframe_select_kernel<<<1, kPoolThreads, 0, st>>>(dT, n_pool, K, novel_rad, dout);
        e = hipGetLastError();
    }
    std::vector<char> res(rb);
    if (e == hipSuccess)
        e = hipMemcpyAsync(res.data(), dout, rb, hipMemcpyDeviceToHost, st);
    const hipError_t ef = hipFreeAsync(mem, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess || ef != hipSuccess)
        return ffail(PG_ERR_HIP, "keyframe selection: %s", hipGetErrorString(e != hipSuccess ? e : ef));
    const int* ri = (const int*)res.data();
    const int n = ri[1];
    if (novel)
        *novel = ri[0];
    *n_selected = n;
    for (int k = 0; k < n && k < K; ++k)
        selected[k] = ri[2 + k];
    if (cost)
        memcpy(cost, res.data() + sizeof(int) * (2 + PG_POOL_MAX), sizeof(double) * n_pool);
    return PG_OK;
}

const char* pg_frontend_last_error(void) { return g_frontend_error.c_str(); }

}  // extern "C"
