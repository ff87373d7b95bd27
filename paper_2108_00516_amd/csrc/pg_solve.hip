// HIP kernels (gfx950) of the FP64 normal equations and their solve in
// BundleTrack's online pose-graph optimisation (Wen & Bekris, IROS 2021),
// Sec. IV-D.
//
//   assemble_kernel    FP64 expansion of the per-pair sums of the association
//                      into the 6x6 node blocks of J^T W J and J^T W r, in a
//                      fixed order (also written as the free-node system
//                      [H_ff | -g_f]); the (i,j), (j,i) and (j,j) blocks of a
//                      pair follow from its (i,i) sums and the adjoint of
//                      A = T_i T_j^-1;
//   solve_mfma_kernel  FP64 block LDL^T (one wavefront) or block Gauss-Jordan
//                      solve of the free-node system on the matrix cores;
//   solve_kernel       FP64 Cholesky (or Jacobi-PCG) solve over the free nodes;
//   mf_pcg_kernel      matrix-free PCG from the per-pair sums;
// each then applies T <- Exp(delta) T and computes the next iteration's
// transforms.
#include "pg_device.hpp"
#include "pg_util.hpp"

#include <math.h>

namespace pg {

__device__ __forceinline__ void st_global_f4(float* p, float x, float y, float z, float w)
{
    pg_f4v v = {x, y, z, w};
    *(__attribute__((address_space(1))) pg_f4v*)p = v;
}

// --------------------------------------------------- FP64 normal equations

// 6x6 adjoint of A = [R t] for twists [v; w]: [[R, [t]x R], [0, R]]
__device__ __forceinline__ double adj(const double* __restrict__ X, int r, int c)
{
    if (r >= 3 && c < 3)
        return 0.0;
    if (r < 3 && c >= 3) {
        const int cc = c - 3;
        const double t0 = X[3], t1 = X[7], t2 = X[11];
        const double R0 = X[cc], R1 = X[4 + cc], R2 = X[8 + cc];
        // ([t]x R)[r][cc] = (t x R_col)[r]
        return (r == 0) ? (t1 * R2 - t2 * R1) : (r == 1) ? (t2 * R0 - t0 * R2) : (t0 * R1 - t1 * R0);
    }
    const int rr = r % 3, cc = c % 3;
    return X[4 * rr + cc];
}

__device__ __forceinline__ double sym6(const double* M, int a, int b)
{
    return (a <= b) ? M[upper_index(a, b, 6)] : M[upper_index(b, a, 6)];
}

__device__ __forceinline__ int sym12_index(int a, int b)
{
    return (a <= b) ? upper_index(a, b, 12) : upper_index(b, a, 12);
}

__device__ __forceinline__ double sym12(const double* F, int a, int b)
{
    return (a <= b) ? F[upper_index(a, b, 12)] : F[upper_index(b, a, 12)];
}

constexpr int kAsmThreads = 1024;
constexpr int kMaxPairsPerBlock = 2 * (kMaxFrames - 1);
constexpr int kMaxTgtPairs = kMaxFrames - 1;
constexpr int kAsmChunks = 8;   // tile-sum chunks per field of an off-diagonal block

constexpr int kSumBatch = 32;   // partial records of one field loaded together

// Sum of the partial records [t0, t1) of one field in a fixed order: batches of
// kSumBatch loads issued together (the tail of a batch reads an in-bounds
// record and drops it), each summed as a pairwise tree, batches in order.
__device__ __forceinline__ double sum_records(const float* __restrict__ src, int t0, int t1)
{
    double s = 0.0;
    for (int t = t0; t < t1; t += kSumBatch) {
        double v[kSumBatch];
#pragma unroll
        for (int k = 0; k < kSumBatch; ++k) {
            const int tk = (t + k < t1) ? t + k : t1 - 1;
            const float x = ld_global(src + (size_t)tk * kDenseStride);
            v[k] = (t + k < t1) ? (double)x : 0.0;
        }
#pragma unroll
        for (int w = kSumBatch / 2; w > 0; w /= 2)
#pragma unroll
            for (int k = 0; k < w; ++k)
                v[k] += v[k + w];
        s += v[0];
    }
    return s;
}

// One block per node block (I, J), I >= J, of the 6N x 6N system.  A diagonal
// block sums the 2(N-1) ordered pairs touching node I (source role: M and v
// as they are; target role: Ad^T M Ad and -Ad^T v), an off-diagonal block the
// pairs (I, J) and (J, I) (-M Ad and -(M Ad)^T); the feature blocks of Eq. 2
// (each match counted for both orderings of Eq. 1) are added; H is written in
// both triangles (diagonal blocks: the upper triangle, mirrored, so H is
// exactly symmetric), with the gradient segment and the node's energy/count
// record.  First phase: every global read of the block at once (partial
// records of each pair and field, summed in FP64 in a fixed order - split into
// kAsmChunks contiguous chunks for the two pairs of an off-diagonal block -,
// the pairs' FP64 transforms and the oriented feature entries); then the
// adjoint expansion in LDS.
__global__ __launch_bounds__(kAsmThreads) void assemble_kernel(const GraphDev* __restrict__ gds,
                                                               const int2* __restrict__ nbs)
{
    const int2 nb = nbs[blockIdx.x];
    const GraphDev& gd = gds[nb.x];
    // the reads of phase 1 are in bounds whatever the status holds: it is
    // loaded with them and tested before anything is written
    const int status = ld_global(gd.status);
    const int I = nb.y & 0xff, J = (nb.y >> 8) & 0xff;
    const int N = gd.n_frames, n6 = 6 * N;
    // free-node positions (-1: fixed)
    const int fI = ld_global(gd.free_pos + I), fJ = ld_global(gd.free_pos + J);
    const int nf1 = 6 * gd.n_free + 1;                       // row length of the free-node system
    const bool diag = (I == J);
    const int np = diag ? 2 * (N - 1) : 2;       // pairs summed
    const int nt = diag ? N - 1 : 2;             // pairs expanded with the adjoint (P, AX)
    const int kt0 = diag ? N - 1 : 0;            // pair index of expanded pair 0
    __shared__ double S[kMaxPairsPerBlock][kDenseFields];
    __shared__ double P[kMaxTgtPairs][36];
    __shared__ double X[kMaxTgtPairs][42];       // off-diagonal blocks: chunk sums
    __shared__ double AX[kMaxTgtPairs][12];      // A = T_i T_j^-1 of the expanded pairs (FP64)
    __shared__ double FS[kMaxFrames][44];        // oriented feature entries per neighbour
    __shared__ double ADJ[kMaxTgtPairs][36];     // the adjoints Ad of the expanded pairs
    double* const chunk = &X[0][0];

    // pair k: diagonal: k < N-1 (I, j), else (i, I); off-diagonal: (I, J), (J, I)
    auto pair_of = [&](int k, int& i, int& j) {
        if (!diag) {
            i = (k == 0) ? I : J;
            j = (k == 0) ? J : I;
        } else if (k < N - 1) {
            i = I;
            j = (k < I) ? k : k + 1;
        } else {
            const int kk = k - (N - 1);
            i = (kk < I) ? kk : kk + 1;
            j = I;
        }
    };

    // ---- phase 1: all global reads
    const int n_sum = diag ? np * kDenseFields : kAsmChunks * 2 * kDenseFields;
    const int n_ax = nt * 12;
    const int n_fs = diag ? N * 22 : 36;          // diagonal: two entries per task
    for (int task = threadIdx.x; task < n_sum + n_ax + n_fs; task += kAsmThreads) {
        if (task < n_sum) {
            int k, f, c;
            if (diag) {
                k = task / kDenseFields;
                f = task % kDenseFields;
                c = 0;
            } else {
                c = task / (2 * kDenseFields);
                k = (task / kDenseFields) & 1;
                f = task % kDenseFields;
            }
            int i, j;
            pair_of(k, i, j);
            const int p = pair_index(i, j, N);
            const int b0 = ld_global(gd.pair_base + p), b1 = ld_global(gd.pair_base + p + 1);
            if (diag) {
                S[k][f] = sum_records(gd.partials + f, b0, b1);
            } else {
                const int len = b1 - b0;
                const int t0 = b0 + (int)(((long long)len * c) / kAsmChunks);
                const int t1 = b0 + (int)(((long long)len * (c + 1)) / kAsmChunks);
                chunk[c * 2 * kDenseFields + k * kDenseFields + f] = sum_records(gd.partials + f, t0, t1);
            }
        } else if (task < n_sum + n_ax) {
            const int q = task - n_sum, pk = q / 12;
            int i, j;
            pair_of(kt0 + pk, i, j);
            AX[pk][q % 12] = ld_global(gd.xf64 + 12 * pair_index(i, j, N) + q % 12);
        } else {
            const int q = task - n_sum - n_ax;
            const int K = diag ? q / 22 : J, e0 = diag ? q % 22 : q;
            double v0 = 0.0, v1 = 0.0;
            const int s = (K != I) ? ld_global(gd.set_of + I * N + K) : -1;
            if (s >= 0) {
                // the entries of both orientations depend only on the set: all
                // loaded at once from computed (in-bounds) indices, the one of
                // node I chosen when the set's first node is known
                const double* F = gd.fpartials + (size_t)s * kFeatStride;
                // entry e of the neighbour's oriented block: H (36), g (6),
                // energy and count (once per set, with the first node)
                auto index = [&](int e, int o) {
                    if (!diag)
                        return sym12_index(e / 6 + o, e % 6 + 6 - o);
                    return (e < 36) ? sym12_index(o + e / 6, o + e % 6) : (e < 42) ? 78 + o + (e - 36) : 90 + (e - 42);
                };
                const int e1 = diag ? e0 + 22 : e0;
                const double a0 = ld_global(F + index(e0, 0)), b0 = ld_global(F + index(e0, 6));
                const double a1 = ld_global(F + index(e1, 0)), b1 = ld_global(F + index(e1, 6));
                // loaded after the entries
                const bool first = ld_global((const int*)(gd.fsets + s)) == I;
                v0 = first ? a0 : b0;                        // diagonal e0 < 22: an H entry
                v1 = first ? a1 : ((e1 < 42) ? b1 : 0.0);
            }
            FS[K][e0] = v0;
            if (diag)
                FS[K][e0 + 22] = v1;
        }
    }
    __syncthreads();
    if (status)
        return;
    // the adjoints of the expanded pairs, once (phases 2 and 3 read them),
    // and on off-diagonal blocks the chunk sums of the two pairs, in chunk
    // order, by other threads (the adjoints take the first 72 there)
    for (int task = threadIdx.x; task < nt * 36; task += kAsmThreads)
        ADJ[task / 36][task % 36] = adj(AX[task / 36], (task % 36) / 6, task % 6);
    if (!diag) {
        const int t = (int)threadIdx.x - kAsmThreads / 2;
        if (t >= 0 && t < 2 * kDenseFields) {
            const int k = t / kDenseFields, f = t % kDenseFields;
            double v = 0.0;
            for (int c = 0; c < kAsmChunks; ++c)
                v += chunk[c * 2 * kDenseFields + k * kDenseFields + f];
            S[k][f] = v;
        }
    }
    __syncthreads();
    // ---- phase 2: P = M Ad of the expanded pairs
    for (int task = threadIdx.x; task < nt * 36; task += kAsmThreads) {
        const int pk = task / 36, e = task % 36, a = e / 6, c = e % 6;
        const double* Sk = S[kt0 + pk];
        double v = 0.0;
        for (int l = 0; l < 6; ++l)
            v += sym6(Sk, a, l) * ADJ[pk][6 * l + c];
        P[pk][e] = v;
    }
    __syncthreads();
    const double lg = (double)gd.lambda_g, lf2 = 2.0 * (double)gd.lambda_f;
    if (!diag) {
        if (threadIdx.x < 36) {
            const int e = threadIdx.x, a = e / 6, c = e % 6;
            // -M Ad of (I, J) and -(M Ad)^T of (J, I)
            double h = lg * (-P[0][e] + -P[1][6 * c + a]);
            h += lf2 * FS[J][e];
            gd.Hm[(size_t)(6 * I + a) * n6 + 6 * J + c] = h;
            gd.Hm[(size_t)(6 * J + c) * n6 + 6 * I + a] = h;
            if (fI >= 0 && fJ >= 0) {
                gd.Hff[(size_t)(6 * fI + a) * nf1 + 6 * fJ + c] = h;
                gd.Hff[(size_t)(6 * fJ + c) * nf1 + 6 * fI + a] = h;
            }
        }
        return;
    }
    // ---- phase 3 (diagonal): target-role terms Ad^T M Ad (upper) and -Ad^T v
    for (int task = threadIdx.x; task < nt * 42; task += kAsmThreads) {
        const int pk = task / 42, e = task % 42;
        double v = 0.0;
        if (e < 36) {
            const int a = e / 6, c = e % 6;
            if (a <= c)
                for (int l = 0; l < 6; ++l)
                    v += ADJ[pk][6 * l + a] * P[pk][6 * l + c];
        } else {
            const int a = e - 36;
            for (int l = 0; l < 6; ++l)
                v -= ADJ[pk][6 * l + a] * S[kt0 + pk][21 + l];
        }
        X[pk][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < 42 && (threadIdx.x >= 36 || threadIdx.x / 6 <= threadIdx.x % 6)) {
        const int e = threadIdx.x;
        double h = 0.0;
        for (int k = 0; k < N - 1; ++k)   // source role: M and v
            h += (e < 36) ? sym6(S[k], e / 6, e % 6) : S[k][21 + (e - 36)];
        for (int pk = 0; pk < nt; ++pk)   // target role
            h += X[pk][e];
        h *= lg;
        double f = 0.0;
        for (int K = 0; K < N; ++K)
            f += FS[K][e];
        h += lf2 * f;
        if (e < 36) {
            gd.Hm[(size_t)(6 * I + e / 6) * n6 + 6 * I + e % 6] = h;
            gd.Hm[(size_t)(6 * I + e % 6) * n6 + 6 * I + e / 6] = h;
            if (fI >= 0) {
                gd.Hff[(size_t)(6 * fI + e / 6) * nf1 + 6 * fI + e % 6] = h;
                gd.Hff[(size_t)(6 * fI + e % 6) * nf1 + 6 * fI + e / 6] = h;
                // the largest positive diagonal entry of H_ff for the solve's
                // singularity tolerance: an atomic maximum of the bit patterns,
                // which order like the values for positive doubles
                if (e / 6 == e % 6 && h > 0.0)
                    atomicMax(gd.maxdiag, (unsigned long long)__double_as_longlong(h));
            }
        } else {
            gd.grad[6 * I + (e - 36)] = h;
            if (fI >= 0)
                gd.Hff[(size_t)(6 * fI + (e - 36)) * nf1 + nf1 - 1] = -h;
        }
    } else if (threadIdx.x == 64) {
        double Eg = 0.0, cg = 0.0, Ef = 0.0, cf = 0.0, rd = 0.0;
        for (int k = 0; k < N - 1; ++k) {
            Eg += S[k][27];
            cg += S[k][28];
            rd += S[k][29];
        }
        for (int K = 0; K < N; ++K) {
            Ef += FS[K][42];
            cf += FS[K][43];
        }
        gd.node_stats[kNodeStats * I + 0] = lg * Eg;
        gd.node_stats[kNodeStats * I + 1] = lf2 * Ef;
        gd.node_stats[kNodeStats * I + 2] = cg;
        gd.node_stats[kNodeStats * I + 3] = cf;
        gd.node_stats[kNodeStats * I + 4] = rd;
    }
}

// ------------------------------------------------------------ FP64 solve

constexpr int kSolveThreads = 512;

// Entry (r, c) of Exp(x) T for one node (x = [v; w], T its pose, 4x4
// row-major): row r of Exp(x) is [I + a K + b K^2 | (I + b K + c K^2) v]
// (Rodrigues and the left Jacobian, K = [w]x, K^2 = w w^T - |w|^2 I), row 3 is
// (0, 0, 0, 1); times column c of T.
__device__ __forceinline__ double se3_exp_entry(const double* __restrict__ xi, const double* __restrict__ T, int r,
                                                int c)
{
    const double t0 = T[c], t1 = T[4 + c], t2 = T[8 + c], t3 = T[12 + c];
    const double v0 = xi[0], v1 = xi[1], v2 = xi[2];
    const double w0 = xi[3], w1 = xi[4], w2 = xi[5];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    // a = sin t / t, b = (1 - cos t) / t^2, c = (t - sin t) / t^3
    double a, b, cc;
    if (th2 < 0.25) {
        // |t| < 0.5 (every Gauss-Newton step in practice): Taylor series in
        // t^2 through t^16, truncation below 1e-22; no cancellation
        const double x = th2;
        a = 1.0 - x * (1.0 / 6) * (1.0 - x * (1.0 / 20) * (1.0 - x * (1.0 / 42) * (1.0 - x * (1.0 / 72) *
            (1.0 - x * (1.0 / 110) * (1.0 - x * (1.0 / 156) * (1.0 - x * (1.0 / 210) * (1.0 - x * (1.0 / 272))))))));
        b = 0.5 * (1.0 - x * (1.0 / 12) * (1.0 - x * (1.0 / 30) * (1.0 - x * (1.0 / 56) * (1.0 - x * (1.0 / 90) *
            (1.0 - x * (1.0 / 132) * (1.0 - x * (1.0 / 182) * (1.0 - x * (1.0 / 240) * (1.0 - x * (1.0 / 306)))))))));
        cc = (1.0 / 6) * (1.0 - x * (1.0 / 20) * (1.0 - x * (1.0 / 42) * (1.0 - x * (1.0 / 72) * (1.0 - x * (1.0 / 110) *
             (1.0 - x * (1.0 / 156) * (1.0 - x * (1.0 / 210) * (1.0 - x * (1.0 / 272) * (1.0 - x * (1.0 / 342)))))))));
    } else {
        const double th = sqrt(th2), sn = sin(th), cs = cos(th);
        a = sn / th;
        b = (1.0 - cs) / th2;
        cc = (th - sn) / (th2 * th);
    }
    // row r of K and of K^2 (r < 3; row 3 is selected at the end)
    const double k0 = (r == 0) ? 0.0 : (r == 1) ? w2 : -w1;
    const double k1 = (r == 0) ? -w2 : (r == 1) ? 0.0 : w0;
    const double k2 = (r == 0) ? w1 : (r == 1) ? -w0 : 0.0;
    const double wr = (r == 0) ? w0 : (r == 1) ? w1 : w2;
    const double i0 = (r == 0) ? 1.0 : 0.0, i1 = (r == 1) ? 1.0 : 0.0, i2 = (r == 2) ? 1.0 : 0.0;
    const double q0 = wr * w0 - i0 * th2, q1 = wr * w1 - i1 * th2, q2 = wr * w2 - i2 * th2;
    const double e0 = i0 + a * k0 + b * q0, e1 = i1 + a * k1 + b * q1, e2 = i2 + a * k2 + b * q2;
    const double e3 = (i0 + b * k0 + cc * q0) * v0 + (i1 + b * k1 + cc * q1) * v1 + (i2 + b * k2 + cc * q2) * v2;
    const double out = e0 * t0 + e1 * t1 + e2 * t2 + e3 * t3;
    return (r == 3) ? t3 : out;
}

// Block barrier that orders LDS only: waits for the thread's own LDS (and
// scalar) accesses, not for its global stores, which nothing in the block
// reads back.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// A = T_i T_j^-1, B = T_j T_i^-1 per ordered pair (FP64, stored FP32 and
// FP64), and T^-1 = [R^T | -R^T t] per node (FP64), from the poses in LDS,
// one thread per row: rows 0 .. 3N-1 are the nodes' inverses, then six per
// pair (three of A, three of B).  Row r of T_a T_b^-1 is
// [R_a(r) R_b^T | t_a(r) + R_a(r) (-R_b^T t_b)].  No barrier: every row reads
// the poses only, so all rows of a thread load together.
constexpr int kTfPer = 3;   // rows per thread and pass

__device__ __forceinline__ double sel3(int r, double x0, double x1, double x2)
{
    return (r == 0) ? x0 : (r == 1) ? x1 : x2;
}

__device__ __forceinline__ void compute_transforms(const GraphDev& gd, const double* __restrict__ Ts)
{
    const int N = gd.n_frames;
    const int np = N * (N - 1);
    const int n_inv = 3 * N, total = n_inv + 6 * np;
    // pair p = i (N - 1) + jj: i from a float reciprocal (exact: the
    // fraction (jj + 1/2) / (N - 1) stays at least 1/62 from an integer)
    const float inv = 1.0f / (float)max(N - 1, 1);
    for (int base = 0; base < total; base += kTfPer * (int)blockDim.x) {
#pragma unroll
        for (int u = 0; u < kTfPer; ++u) {
            const int e = base + u * (int)blockDim.x + (int)threadIdx.x;
            if (e >= total)
                continue;
            const bool tinv = e < n_inv;
            const int f = tinv ? 0 : e - n_inv;
            const int p = f / 6, w = f - 6 * p;
            const int i = (int)(((float)p + 0.5f) * inv), jj = p - i * (N - 1), j = (jj < i) ? jj : jj + 1;
            const bool isA = w < 3;   // rows of A, then of B = T_j T_i^-1
            const int node = e / 3;
            const int r = tinv ? e - 3 * node : (isA ? w : w - 3);
            const double* Ta = Ts + 16 * (tinv ? node : (isA ? i : j));
            const double* Tb = Ts + 16 * (tinv ? node : (isA ? j : i));
            const double a0 = Ta[4 * r], a1 = Ta[4 * r + 1], a2 = Ta[4 * r + 2], a3 = Ta[4 * r + 3];
            double bm[12];
#pragma unroll
            for (int k = 0; k < 12; ++k)
                bm[k] = Tb[k];
            double su[3];   // -R_b^T t_b
#pragma unroll
            for (int k = 0; k < 3; ++k)
                su[k] = -(bm[k] * bm[3] + bm[4 + k] * bm[7] + bm[8 + k] * bm[11]);
            if (tinv) {
                double* dst = gd.tinv64 + 12 * node + 4 * r;
                st_global(dst, sel3(r, bm[0], bm[1], bm[2]));
                st_global(dst + 1, sel3(r, bm[4], bm[5], bm[6]));
                st_global(dst + 2, sel3(r, bm[8], bm[9], bm[10]));
                st_global(dst + 3, sel3(r, su[0], su[1], su[2]));
                continue;
            }
            double v[4];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                v[c] = a0 * bm[4 * c] + a1 * bm[4 * c + 1] + a2 * bm[4 * c + 2];
            v[3] = a3 + (a0 * su[0] + a1 * su[1] + a2 * su[2]);
            st_global_f4(gd.xf32 + 24 * p + (isA ? 0 : 12) + 4 * r, (float)v[0], (float)v[1], (float)v[2],
                         (float)v[3]);
            if (isA) {
                double* d64 = gd.xf64 + 12 * p + 4 * r;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    st_global(d64 + c, v[c]);
            }
        }
    }
}

// T_q <- Exp(x_q) T_q for the free nodes q (x: 6 per free node, Ts: the
// poses, both in LDS), 16 threads per node, one entry each; then the new
// poses in LDS and in the graph.  A node's 16 entries are read and written by
// 16 consecutive threads of one wavefront, whose writes wait for all their
// reads (each written value depends on the entry's whole column), so only
// the final barrier is needed.  Every thread of the block takes part; at
// least 256 threads.
__device__ __forceinline__ void update_poses(const GraphDev& gd, const double* __restrict__ xs, const int* __restrict__ sfree,
                             double* __restrict__ Ts)
{
    static_assert(16 * kMaxFrames <= 2 * 256, "pose update: two entries per thread");
    const int nf = gd.n_free;
    double tn[2];
    int at[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = threadIdx.x + u * blockDim.x;
        at[u] = -1;
        tn[u] = 0.0;
        if (e < 16 * nf) {
            const int q = e >> 4, r = (e >> 2) & 3, c = e & 3;
            const int node = sfree[q];
            tn[u] = se3_exp_entry(xs + 6 * q, Ts + 16 * node, r, c);
            at[u] = 16 * node + (e & 15);
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (at[u] >= 0) {
            Ts[at[u]] = tn[u];
            st_global(gd.poses + at[u], tn[u]);
        }
    lds_barrier();
}

__device__ double block_sum(double v, double* scratch)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
        scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w)
        s += scratch[w];
    return s;
}

__device__ double block_max(double v, double* scratch)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
        scratch[wave] = v;
    __syncthreads();
    double s = scratch[0];
    for (int w = 1; w < nw; ++w)
        s = fmax(s, scratch[w]);
    return s;
}

__device__ __forceinline__ double sym_tri(const double* L, int i, int j) { return (i >= j) ? L[tri(i, j)] : L[tri(j, i)]; }

// row/column of entry e of a packed lower triangle (e = i(i+1)/2 + j)
__device__ __forceinline__ void tri_rc(int e, int& i, int& j)
{
    int a = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((a + 1) * (a + 2) / 2 <= e)
        ++a;
    while (a * (a + 1) / 2 > e)
        --a;
    i = a;
    j = e - a * (a + 1) / 2;
}

// mode 1: start of an optimize (clear status, iteration counter; transforms).
// mode 0: one Gauss-Newton solve (Cholesky or PCG) + update + transforms for
// the next iteration.  Dynamic LDS: the packed lower triangle of the bordered
// matrix with -g_f^T as row n, then 2(n+1) + 4n doubles of vectors, then 16N
// poses.
__global__ __launch_bounds__(kSolveThreads) void solve_kernel(const GraphDev* __restrict__ gds, int mode)
{
    const GraphDev& gd = gds[blockIdx.x];
    const int N = gd.n_frames;
    const int n = 6 * gd.n_free, n6 = 6 * N;
    const int msize = (n + 1) * (n + 2) / 2;
    extern __shared__ double sm[];
    double* Lm = sm;
    double* piv = Lm + msize;   // n+1: Cholesky 1/sqrt(pivot); PCG diagonal
    double* xv = piv + 2 * (n + 1);
    double* rv = xv + n;
    double* pv = rv + n;
    double* qv = pv + n;
    double* Ts = qv + n;        // 16 N poses
    __shared__ double scratch[kSolveThreads / 64];
    __shared__ double ns[kMaxFrames * kNodeStats];
    __shared__ int sfree[kMaxFrames];
    const int tid = threadIdx.x;

    // mode 1 takes the poses from the pinned staging buffer of the host
    for (int k = tid; k < 16 * N; k += blockDim.x) {
        const double v = (mode == 1) ? gd.poses_in[k] : gd.poses[k];
        Ts[k] = v;
        if (mode == 1)
            gd.poses[k] = v;
    }
    if (mode == 1) {
        if (tid == 0) {
            *gd.status = 0;
            *gd.iters_done = 0;
            *gd.maxdiag = 0ull;
        }
        __syncthreads();
        compute_transforms(gd, Ts);
        return;
    }
    if (*gd.status)
        return;
    const int it = *gd.iters_done;
    for (int k = tid; k < kNodeStats * N; k += blockDim.x)
        ns[k] = gd.node_stats[k];
    for (int k = tid; k < gd.n_free; k += blockDim.x)
        sfree[k] = gd.free_ids[k];
    __syncthreads();
    for (int e = tid; e < msize; e += blockDim.x) {
        int a, b;
        tri_rc(e, a, b);
        double v = 0.0;
        if (a < n)
            v = gd.Hm[(size_t)(6 * sfree[a / 6] + a % 6) * n6 + 6 * sfree[b / 6] + b % 6];
        else if (b < n)
            v = -gd.grad[6 * sfree[b / 6] + b % 6];
        Lm[e] = v;
    }
    // iteration record: one field per thread, nodes summed in order
    if (tid < kNodeStats) {
        // record fields E_f, E_g, n_g, n_f, target reads from node fields
        // 1, 0, 2, 3, 4 (arithmetic, not a table in memory)
        const int src = (tid < 2) ? 1 - tid : tid;
        double s = 0.0;
        for (int k = 0; k < N; ++k)
            s += ns[kNodeStats * k + src];
        gd.iter_stats[kIterRecord * it + tid] = s;
    }
    if (n == 0) {                                   // every node fixed
        if (tid == 0)
            *gd.iters_done = it + 1;
        return;
    }
    __syncthreads();
    double md = 0.0;
    for (int a = tid; a < n; a += blockDim.x)
        md = fmax(md, Lm[tri(a, a)]);
    const double maxdiag = block_max(md, scratch);
    bool singular = !(maxdiag > 0.0);

    if (!singular && gd.solver == kSolverCholesky) {
        // right-looking Cholesky of the bordered matrix, one barrier per
        // column; the trailing block is updated by a 16 x 32 thread grid.
        // The border row ends as L^-1 (-g_f) scaled by the pivots.
        double* dv = piv;
        const int ty = tid >> 5, tx = tid & 31;
        for (int k = 0; k < n; ++k) {
            const double akk = Lm[tri(k, k)];
            if (!(akk > 1e-12 * maxdiag)) {
                singular = true;
                break;
            }
            const double inv = 1.0 / akk;
            for (int ii = k + 1 + ty; ii <= n; ii += kSolveThreads / 32) {
                const double lik = Lm[tri(ii, k)] * inv;
                const int jmax = (ii < n) ? ii : n - 1;
                for (int jj = k + 1 + tx; jj <= jmax; jj += 32)
                    Lm[tri(ii, jj)] -= lik * Lm[tri(jj, k)];
            }
            __syncthreads();
        }
        if (!singular) {
            for (int k = tid; k < n; k += blockDim.x)
                dv[k] = 1.0 / sqrt(Lm[tri(k, k)]);
            __syncthreads();
            // back substitution L^T x = y by one wave, y_k = border_k / d_k;
            // with unscaled columns, x_r = (y_r - t_r / d_r) / d_r where
            // t_r = sum over k > r of Lm(k, r) x_k
            if (tid < 64) {
                const int lane = tid;
                double t0 = 0.0, t1 = 0.0, t2 = 0.0;
                for (int k = n - 1; k >= 0; --k) {
                    const int mk = k >> 6, lk = k & 63;
                    const double tk = (mk == 0) ? t0 : (mk == 1) ? t1 : t2;
                    double xk = 0.0;
                    if (lane == lk)
                        xk = (Lm[tri(n, k)] * dv[k] - tk * dv[k]) * dv[k];
                    xk = __shfl(xk, lk);
                    if (lane < k) t0 += Lm[tri(k, lane)] * xk;
                    if (lane + 64 < k) t1 += Lm[tri(k, lane + 64)] * xk;
                    if (lane + 128 < k) t2 += Lm[tri(k, lane + 128)] * xk;
                    if (lane == lk)
                        xv[k] = xk;
                }
            }
            __syncthreads();
        }
    } else if (!singular) {
        // Jacobi-preconditioned conjugate gradients (the solver the paper names)
        double* dv = piv;
        const double* bv = Lm + tri(n, 0);
        for (int a = tid; a < n; a += blockDim.x) {
            dv[a] = Lm[tri(a, a)];
            xv[a] = 0.0;
            rv[a] = bv[a];
            pv[a] = bv[a] / dv[a];
        }
        __syncthreads();
        double rz = 0.0, bb = 0.0;
        for (int a = tid; a < n; a += blockDim.x) {
            rz += rv[a] * rv[a] / dv[a];
            bb += bv[a] * bv[a];
        }
        rz = block_sum(rz, scratch);
        bb = block_sum(bb, scratch);
        const double tol2 = gd.pcg_rel_tol * gd.pcg_rel_tol * bb;
        for (int iter = 0; iter < gd.pcg_max_iters; ++iter) {
            double pq = 0.0;
            for (int a = tid; a < n; a += blockDim.x) {
                double s = 0.0;
                for (int c = 0; c < n; ++c)
                    s += sym_tri(Lm, a, c) * pv[c];
                qv[a] = s;
                pq += pv[a] * s;
            }
            pq = block_sum(pq, scratch);
            if (!(pq > 0.0)) {
                singular = true;
                break;
            }
            const double alpha = rz / pq;
            double rr = 0.0, rzn = 0.0;
            for (int a = tid; a < n; a += blockDim.x) {
                xv[a] += alpha * pv[a];
                rv[a] -= alpha * qv[a];
                rr += rv[a] * rv[a];
                rzn += rv[a] * rv[a] / dv[a];
            }
            rr = block_sum(rr, scratch);
            rzn = block_sum(rzn, scratch);
            if (rr <= tol2)
                break;
            const double beta = rzn / rz;
            rz = rzn;
            for (int a = tid; a < n; a += blockDim.x)
                pv[a] = rv[a] / dv[a] + beta * pv[a];
            __syncthreads();
        }
        __syncthreads();
    }
    if (singular) {
        if (tid == 0)
            *gd.status |= kStatusSingular;
        return;
    }
    bool bad = false;
    for (int a = tid; a < n; a += blockDim.x)
        bad |= !isfinite(xv[a]);
    if (__syncthreads_or(bad)) {
        if (tid == 0)
            *gd.status |= kStatusNonFinite;
        return;
    }
    // T <- Exp(delta) T for the free nodes
    update_poses(gd, xv, sfree, Ts);
    if (tid == 0)
        *gd.iters_done = it + 1;
    compute_transforms(gd, Ts);
}

// ------------------------------------------------- Gauss-Jordan solve

typedef double gj_d4 __attribute__((ext_vector_type(4)));

// One Gauss-Newton solve by block Gauss-Jordan elimination without pivoting
// of the augmented system [H_ff | -g_f] (n = 6 x free nodes, a multiple of 3),
// with 3 x 3 pivot blocks.  H_ff is symmetric positive definite: the LU pivots
// of each pivot block are the Schur-complement pivots of the Cholesky
// factorisation, so the usual singularity test applies, and at the end the
// right-hand column holds the solution (no back substitution).  The rank-3
// update of each block step runs on the FP64 matrix cores.  The
// augmented n x (n+1) system is padded with zeros to NT x NT tiles of 16 x 16;
// wave w of the four owns the tiles (tr, tc) with (tr + tc) mod 4 = w, so the
// tile columns that elimination retires drop out of every wave alike.  A tile
// lives in one v_mfma_f64_16x16x4f64 accumulator: lane l holds entries
// (16 tr + 4 v + l / 16, 16 tc + l % 16), v < 4; the A operand of lane l is
// entry (l % 16, l / 16) of the 16 x 4 column block, the B operand entry
// (l / 16, l % 16) of the 4 x 16 row block (k = 3 is zero padding).  The
// trailing (not yet eliminated) part of the system stays symmetric, so the
// pivot rows' entries RP there are read from the published pivot columns; only
// their right-hand side is published apart.  Block step K: every lane inverts
// the pivot block D and forms its entry of R = D^-1 RP, and each live tile takes
// V <- V - (C - E) R in one matrix instruction, E holding the unit entries of
// the pivot rows: other rows get V - C R, the pivot rows RP - D R + R = R up to
// one rounding (no separate pass over them).  The owners of the next
// block's columns (and right-hand side) publish them to double-buffered LDS
// panels: one barrier per block step.  Then the update T <- Exp(x) T and the next
// iteration's transforms.
// one block of 256 threads: two pose entries, a node-statistics entry and a
// free-node id per thread at most
static_assert(16 * kMaxFrames <= 2 * 256 && kNodeStats * kMaxFrames <= 256 && kMaxFrames <= 256, "GJ prologue");

template <int NT>
__device__ __forceinline__ void gj_solve(const GraphDev& gd)
{
    constexpr int kS = (NT + 3) / 4;   // tile slots per tile row and wave
    constexpr int kM = 16 * NT;        // padded side
    const int N = gd.n_frames;
    const int n = 6 * gd.n_free;
    __shared__ double CP[2][3][kM];    // column panel v(i, 3K + m), by column
    __shared__ double RPn[2][3];       // right-hand side of the pivot rows v(3K + m, n)
    __shared__ double sink[256];       // publish target of the lanes that own nothing to publish
    __shared__ double xs[kM];
    __shared__ double Ts[16 * kMaxFrames];
    __shared__ double ns[kMaxFrames * kNodeStats];
    __shared__ int sfree[kMaxFrames];
    __shared__ int sflags;             // 1: singular pivot, 2: non-finite solution
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane >> 4, lc = lane & 15;
    // the owned tiles of [H_ff | -g_f], every load issued first, from clamped
    // addresses (padding applied once the system size is checked)
    gj_d4 acc[NT][kS];
    const double* __restrict__ Hff = gd.Hff;
#pragma unroll
    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
        for (int s = 0; s < kS; ++s) {
            const int tc = ((wave - tr) & 3) + 4 * s;
            const int j = 16 * tc + lc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * tr + 4 * v + lr;
                const bool in = tc < NT && i < n && j <= n;
                acc[tr][s][v] = Hff[in ? (size_t)i * (n + 1) + j : 0];
            }
        }
    // the poses, node statistics and free-node ids, loaded with the system
    double tv[2], nv = 0.0;
    int fv = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
        tv[u] = (tid + 256 * u < 16 * N) ? gd.poses[tid + 256 * u] : 0.0;
    if (tid < kNodeStats * N)
        nv = gd.node_stats[tid];
    if (tid < gd.n_free)
        fv = gd.free_ids[tid];
    const int it = *gd.iters_done;
    const int status = *gd.status;
    const double maxdiag = __longlong_as_double((long long)*gd.maxdiag);   // written by the assembly
    // both values in hand before the branch (the iteration counter is not
    // loaded after it, one memory round trip later)
    asm volatile("" ::"v"(it), "v"(status));
    if (status)
        return;
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (tid + 256 * u < 16 * N)
            Ts[tid + 256 * u] = tv[u];
    if (tid < kNodeStats * N)
        ns[tid] = nv;
    if (tid < gd.n_free)
        sfree[tid] = fv;
    if (tid == 0)
        sflags = 0;
    __syncthreads();
    if (tid < kNodeStats) {
        // record fields E_f, E_g, n_g, n_f, target reads from node fields
        // 1, 0, 2, 3, 4 (arithmetic, not a table in memory)
        const int src = (tid < 2) ? 1 - tid : tid;
        double s = 0.0;
        for (int k = 0; k < N; ++k)
            s += ns[kNodeStats * k + src];
        gd.iter_stats[kIterRecord * it + tid] = s;
    }
    if (n == 0) {
        if (tid == 0)
            *gd.iters_done = it + 1;
        return;
    }
    // zero padding and the first panels
#pragma unroll
    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
        for (int s = 0; s < kS; ++s) {
            const int tc = ((wave - tr) & 3) + 4 * s;
            const int j = 16 * tc + lc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * tr + 4 * v + lr;
                const bool in = tc < NT && i < n && j <= n;
                const double h = in ? acc[tr][s][v] : 0.0;
                acc[tr][s][v] = h;
                if (tc < NT && j < 3)
                    CP[0][j][i] = h;
                if (in && i < 3 && j == n)
                    RPn[0][i] = h;
            }
        }
    __syncthreads();   // padding and first panels
    const double tol = 1e-12 * maxdiag;
    bool singular = !(maxdiag > 0.0);
    // the lane's row r of each pivot block's inverse (the padding row lr = 3
    // computes row 0 and drops it) and the other two columns, cyclically
    const int r0 = (lr < 3) ? lr : 0;
    const int r1 = (r0 == 2) ? 0 : r0 + 1, r2 = (r0 == 0) ? 2 : r0 - 1;
    for (int K = 0; 3 * K < n; ++K) {
        const int bf = K & 1, c0 = 3 * K, c1 = c0 + 3;
        // pivot block and row panel from the column panel: the trailing part of
        // the system stays symmetric under elimination, so row c0 + m of it is
        // column c0 + m; only the right-hand side of the pivot rows is separate.
        // Pivot block D, entry (l, m) = v(c0 + l, c0 + m) at CP[m][c0 + l]:
        // the lane reads its columns r0, r1, r2
        double d0[3], d1[3], d2[3];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            d0[l] = CP[bf][r0][c0 + l];
            d1[l] = CP[bf][r1][c0 + l];
            d2[l] = CP[bf][r2][c0 + l];
        }
        // operands of every owned tile, read together: A from the column panel,
        // the three panel entries of the lane's column for B
        double ca[NT], rb[NT][kS][3];
#pragma unroll
        for (int tr = 0; tr < NT; ++tr) {
            ca[tr] = CP[bf][lr < 3 ? lr : 0][16 * tr + lc];
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                const int tc = ((wave - tr) & 3) + 4 * s;
                const int j = 16 * (tc < NT ? tc : 0) + lc;
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    rb[tr][s][m] = (j == n) ? RPn[bf][m] : CP[bf][m][j];
            }
        }
        // row r0 of D^-1 = cofactors (m, r0) / det, det expanded along column
        // r0 (no full inverse per lane); 1/det by the hardware reciprocal and
        // two Newton steps.  cof(m, r0) = D(m+1, r1) D(m+2, r2) - D(m+1, r2) D(m+2, r1)
        double cf[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
            cf[m] = d1[m1] * d2[m2] - d2[m1] * d1[m2];
        }
        const double det = d0[0] * cf[0] + d0[1] * cf[1] + d0[2] * cf[2];
        double id = __builtin_amdgcn_rcp(det);
        id = fma(id, fma(-det, id, 1.0), id);
        id = fma(id, fma(-det, id, 1.0), id);
        // the LU (Schur) pivots D00, c22 / D00 and det / c22 of an SPD block all
        // exceed tol (tested by products); lanes of row 2 hold D00 = d1[0] and
        // c22 = cf[2]
        if (lr == 2)
            singular |= !((d1[0] > tol) && (cf[2] > tol * d1[0]) && (det > tol * cf[2]));
        double Dl[3];
#pragma unroll
        for (int m = 0; m < 3; ++m)
            Dl[m] = (lr < 3) ? cf[m] * id : 0.0;
        // A operand: -(C - E)(16 tr + lc, lr), E the unit entries of the pivot
        // rows, so the update leaves R in the pivot rows: V - C R + E R
        double a[NT];
#pragma unroll
        for (int tr = 0; tr < NT; ++tr) {
            const int ia = 16 * tr + lc;
            a[tr] = (lr < 3) ? ((ia == c0 + lr ? 1.0 : 0.0) - ca[tr]) : 0.0;
        }
#pragma unroll
        for (int tr = 0; tr < NT; ++tr)
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                const int tc = ((wave - tr) & 3) + 4 * s;
                if (tc >= NT || 16 * tc + 15 < c1)   // not owned, or every column eliminated (uniform)
                    continue;
                const double b = fma(Dl[0], rb[tr][s][0], fma(Dl[1], rb[tr][s][1], Dl[2] * rb[tr][s][2]));
                acc[tr][s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[tr], b, acc[tr][s], 0, 0, 0);
            }
        // publish the next block's three columns, and the right-hand side of its
        // rows (their owners only)
        if (c1 < n) {
#pragma unroll
            for (int tr = 0; tr < NT; ++tr)
#pragma unroll
                for (int s = 0; s < kS; ++s) {
                    const int tc = ((wave - tr) & 3) + 4 * s;
                    if (tc >= NT || 16 * tc + 15 < c1)
                        continue;
                    const int j = 16 * tc + lc;
                    const int m = j - c1;
                    if (tc == (c1 >> 4) || tc == ((c1 + 2) >> 4)) {   // uniform: the tile holds next columns
                        // every lane writes: the owners of columns c1.. to the
                        // panel, the others to their sink slot
                        const bool own = m >= 0 && m < 3;
                        double* dst = own ? &CP[bf ^ 1][own ? m : 0][16 * tr + lr] : &sink[tid];
                        const int step = own ? 4 : 0;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            dst[step * v] = acc[tr][s][v];
                    }
                    if (j == n && 16 * tr <= c1 + 2 && c1 < 16 * tr + 16) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int d = 16 * tr + 4 * v + lr - c1;
                            if (d >= 0 && d < 3)
                                RPn[bf ^ 1][d] = acc[tr][s][v];
                        }
                    }
                }
        }
        __syncthreads();
    }
    // the right-hand column holds the solution; one barrier publishes it with
    // the singularity and finiteness flags
    bool bad = false;
#pragma unroll
    for (int tr = 0; tr < NT; ++tr)
#pragma unroll
        for (int s = 0; s < kS; ++s) {
            const int tc = ((wave - tr) & 3) + 4 * s;
            if (tc < NT && 16 * tc + lc == n) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * tr + 4 * v + lr;
                    if (i < n) {
                        xs[i] = acc[tr][s][v];
                        bad |= !isfinite(acc[tr][s][v]);
                    }
                }
            }
        }
    if (singular || bad)
        atomicOr(&sflags, (singular ? 1 : 0) | (bad ? 2 : 0));
    __syncthreads();
    const int flags = sflags;
    // every thread has used the diagonal maximum by now: cleared for the
    // next iteration's assembly
    if (tid == 0)
        *gd.maxdiag = 0ull;
    if (flags) {
        if (tid == 0)
            *gd.status |= (flags & 1) ? kStatusSingular : kStatusNonFinite;
        return;
    }
    update_poses(gd, xs, sfree, Ts);
    if (tid == 0)
        *gd.iters_done = it + 1;
    compute_transforms(gd, Ts);
}

// ------------------------------------------------- single-wavefront block LDL^T solve

// v of lane L (a constant), in scalar registers
__device__ __forceinline__ double lane_f64(double v, int L)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, L);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double rcp_f64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// One Gauss-Newton solve on one wavefront: block LDL^T factorisation without
// pivoting of the symmetric positive definite H_ff with 4 x 4 pivot blocks,
// the right-hand side -g_f carried as the last column of the padded system,
// then block back substitution.  Only the upper NT(NT+1)/2 tiles of 16 x 16
// are kept, each in one v_mfma_f64_16x16x4f64 accumulator in registers (lane l
// holds entries (16 I + 4 v + l / 16, 16 J + l % 16), v < 4).  At pivot rows
// k..k+3 (k = 16 J + 4 v) the row panel P = rows k..k+3 sits in register v of
// tiles (J, I >= J) in exactly the matrix cores' operand layout: lane l holds
// P(l / 16, 16 I + l % 16), which is the A operand entry (row l % 16, column
// l / 16) of the 16 x 4 block P^T of tile row I (the trailing system is
// symmetric) and the B operand entry of the 4 x 16 block of tile column I.  So
// the rank-4 update of the trailing system, V <- V - P^T D^-1 P, is one matrix
// instruction per upper tile, with A = -P^T (rows at or above the pivot rows
// zeroed, which leaves them unchanged) and B = R = D^-1 P (the lane's row of
// D^-1 times P's column, gathered from the four rows of lanes).  R replaces P
// in register v, for the back substitution x_k = R(., rhs) - R(., > k) x.
// D^-1 comes from the 2 x 2 blocks of D (two Schur steps) in every lane, from
// D's entries read into scalar registers.  Every size runs the same 4 NT - 1
// block steps (rows 0 .. 16 NT - 5, n <= 16 NT - 4): rows n and up to there are
// decoupled padding rows with a diagonal equal to the largest diagonal entry of
// H_ff, so the steps are straight-line code the compiler can overlap (the
// next step's pivot work with this step's matrix instructions).  The
// right-hand side is column 16 NT - 1.  No barrier and no shared memory until
// the solution is written; the other three waves load the poses and node
// statistics meanwhile.  Then T <- Exp(x) T and the next iteration's
// transforms, as the other solves.
constexpr int kLdlStride = 66;   // doubles per row of the R rows in LDS (16-byte aligned rows)

template <int NT>
__device__ __forceinline__ void ldl_solve(const GraphDev& gd, double* __restrict__ Rl)
{
    constexpr int kM = 16 * NT;          // padded side; the right-hand side is column kM - 1
    constexpr int kSteps = 4 * NT - 1;   // pivot rows 0 .. kM - 5
    static_assert(kM + 2 <= kLdlStride, "LDL row stride");
    const int N = gd.n_frames;
    const int n = 6 * gd.n_free;
    __shared__ double xs[kM];
    __shared__ double Ts[16 * kMaxFrames];
    __shared__ int sfree[kMaxFrames];
    __shared__ int sflags;   // 1: singular pivot, 2: non-finite solution
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane >> 4, c = lane & 15;
    const int it = ld_global(gd.iters_done);
    const int status = ld_global(gd.status);
    // written by the assembly
    const double maxdiag = __longlong_as_double((long long)ld_global(gd.maxdiag));
    if (wave == 0) {
        // the upper tiles of the padded system, every load issued first from
        // a clamped (always valid) address; padding pivots equal the largest
        // diagonal entry (decoupled rows that pass the pivot test at any scale)
        const double pad = (maxdiag > 0.0) ? maxdiag : 1.0;
        const int ilast = (n > 0) ? n - 1 : 0;
        gj_d4 t[NT][NT];
        const double* __restrict__ Hff = gd.Hff;
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int K = I; K < NT; ++K)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * I + 4 * v + m;
                    const int j = 16 * K + c;
                    const int col = (j == kM - 1) ? n : min(j, n);
                    t[I][K][v] = ld_global(Hff + (min(i, ilast) * (n + 1) + col));
                }
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
            for (int K = I; K < NT; ++K)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * I + 4 * v + m;
                    const int j = 16 * K + c;
                    const bool in = i < n && (j == kM - 1 || j < n);
                    t[I][K][v] = in ? t[I][K][v] : ((i == j && i < kM - 4) ? pad : 0.0);
                }
        if (status == 0 && n > 0 && n <= kM - 4) {
            const double tol = 1e-12 * maxdiag;
            int singular = (maxdiag > 0.0) ? 0 : 1;
            const bool odd = (m & 1) != 0, hi2 = (m & 2) != 0, mid = (m == 1) || (m == 2);
#pragma unroll
            for (int s = 0; s < kSteps; ++s) {
                const int J = s >> 2, v = s & 3;
                // pivot block D (rows and columns k..k+3, k = 16 J + 4 v) into scalar registers
                const double d00 = lane_f64(t[J][J][v], 4 * v + 0);
                const double d01 = lane_f64(t[J][J][v], 4 * v + 1);
                const double d02 = lane_f64(t[J][J][v], 4 * v + 2);
                const double d03 = lane_f64(t[J][J][v], 4 * v + 3);
                const double d11 = lane_f64(t[J][J][v], 16 + 4 * v + 1);
                const double d12 = lane_f64(t[J][J][v], 16 + 4 * v + 2);
                const double d13 = lane_f64(t[J][J][v], 16 + 4 * v + 3);
                const double d22 = lane_f64(t[J][J][v], 32 + 4 * v + 2);
                const double d23 = lane_f64(t[J][J][v], 32 + 4 * v + 3);
                const double d33 = lane_f64(t[J][J][v], 48 + 4 * v + 3);
                // the row panel's four rows of each column, from the other rows of lanes
                double x1[NT], x2[NT], x3[NT];
#pragma unroll
                for (int I = J; I < NT; ++I) {
                    x1[I] = __shfl_xor(t[J][I][v], 16);
                    x2[I] = __shfl_xor(t[J][I][v], 32);
                    x3[I] = __shfl_xor(t[J][I][v], 48);
                }
                // D^-1 by two 2 x 2 Schur steps: D = [[P, Q], [Q^T, S]],
                // D^-1 = [[F, E], [E^T, Z]], Z = (S - Q^T P^-1 Q)^-1,
                // E = -P^-1 Q Z, F = P^-1 - E (P^-1 Q)^T
                const double detP = fma(d00, d11, -d01 * d01);
                const double ip = rcp_f64(detP);
                const double p00 = d11 * ip, p01 = -d01 * ip, p11 = d00 * ip;
                const double w00 = fma(p00, d02, p01 * d12), w01 = fma(p00, d03, p01 * d13);
                const double w10 = fma(p01, d02, p11 * d12), w11 = fma(p01, d03, p11 * d13);
                const double s00 = d22 - fma(d02, w00, d12 * w10);
                const double s01 = d23 - fma(d02, w01, d12 * w11);
                const double s11 = d33 - fma(d03, w01, d13 * w11);
                const double detS = fma(s00, s11, -s01 * s01);
                const double is = rcp_f64(detS);
                const double z00 = s11 * is, z01 = -s01 * is, z11 = s00 * is;
                const double e00 = -fma(w00, z00, w01 * z01), e01 = -fma(w00, z01, w01 * z11);
                const double e10 = -fma(w10, z00, w11 * z01), e11 = -fma(w10, z01, w11 * z11);
                const double f00 = p00 - fma(e00, w00, e01 * w01);
                const double f01 = p01 - fma(e00, w10, e01 * w11);
                const double f11 = p11 - fma(e10, w10, e11 * w11);
                // the scalar pivots d00, detP / d00, s00, detS / s00 all exceed
                // tol; tested here, beside the step's matrix instructions (the
                // empty asm keeps the test from sinking to the end of the loop,
                // where the 15 steps' tests would run one after another)
                singular |= ((d00 > tol) && (detP > tol * d00) && (s00 > tol) && (detS > tol * s00)) ? 0 : 1;
                asm volatile("" : "+v"(singular));
                // row m of D^-1 at columns m, m ^ 1, m ^ 2, m ^ 3 (D^-1 symmetric)
                const double dq0 = hi2 ? (odd ? z11 : z00) : (odd ? f11 : f00);
                const double dq1 = hi2 ? z01 : f01;
                const double dq2 = odd ? e11 : e00;
                const double dq3 = mid ? e10 : e01;
                // operands: A = -P^T, B = R = D^-1 P; the pivot rows' own
                // columns and those left of them give zero (masked)
                double a[NT], b[NT];
#pragma unroll
                for (int I = J; I < NT; ++I) {
                    const double p = t[J][I][v];
                    const bool left = (I == J) && (c <= 4 * v + 3);
                    const bool rhs = (I == NT - 1) && (c == 15);
                    const double r = fma(dq0, p, fma(dq1, x1[I], fma(dq2, x2[I], dq3 * x3[I])));
                    a[I] = (left || rhs) ? 0.0 : -p;
                    b[I] = left ? 0.0 : r;
                    t[J][I][v] = b[I];
                    // the row panel of R, row-major in LDS, for the back substitution
                    Rl[(16 * J + 4 * v + m) * kLdlStride + 16 * I + c] = b[I];
                }
                // the next pivot rows' tiles first
                const int Jn = (v < 3) ? J : J + 1;
#pragma unroll
                for (int I = Jn; I < NT; ++I)
                    t[Jn][I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[Jn], b[I], t[Jn][I], 0, 0, 0);
#pragma unroll
                for (int Ir = J; Ir < NT; ++Ir) {
                    if (Ir == Jn)
                        continue;
#pragma unroll
                    for (int I = Ir; I < NT; ++I)
                        t[Ir][I] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[Ir], b[I], t[Ir][I], 0, 0, 0);
                }
            }
            // back substitution, one row per lane: lane i loads row i of R
            // (its own 4 x 4 block and everything left of it are zero or never
            // read), y starts as R(i, rhs) = (D^-1 z)_i; going up the blocks,
            // the block's four x are the y of its lanes (every later block
            // already subtracted), read into scalar registers, and every lane
            // subtracts R(i, block) x
            double Rrow[kM];
            {
                const double* __restrict__ src = Rl + min(lane, kM - 5) * kLdlStride;
#pragma unroll
                for (int j = 0; j < kM; j += 2) {
                    const double2 w = *(const double2*)(src + j);
                    Rrow[j] = w.x;
                    Rrow[j + 1] = w.y;
                }
            }
            double y = Rrow[kM - 1], xf = 0.0;
#pragma unroll
            for (int s = kSteps - 1; s >= 0; --s) {
                const int k = 4 * s;
                const double x0 = lane_f64(y, k), x1 = lane_f64(y, k + 1);
                const double x2 = lane_f64(y, k + 2), x3 = lane_f64(y, k + 3);
                xf = (lane >= k && lane < k + 4) ? y : xf;
                y -= fma(Rrow[k], x0, Rrow[k + 1] * x1) + fma(Rrow[k + 2], x2, Rrow[k + 3] * x3);
            }
            bool bad = false;
            if (lane < n) {
                xs[lane] = xf;
                bad = !isfinite(xf);
            }
            bad = __any(bad);
            if (lane == 0)
                sflags = (singular ? 1 : 0) | (bad ? 2 : 0);
        } else if (lane == 0) {
            // nothing to solve (every node fixed); a system too large for the
            // tiles is refused on the host
            sflags = (n > 0) ? 1 : 0;
        }
    } else {
        // the poses, the free-node ids and this iteration's statistics
        // (record fields E_f, E_g, n_g, n_f, target reads from node fields
        // 1, 0, 2, 3, 4), while wave 0 solves
        const int u = tid - 64;
        double tv[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            tv[r] = (u + 192 * r < 16 * N) ? ld_global(gd.poses + u + 192 * r) : 0.0;
        const int fv = (u < gd.n_free) ? ld_global(gd.free_ids + u) : 0;
        if (u < kNodeStats && status == 0) {
            const int src = (u < 2) ? 1 - u : u;
            double s = 0.0;
            for (int k = 0; k < N; ++k)
                s += ld_global(gd.node_stats + kNodeStats * k + src);
            st_global(gd.iter_stats + kIterRecord * it + u, s);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
            if (u + 192 * r < 16 * N)
                Ts[u + 192 * r] = tv[r];
        if (u < gd.n_free)
            sfree[u] = fv;
    }
    if (status)
        return;   // uniform: every wave read the same status
    lds_barrier();
    const int flags = sflags;
    // every thread has used the diagonal maximum by now: cleared for the
    // next iteration's assembly
    if (tid == 0)
        st_global(gd.maxdiag, 0ull);
    if (n == 0) {
        if (tid == 0)
            st_global(gd.iters_done, it + 1);
        return;
    }
    if (flags) {
        if (tid == 0)
            st_global(gd.status, status | ((flags & 1) ? kStatusSingular : kStatusNonFinite));
        return;
    }
    update_poses(gd, xs, sfree, Ts);
    if (tid == 0)
        st_global(gd.iters_done, it + 1);
    compute_transforms(gd, Ts);
}

// ------------------------------------------------- matrix-free PCG

constexpr int kMfThreads = 256;

// Dynamic LDS of the matrix-free solve (doubles): per ordered pair the Gram
// block M = sum w J_i^T J_i (21), the pair transform A (12) and a product slot
// (12); per feature set its 12 x 12 block (78) and a product slot (12); six
// 6N vectors; a reduction scratch.
__host__ __device__ inline size_t mf_lds_doubles(int n_frames, int n_sets)
{
    const size_t P = (size_t)n_frames * (n_frames - 1);
    return 45 * P + 90 * (size_t)n_sets + 6 * 6 * (size_t)n_frames + 16;
}

// (Ad^T y) for the adjoint of A = [R | t] (xi = [v; w]): [R^T y_v; R^T (y_w - t x y_v)]
__device__ __forceinline__ void adjT_apply(const double* __restrict__ A, const double* y, double* out)
{
    const double t0 = A[3], t1 = A[7], t2 = A[11];
    const double w0 = y[3] - (t1 * y[2] - t2 * y[1]);
    const double w1 = y[4] - (t2 * y[0] - t0 * y[2]);
    const double w2 = y[5] - (t0 * y[1] - t1 * y[0]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out[c] = A[c] * y[0] + A[4 + c] * y[1] + A[8 + c] * y[2];
        out[3 + c] = A[c] * w0 + A[4 + c] * w1 + A[8 + c] * w2;
    }
}

// (Ad x) for the adjoint of A: [R x_v + t x (R x_w); R x_w]
__device__ __forceinline__ void adj_apply(const double* __restrict__ A, const double* x, double* out)
{
    double rw[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        rw[r] = A[4 * r] * x[3] + A[4 * r + 1] * x[4] + A[4 * r + 2] * x[5];
    const double t0 = A[3], t1 = A[7], t2 = A[11];
    out[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2] + (t1 * rw[2] - t2 * rw[1]);
    out[1] = A[4] * x[0] + A[5] * x[1] + A[6] * x[2] + (t2 * rw[0] - t0 * rw[2]);
    out[2] = A[8] * x[0] + A[9] * x[1] + A[10] * x[2] + (t0 * rw[1] - t1 * rw[0]);
    out[3] = rw[0];
    out[4] = rw[1];
    out[5] = rw[2];
}

// Sum of two values over the block (fixed order over the waves); every thread
// gets both.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red)
{
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    lds_barrier();
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    lds_barrier();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < kMfThreads / 64; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
}

// One Gauss-Newton step by preconditioned conjugate gradients on the normal
// equations without forming them (the solver Sec. IV-D names: PCG with the
// preconditioner diag(J^T W J)).  The association pass left per work item the
// sums of w J_i^T J_i, w r J_i, energy, count and target reads; this block
// reduces them per ordered pair (fixed order) to M and v.  A dense residual
// row's Jacobian is [J_i | -J_i Ad_A], so J^T W J p = sum over pairs of
// [M u; -Ad^T M u] with u = p_i - Ad_A p_j; the feature term (Eq. 2) adds each
// set's 12 x 12 block times [p_i; p_j] (both orderings of Eq. 1: factor 2).
// Gradient and preconditioner come from the same pieces.  x = 0 start,
// stopped at |r| <= pcg_rel_tol |b| or pcg_max_iters; a non-positive curvature
// p^T H p is a singular system.  Then T <- Exp(x) T and the next iteration's
// transforms, as the other solves.  One block of 256 threads per graph; the
// per-pair data lives in LDS (mf_lds_doubles).
__global__ __launch_bounds__(kMfThreads) void mf_pcg_kernel(const GraphDev* __restrict__ gds)
{
    const GraphDev& gd = gds[blockIdx.x];
    const int N = gd.n_frames, P = N * (N - 1), NS = gd.n_sets, n6 = 6 * N;
    extern __shared__ double sm[];
    double* Mg = sm;              // P x 21
    double* Ax = Mg + 21 * P;     // P x 12
    double* Yp = Ax + 12 * P;     // P x 12: M u, then -Ad^T M u
    double* Fb = Yp + 12 * P;     // NS x 78
    double* Fy = Fb + 78 * NS;    // NS x 12
    double* xv = Fy + 12 * NS;    // six 6N vectors
    double* rv = xv + n6;
    double* zv = rv + n6;
    double* pv = zv + n6;
    double* dg = pv + n6;
    double* gv = dg + n6;
    double* red = gv + n6;        // 16
    __shared__ double Ts[16 * kMaxFrames];
    __shared__ double xs[6 * kMaxFrames];
    __shared__ int sfree[kMaxFrames];
    __shared__ int sflags;
    const int tid = threadIdx.x;
    const int status = *gd.status;
    const int it = *gd.iters_done;
    if (status)
        return;
    // per-pair sums of the association records, transforms, feature blocks
    for (int task = tid; task < 30 * P; task += kMfThreads) {
        const int p = task / 30, f = task - 30 * p;
        const double v = sum_records(gd.partials + f, gd.pair_base[p], gd.pair_base[p + 1]);
        if (f < 21)
            Mg[21 * p + f] = v;
        else
            Yp[12 * p + (f - 21)] = v;   // v (6), energy, count, target reads
    }
    for (int task = tid; task < 12 * P; task += kMfThreads)
        Ax[task] = gd.xf64[task];
    for (int task = tid; task < 78 * NS; task += kMfThreads)
        Fb[task] = gd.fpartials[(size_t)(task / 78) * kFeatStride + task % 78];
    for (int task = tid; task < 16 * N; task += kMfThreads)
        Ts[task] = gd.poses[task];
    if (tid < gd.n_free)
        sfree[tid] = gd.free_ids[tid];
    if (tid == 0)
        sflags = 0;
    __syncthreads();
    const double lg = (double)gd.lambda_g, lf2 = 2.0 * (double)gd.lambda_f;
    // iteration record: E_f, E_g, n_g, n_f, target reads
    if (tid < kNodeStats) {
        double s = 0.0;
        if (tid == 0 || tid == 3)
            for (int q = 0; q < NS; ++q)
                s += gd.fpartials[(size_t)q * kFeatStride + (tid == 0 ? 90 : 91)];
        else
            for (int p = 0; p < P; ++p)
                s += Yp[12 * p + (tid == 1 ? 6 : tid == 2 ? 7 : 8)];
        gd.iter_stats[kIterRecord * it + tid] = (tid == 0) ? lf2 * s : (tid == 1) ? lg * s : s;
    }
    // gradient and the diagonal of J^T W J per node entry (fixed order)
    const int n = 6 * gd.n_free;
    for (int e = tid; e < n6; e += kMfThreads) {
        const int k = e / 6, c = e - 6 * k;
        double g = 0.0, d = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == k)
                continue;
            const int ps = pair_index(k, j, N), pt = pair_index(j, k, N);   // k as source, as target
            g += Yp[12 * ps + c];
            d += sym6(Mg + 21 * ps, c, c);
            // target role: -Ad^T v and (Ad^T M Ad)_cc = a^T M a, a = column c of Ad
            double y[6], tv[6], col[6], ec[6];
#pragma unroll
            for (int l = 0; l < 6; ++l) {
                y[l] = Yp[12 * pt + l];
                ec[l] = (l == c) ? 1.0 : 0.0;
            }
            adjT_apply(Ax + 12 * pt, y, tv);
            g -= tv[c];
            adj_apply(Ax + 12 * pt, ec, col);
            double q = 0.0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                double ma = 0.0;
#pragma unroll
                for (int b = 0; b < 6; ++b)
                    ma += sym6(Mg + 21 * pt, a, b) * col[b];
                q += col[a] * ma;
            }
            d += q;
        }
        g *= lg;
        d *= lg;
        for (int j = 0; j < N; ++j) {
            const int q = (j != k) ? gd.set_of[k * N + j] : -1;
            if (q < 0)
                continue;
            const int o = (gd.fsets[q].x == k) ? 0 : 6;
            g += lf2 * gd.fpartials[(size_t)q * kFeatStride + 78 + o + c];
            d += lf2 * Fb[78 * q + sym12_index(o + c, o + c)];
        }
        const bool fr = gd.free_pos[k] >= 0;
        gv[e] = g;
        dg[e] = d;
        xv[e] = 0.0;
        rv[e] = fr ? -g : 0.0;
        zv[e] = (fr && d > 0.0) ? -g / d : 0.0;
        pv[e] = zv[e];
    }
    double bb = 0.0, rz = 0.0, nbad = 0.0, unused = 0.0;
    for (int e = tid; e < n6; e += kMfThreads) {
        bb += rv[e] * rv[e];
        rz += rv[e] * zv[e];
        nbad += (gd.free_pos[e / 6] >= 0 && !(dg[e] > 0.0)) ? 1.0 : 0.0;
    }
    block_sum2(bb, rz, red);
    block_sum2(nbad, unused, red);
    bool singular = nbad > 0.0;   // a free unknown without curvature
    int iters = 0;
    if (n > 0 && bb > 0.0 && !singular) {
        const double tol2 = gd.pcg_rel_tol * gd.pcg_rel_tol * bb;
        for (iters = 0; iters < gd.pcg_max_iters;) {
            // q = J^T W J p: per pair M u and -Ad^T M u, per set F [p_i; p_j]
            for (int p = tid; p < P + NS; p += kMfThreads) {
                if (p < P) {
                    const int i = p / (N - 1), jj = p - i * (N - 1), j = (jj < i) ? jj : jj + 1;
                    double pj[6], ap[6], u[6], y[6], w[6];
#pragma unroll
                    for (int l = 0; l < 6; ++l)
                        pj[l] = pv[6 * j + l];
                    adj_apply(Ax + 12 * p, pj, ap);
#pragma unroll
                    for (int l = 0; l < 6; ++l)
                        u[l] = pv[6 * i + l] - ap[l];
#pragma unroll
                    for (int a = 0; a < 6; ++a) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < 6; ++b)
                            s += sym6(Mg + 21 * p, a, b) * u[b];
                        y[a] = s;
                    }
                    adjT_apply(Ax + 12 * p, y, w);
#pragma unroll
                    for (int l = 0; l < 6; ++l) {
                        Yp[12 * p + l] = y[l];
                        Yp[12 * p + 6 + l] = -w[l];
                    }
                } else {
                    const int q = p - P;
                    const int4 fs = gd.fsets[q];
                    double v[12];
#pragma unroll
                    for (int l = 0; l < 6; ++l) {
                        v[l] = pv[6 * fs.x + l];
                        v[6 + l] = pv[6 * fs.y + l];
                    }
#pragma unroll
                    for (int a = 0; a < 12; ++a) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < 12; ++b)
                            s += Fb[78 * q + sym12_index(a, b)] * v[b];
                        Fy[12 * q + a] = s;
                    }
                }
            }
            lds_barrier();
            double pq = 0.0, dummy = 0.0;
            double qv[(6 * kMaxFrames + kMfThreads - 1) / kMfThreads];
#pragma unroll
            for (int u = 0; u < (6 * kMaxFrames + kMfThreads - 1) / kMfThreads; ++u) {
                const int e = tid + u * kMfThreads;
                qv[u] = 0.0;
                if (e >= n6)
                    continue;
                const int k = e / 6, c = e - 6 * k;
                if (gd.free_pos[k] < 0)
                    continue;
                double h = 0.0;
                for (int j = 0; j < N; ++j)
                    if (j != k)
                        h += Yp[12 * pair_index(k, j, N) + c] + Yp[12 * pair_index(j, k, N) + 6 + c];
                h *= lg;
                double f = 0.0;
                for (int j = 0; j < N; ++j) {
                    const int q = (j != k) ? gd.set_of[k * N + j] : -1;
                    if (q >= 0)
                        f += Fy[12 * q + ((gd.fsets[q].x == k) ? 0 : 6) + c];
                }
                qv[u] = h + lf2 * f;
                pq += pv[e] * qv[u];
            }
            block_sum2(pq, dummy, red);
            if (!(pq > 0.0)) {
                singular = true;
                break;
            }
            const double alpha = rz / pq;
            double rr = 0.0, rzn = 0.0;
#pragma unroll
            for (int u = 0; u < (6 * kMaxFrames + kMfThreads - 1) / kMfThreads; ++u) {
                const int e = tid + u * kMfThreads;
                if (e >= n6 || gd.free_pos[e / 6] < 0)
                    continue;
                xv[e] += alpha * pv[e];
                rv[e] -= alpha * qv[u];
                zv[e] = rv[e] / dg[e];
                rr += rv[e] * rv[e];
                rzn += rv[e] * zv[e];
            }
            block_sum2(rr, rzn, red);
            ++iters;
            if (rr <= tol2)
                break;
            const double beta = rzn / rz;
            rz = rzn;
            for (int e = tid; e < n6; e += kMfThreads)
                if (gd.free_pos[e / 6] >= 0)
                    pv[e] = zv[e] + beta * pv[e];
            lds_barrier();
        }
    }
    // solution in free-node order, flags
    bool bad = false;
    for (int e = tid; e < n6; e += kMfThreads) {
        const int fp = gd.free_pos[e / 6];
        if (fp >= 0) {
            xs[6 * fp + e % 6] = xv[e];
            bad |= !isfinite(xv[e]);
        }
    }
    if (singular || bad)
        atomicOr(&sflags, (singular ? 1 : 0) | (bad ? 2 : 0));
    if (tid == 0)
        gd.iter_stats[kIterRecord * it + 5] = (double)iters;
    __syncthreads();
    const int flags = sflags;
    if (n == 0) {
        if (tid == 0)
            *gd.iters_done = it + 1;
        return;
    }
    if (flags) {
        if (tid == 0)
            *gd.status |= (flags & 1) ? kStatusSingular : kStatusNonFinite;
        return;
    }
    update_poses(gd, xs, sfree, Ts);
    if (tid == 0)
        *gd.iters_done = it + 1;
    compute_transforms(gd, Ts);
}

hipError_t mf_set_max_lds(size_t bytes)
{
    return hipFuncSetAttribute((const void*)mf_pcg_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t mf_lds_bytes(int n_frames, int n_sets) { return sizeof(double) * mf_lds_doubles(n_frames, n_sets); }

void launch_mf_pcg(const GraphDev* gds, int n_graphs, size_t lds, hipStream_t st)
{
    mf_pcg_kernel<<<n_graphs, kMfThreads, lds, st>>>(gds);
}

// One block of 256 threads per graph: the single-wavefront block LDL^T for
// graphs resolved to it (16 x 16 tiles: 2 x 2 up to 28 unknowns, else 4 x 4),
// else block Gauss-Jordan on GNT x GNT tiles.
template <int GNT>
__global__ __launch_bounds__(256) void solve_mfma_kernel(const GraphDev* __restrict__ gds)
{
    __shared__ __attribute__((aligned(16))) double Rl[64 * kLdlStride];   // R rows of the LDL^T solve
    const GraphDev& gd = gds[blockIdx.x];
    if (gd.solver == kSolverLDL) {
        if (6 * gd.n_free <= kLdlMaxN2)
            ldl_solve<2>(gd, Rl);
        else
            ldl_solve<4>(gd, Rl);
    } else {
        gj_solve<GNT>(gd);
    }
}

// ------------------------------------------------------------ launchers

void launch_assemble(const GraphDev* gds, const int2* nbs, int n, hipStream_t st)
{
    if (n > 0)
        assemble_kernel<<<n, kAsmThreads, 0, st>>>(gds, nbs);
}

size_t solve_lds_bytes(int n_free, int n_frames)
{
    const size_t n = 6 * (size_t)n_free;
    return sizeof(double) * ((n + 1) * (n + 2) / 2 + 2 * (n + 1) + 4 * n + 16 * (size_t)n_frames);
}

// columns (n + 1) of the Gauss-Jordan system of n_free free nodes
int gj_slots(int n_free) { return 6 * n_free + 1; }

// Matrix-core solves: LDL^T graphs on their own tiles, Gauss-Jordan graphs on
// NT x NT tiles of 16 x 16, 16 NT >= cols (the widest Gauss-Jordan system).
void launch_mfma_solve(const GraphDev* gds, int n_graphs, int cols, hipStream_t st)
{
    static_assert(kGjMaxN + 1 <= 16 * 8, "Gauss-Jordan tiles too few for kGjMaxN");
    static_assert(kLdlMaxN <= 16 * 4 - 4 && kLdlMaxN2 <= 16 * 2 - 4, "LDL tiles too few");
    if (cols <= 32)
        solve_mfma_kernel<2><<<n_graphs, 256, 0, st>>>(gds);
    else if (cols <= 64)
        solve_mfma_kernel<4><<<n_graphs, 256, 0, st>>>(gds);
    else
        solve_mfma_kernel<8><<<n_graphs, 256, 0, st>>>(gds);
}

hipError_t solve_set_max_lds(size_t bytes)
{
    return hipFuncSetAttribute((const void*)solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_solve(const GraphDev* gds, int n_graphs, size_t lds, int mode, hipStream_t st)
{
    solve_kernel<<<n_graphs, kSolveThreads, lds, st>>>(gds, mode);
}

}  // namespace pg
