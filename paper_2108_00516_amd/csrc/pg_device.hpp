// Internal layout shared by the kernels and the host library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace pg {

constexpr int kMaxFrames = 32;       // hard cap of nodes per graph
constexpr int kMaxIters = 32;
constexpr int kDenseFields = 30;     // per item sums: 21 (J^T W J upper) + 6 (J^T W r) + E + count + target reads
constexpr int kDenseStride = 32;     // floats per dense partial record
constexpr int kFeatFields = 92;      // 78 (12x12 upper) + 12 + E + count
constexpr int kFeatStride = 96;
constexpr int kAssocThreads = 256;   // threads per association work item
constexpr int kTileMaxPixels = 8 * kAssocThreads;  // largest association tile
constexpr int kNodeStats = 5;        // per node: E_g, E_f, n_g, n_f, target reads (doubles)
constexpr int kIterRecord = 8;       // per iteration: E_f, E_g, n_g, n_f, target reads

// resolved solver of a graph (GraphDev::solver)
constexpr int kSolverPCG = 1;
constexpr int kSolverCholesky = 2;
constexpr int kSolverGaussJordan = 3;
constexpr int kSolverLDL = 4;
constexpr int kSolverPcgMatrixFree = 5;
constexpr int kMfMaxFrames = 14;   // matrix-free PCG: per-pair Gram blocks and feature blocks in LDS
constexpr int kGjMaxN = 126;
constexpr int kLdlMaxN = 60;     // single-wavefront LDL^T: 4 x 4 tiles of 16, rows padded to 4, one column for -g
constexpr int kLdlMaxN2 = 28;    //   2 x 2 tiles up to this size
constexpr int kSolveStaticLds = 4096;  // static LDS of the solve kernel (upper bound)         // Gauss-Jordan: at most 21 free nodes (n x (n+1) doubles in LDS)

// status bits (sticky, per graph)
constexpr int kStatusSingular = 1;
constexpr int kStatusNonFinite = 2;

// One association work item: source frame i, target frame j, a contiguous
// range of frame i's valid-pixel list.  'slot' is the index of its partial
// record within its graph.
struct WorkItem {
    int gij;    // i | (j << 8) | (graph << 16)
    int start;
    int count;
    int slot;
};

// Device view of one graph (one entry per graph of a batch).
struct GraphDev {
    int W, H, HW, n_frames;
    float fx, fy, cx, cy;
    double fx64, fy64, cx64, cy64;
    float ifx, ify;
    float lambda_f, lambda_g, huber_f, huber_g, gate_d2, gate_cos;
    int n_sets;       // feature match sets
    int n_free;
    int precision;
    int weighting;
    int solver;
    int pcg_max_iters;
    double pcg_rel_tol;

    const float4* maps;       // n_frames * HW packed {nx, ny, nz, z}; z = 0 invalid
    const float4* src_nz;     // frame f list at f*HW: {nx, ny, nz, z}
    const uint32_t* src_uv;   // frame f list at f*HW: u | v << 16
    const int* n_src;         // valid source pixels per frame
    const int* pair_base;     // N(N-1)+1 prefix sums: partial records of ordered pair p are [pair_base[p], pair_base[p+1])
    float* partials;          // dense partial records (global item index)
    double* fpartials;        // feature partial records per set (FP64)
    const float4* fpts;       // per match: {u, v, z, valid} of the pixel in frame i, then in frame j
    const int4* fsets;        // per set: {i, j, first match, count}
    const int* set_of;        // N*N: feature set of node pair, or -1
    float* xf32;              // per ordered pair: A (12) then B (12), rows of [R|t]
    double* xf64;             // per ordered pair: A (12)
    double* tinv64;           // per node: T^-1 = [R^T | -R^T t] (12)
    unsigned long long* maxdiag;  // bits of the largest positive diagonal entry of H_ff (an atomic
                                  // maximum by the assembly; cleared by the start and by each solve)
    double* poses;            // N * 16
    const double* poses_in;   // N * 16, pinned host memory: the poses an optimize starts from
    double* Hm;               // 6N * 6N normal matrix, row-major
    double* grad;             // 6N
    double* node_stats;       // N * kNodeStats
    const int* free_ids;      // n_free node ids
    const int* free_pos;      // per node: index among the free nodes, -1 if fixed
    double* Hff;              // free-node system [H_ff | -g_f], 6 n_free rows of 6 n_free + 1, row-major
    int* status;              // sticky status bits
    int* iters_done;
    double* iter_stats;       // kMaxIters * kIterRecord
    const __half* mlp;        // learned weighting parameters (fp16, as given)
    // learned weighting
    const float* mlp32;       // the same parameters as FP32 (read with uniform addresses)
    float gate_dist, inv_halfdiag, inv_iters;
    float4* psrc_nz;          // pruned source lists (learned weighting), frame f at f*HW;
    uint32_t* psrc_uv;        //   the unpruned lists when nothing is pruned
    unsigned int* score;      // per frame f: score bits of its source list entries at f*HW
    const int* n_drop;        // per frame: source pixels pruned
};

__host__ __device__ inline int pair_index(int i, int j, int n) { return i * (n - 1) + (j < i ? j : j - 1); }

}  // namespace pg
