// Host side of the C ABI declared in include/posegraph.h: argument checking,
// device buffers, the per-graph work tables, the Gauss-Newton schedule (plain
// launches or a captured hipGraph) and the batched path.
#include "pg_device.hpp"
#include "posegraph.h"
#include "pg_frontend.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace pg {
void launch_preprocess(const float* depth, const uint8_t* mask, int W, int H, float cx, float cy, float ifx,
                       float ify, float4* map, uint8_t* flag, int* row_cnt, int* total, float4* src_nz,
                       uint32_t* src_uv, hipStream_t st);
void launch_match_points(const float* di, const uint8_t* mi, const float* dj, const uint8_t* mj, int W, int H,
                         const float* uvi, const float* uvj, int n, float4* out, hipStream_t st);
int assoc_ppt_supported(int ppt);
void launch_assoc(const GraphDev* gds, const WorkItem* items, int n_items, int ppt, int precision, bool learned,
                  int iteration, const int2* fitems, int n_fitems, unsigned* ctr, int blocks_per_xcd,
                  hipStream_t st);
int assoc_persistent_blocks(int ppt, int precision, bool learned);
void launch_assoc_debug(const GraphDev* gds, int HW, int i, int j, int iteration, int* target, float* r,
                        float* uv, float* feat, float* sigma, hipStream_t st);
void launch_prune(const GraphDev* gds, const WorkItem* pitems, int n_pitems, const int2* pframes, int n_pframes,
                  int max_src, hipStream_t st);
void launch_mlp_to_float(const __half* p16, float* p32, hipStream_t st);
void launch_assemble(const GraphDev* gds, const int2* nbs, int n, hipStream_t st);
size_t solve_lds_bytes(int n_free, int n_frames);
int gj_slots(int n_free);   // columns of the Gauss-Jordan system
void launch_mfma_solve(const GraphDev* gds, int n_graphs, int cols, hipStream_t st);
hipError_t solve_set_max_lds(size_t bytes);
void launch_solve(const GraphDev* gds, int n_graphs, size_t lds, int mode, hipStream_t st);
size_t mf_lds_bytes(int n_frames, int n_sets);
hipError_t mf_set_max_lds(size_t bytes);
void launch_mf_pcg(const GraphDev* gds, int n_graphs, size_t lds, hipStream_t st);
hipError_t launch_ransac(const float4* maps, int W, int H, double fx, double fy, double cx, double cy,
                         const int4* pairs, int n_pairs, const float* uv_i, const float* uv_j, const int* samples,
                         int n_hyp, double delta, double cos_alpha, int* score, double* T, int* best, double* T_best,
                         unsigned char* inlier, hipStream_t st);
}  // namespace pg

using namespace pg;

namespace {

thread_local std::string g_create_error;

// RAII device buffer
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p)
            return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n ? n : 16);
        if (e == hipSuccess)
            bytes = n ? n : 16;
        return e;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

struct MatchSetHost {
    int i = 0, j = 0, n = 0;
    DevBuf pts;   // 2n float4
};

// Tables and buffers of one schedule (a single graph or a batch).
struct Schedule {
    std::vector<pg_graph*> graphs;
    std::vector<unsigned long long> versions;
    DevBuf gds, items, fitems, nbs, pitems, pframes;
    int n_items = 0, n_fitems = 0, n_nbs = 0, n_pitems = 0, n_pframes = 0;
    int max_src = 0;      // largest source list of a pruned frame
    bool learned = false; // learned weighting in every graph of the schedule
    size_t lds = 0;
    int ppt = 4;
    int iters = 0;
    bool gj = false;      // every graph solved on the matrix cores (LDL^T or Gauss-Jordan)
    bool mf = false;      // every graph solved by matrix-free PCG (no assembly)
    size_t mf_lds = 0;    // dynamic LDS of the matrix-free solve
    int precision = 0;    // PG_PREC_* of every graph of the schedule
    int gj_slots = 1;   // widest Gauss-Jordan system (columns) of the schedule (1 if none)
    bool persistent = false;   // persistent association blocks draining the work table
    int persist_bpx = 0;       //   their count per XCD
    DevBuf ctr;                //   8 run counters and a finished-block count (zero between launches)
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> events;   // timing: start, then 5 per iteration
    ~Schedule()
    {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        for (hipEvent_t e : events)
            (void)hipEventDestroy(e);
    }
};

}  // namespace

struct pg_graph {
    pg_config cfg;
    pg_camera cam;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = 0;
    int HW = 0;
    std::string err;
    unsigned long long version = 1;   // bumped whenever the schedule must be rebuilt

    int n_frames = 0;
    std::vector<int> fixed;
    std::vector<int> n_src;
    std::vector<double> poses;        // host mirror, 16 per node

    // per-frame device data (max_frames slots)
    DevBuf depth, mask, maps, src_nz, src_uv, flag, rowcnt, total;
    std::map<std::pair<int, int>, MatchSetHost> msets;

    // per-optimize device state
    DevBuf d_partials, d_fpartials, d_fpts, d_fsets, d_set_of, d_xf32, d_xf64, d_H, d_grad, d_node_stats,
        d_free_ids, d_free_pos, d_Hff, d_tinv64, d_maxdiag, d_n_src, d_pair_base, d_mlp;
    // results of an optimize, one block read back with one copy (same layout
    // as the pinned host mirror): status, iterations done, per-iteration
    // records (kMaxIters), poses (max_frames)
    DevBuf d_result;
    int* dev_status() const { return d_result.as<int>(); }
    int* dev_iters() const { return d_result.as<int>() + 1; }
    double* dev_iter_stats() const { return reinterpret_cast<double*>(d_result.as<int>() + 2); }
    double* dev_poses() const { return dev_iter_stats() + kIterRecord * kMaxIters; }
    size_t result_bytes() const { return sizeof(int) * 2 + sizeof(double) * (kIterRecord * kMaxIters + 16 * n_frames); }
    // learned weighting: FP32 parameters, pruned source lists, scores, drop counts
    DevBuf d_mlp32, d_psrc_nz, d_psrc_uv, d_score, d_n_drop;
    bool poses_dirty = true;          // host mirror newer than d_poses
    int n_sets = 0, n_free = 0, n_items = 0, tile = 0;
    int solver = kSolverCholesky;     // resolved solver of the current tables
    int lds_limit = 65536;            // device LDS per workgroup
    unsigned long long tables_version = 0;   // version the tables were built for
    std::vector<int> pair_base;
    std::vector<WorkItem> items;      // local items (graph field 0)
    std::vector<int4> fsets;
    bool has_mlp = false;
    bool learned = false, pruned = false;   // of the current tables
    std::vector<int> n_drop;          // source pixels pruned per frame
    std::vector<int> n_eff;           // source pixels associated per frame (n_src - n_drop)
    std::vector<WorkItem> pitems;     // pruning score items (frame, 256-entry tile)

    std::unique_ptr<Schedule> sched;  // single-graph schedule cache
    // pinned readback
    int* h_status = nullptr;
    int* h_iters = nullptr;
    double* h_iter_stats = nullptr;
    double* h_poses = nullptr;
    double* h_up = nullptr;           // pinned staging of pose uploads
    hipEvent_t up_done = nullptr;     // the last upload from h_up has completed
};

namespace {

std::mutex g_batch_mutex;
std::vector<std::unique_ptr<Schedule>> g_batch_cache;

pg_status fail(pg_graph* g, pg_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (g)
        g->err = buf;
    else
        g_create_error = buf;
    return s;
}

#define HIP_OR_FAIL(g, call)                                                                             \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return fail((g), e_ == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP, "%s: %s",   \
                        #call, hipGetErrorString(e_));                                                   \
    } while (0)

bool finite_pose(const double* T)
{
    for (int k = 0; k < 16; ++k)
        if (!isfinite(T[k]))
            return false;
    if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0)
        return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += T[4 * k + a] * T[4 * k + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6)
                return false;
        }
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    return det > 0.0;
}

bool is_device_ptr(const void* p)
{
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

// copy 'bytes' from a host or device pointer into device memory on the stream
hipError_t copy_in(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    return hipMemcpyAsync(dst, src, bytes, is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          st);
}

// Tuned association tiles by window class (resolution, node-count range),
// set with pg_set_tile_table; consulted when a graph's tile_pixels is 0.
struct TileClass {
    int width, height, lo, hi, tile;
};
std::mutex g_tile_mutex;
std::vector<TileClass> g_tile_table;
constexpr int kTileTableMax = 256;

int table_tile(int width, int height, int n_frames)
{
    std::lock_guard<std::mutex> lk(g_tile_mutex);
    for (const TileClass& e : g_tile_table)
        if (e.width == width && e.height == height && e.lo <= n_frames && n_frames <= e.hi)
            return e.tile;
    return 0;
}

// Source pixels per work item (a multiple of 256, at most kTileMaxPixels) and
// the pixels per thread of the kernel that runs it (1, 2, 4 or 8: the
// smallest whose 256-thread block covers the tile).  A batch runs with the
// largest pixels per thread of its graphs; a shorter item leaves the slots
// past its end empty, so every graph keeps its own tile.
int pick_tile(const pg_graph* g, int* ppt)
{
    int t = g->cfg.tile_pixels;
    if (t <= 0)
        t = table_tile(g->cam.width, g->cam.height, g->n_frames);
    if (t <= 0)
        t = 1024;
    t = std::min(std::max(t, kAssocThreads), kTileMaxPixels);
    t = (t + kAssocThreads - 1) / kAssocThreads * kAssocThreads;
    int p = t / kAssocThreads;
    while (!assoc_ppt_supported(p))
        ++p;
    *ppt = p;
    return t;
}

// (Re)build the graph's tables and device state for the current frames/matches.
pg_status prepare_graph(pg_graph* g)
{
    const int N = g->n_frames;
    if (N < 1)
        return fail(g, PG_ERR_INVALID_ARG, "graph has no frames");
    int ppt;
    const int tile = pick_tile(g, &ppt);
    if (g->tables_version == g->version && g->tile == tile)
        return PG_OK;
    g->tile = tile;
    // free nodes
    std::vector<int> free_ids;
    for (int f = 0; f < N; ++f)
        if (!g->fixed[f])
            free_ids.push_back(f);
    g->n_free = (int)free_ids.size();
    {
        const int nf = 6 * g->n_free;
        const bool gj_fits = nf <= kGjMaxN, ldl_fits = nf <= kLdlMaxN;
        switch (g->cfg.solver) {
        case PG_SOLVER_PCG: g->solver = kSolverPCG; break;
        case PG_SOLVER_CHOLESKY: g->solver = kSolverCholesky; break;
        case PG_SOLVER_GAUSS_JORDAN:
            if (!gj_fits)
                return fail(g, PG_ERR_CAPACITY, "Gauss-Jordan solve of %d unknowns exceeds %d", nf, kGjMaxN);
            g->solver = kSolverGaussJordan;
            break;
        case PG_SOLVER_LDL:
            if (!ldl_fits)
                return fail(g, PG_ERR_CAPACITY, "LDL^T solve of %d unknowns exceeds %d", nf, kLdlMaxN);
            g->solver = kSolverLDL;
            break;
        case PG_SOLVER_PCG_MATRIX_FREE:
            if (N > kMfMaxFrames)
                return fail(g, PG_ERR_CAPACITY, "matrix-free PCG holds at most %d frames", kMfMaxFrames);
            g->solver = kSolverPcgMatrixFree;
            break;
        default: g->solver = ldl_fits ? kSolverLDL : gj_fits ? kSolverGaussJordan : kSolverCholesky; break;
        }
        // the LDS kernel runs every optimisation's transforms prologue (and
        // the Cholesky/PCG solve) with this graph's packed layout: creation
        // checked it for one fixed node, a window with fewer must fit as well
        const size_t lds = solve_lds_bytes(g->n_free, N);
        if (lds > (size_t)g->lds_limit)
            return fail(g, PG_ERR_CAPACITY, "%d free nodes need %zu B of LDS for the solve, the limit is %d B",
                        g->n_free, lds, g->lds_limit);
    }
    // learned weighting: each frame keeps its n_src - floor(frac * n_src)
    // best-scored source pixels; the counts are known here, the choice is
    // made on the device at the start of every optimize
    g->learned = g->cfg.weighting == PG_WEIGHT_LEARNED;
    if (g->learned && !g->has_mlp)
        return fail(g, PG_ERR_INVALID_ARG, "learned weighting needs the network parameters (pose_graph_set_mlp)");
    g->pruned = g->learned && g->cfg.prune_frac > 0.0;
    g->n_drop.assign(N, 0);
    g->n_eff = g->n_src;
    g->pitems.clear();
    if (g->pruned)
        for (int i = 0; i < N; ++i) {
            g->n_drop[i] = (int)floor(g->cfg.prune_frac * (double)g->n_src[i]);
            g->n_eff[i] = g->n_src[i] - g->n_drop[i];
            for (int k = 0; k < g->n_src[i]; k += 256) {
                WorkItem w;
                w.gij = i;
                w.start = k;
                w.count = std::min(256, g->n_src[i] - k);
                w.slot = 0;
                g->pitems.push_back(w);
            }
        }
    // dense work items, ordered (source frame, tile, target frame); the
    // partial records of each ordered pair are contiguous (pair_base)
    const int P = N * (N - 1);
    std::vector<int> n_tiles(N, 0);
    for (int i = 0; i < N; ++i)
        n_tiles[i] = (g->n_eff[i] + tile - 1) / tile;
    g->pair_base.assign(P + 1, 0);
    for (int p = 0; p < P; ++p)
        g->pair_base[p + 1] = g->pair_base[p] + n_tiles[p / std::max(N - 1, 1)];
    g->items.clear();
    for (int i = 0; i < N && N > 1; ++i)
        for (int t = 0; t < n_tiles[i]; ++t)
            for (int j = 0; j < N; ++j) {
                if (j == i)
                    continue;
                WorkItem w;
                w.gij = i | (j << 8);
                w.start = t * tile;
                w.count = std::min(tile, g->n_eff[i] - t * tile);
                w.slot = g->pair_base[pair_index(i, j, N)] + t;
                g->items.push_back(w);
            }
    const int slot = g->pair_base[P];
    g->n_items = slot;
    // feature sets, in (i, j) order
    g->fsets.clear();
    std::vector<int> set_of(N * N, -1);
    size_t total_m = 0;
    for (auto& kv : g->msets)
        total_m += kv.second.n;
    HIP_OR_FAIL(g, g->d_fpts.ensure(sizeof(float4) * 2 * std::max<size_t>(total_m, 1)));
    size_t off = 0;
    for (auto& kv : g->msets) {
        MatchSetHost& m = kv.second;
        if (m.n <= 0)
            continue;
        set_of[m.i * N + m.j] = set_of[m.j * N + m.i] = (int)g->fsets.size();
        g->fsets.push_back(make_int4(m.i, m.j, (int)off, m.n));
        HIP_OR_FAIL(g, hipMemcpyAsync(g->d_fpts.as<float4>() + 2 * off, m.pts.p, sizeof(float4) * 2 * m.n,
                                      hipMemcpyDeviceToDevice, g->stream));
        off += m.n;
    }
    g->n_sets = (int)g->fsets.size();
    HIP_OR_FAIL(g, g->d_partials.ensure(sizeof(float) * kDenseStride * std::max(g->n_items, 1)));
    HIP_OR_FAIL(g, g->d_fpartials.ensure(sizeof(double) * kFeatStride * std::max(g->n_sets, 1)));
    HIP_OR_FAIL(g, g->d_fsets.ensure(sizeof(int4) * std::max(g->n_sets, 1)));
    HIP_OR_FAIL(g, g->d_set_of.ensure(sizeof(int) * N * N));
    HIP_OR_FAIL(g, g->d_xf32.ensure(sizeof(float) * 24 * std::max(P, 1)));
    HIP_OR_FAIL(g, g->d_xf64.ensure(sizeof(double) * 12 * std::max(P, 1)));
    HIP_OR_FAIL(g, g->d_tinv64.ensure(sizeof(double) * 12 * N));
    HIP_OR_FAIL(g, g->d_maxdiag.ensure(sizeof(unsigned long long)));
    HIP_OR_FAIL(g, g->d_H.ensure(sizeof(double) * 36 * N * N));
    HIP_OR_FAIL(g, g->d_grad.ensure(sizeof(double) * 6 * N));
    HIP_OR_FAIL(g, g->d_node_stats.ensure(sizeof(double) * kNodeStats * N));
    HIP_OR_FAIL(g, g->d_free_ids.ensure(sizeof(int) * std::max(g->n_free, 1)));
    HIP_OR_FAIL(g, g->d_free_pos.ensure(sizeof(int) * N));
    HIP_OR_FAIL(g, g->d_Hff.ensure(sizeof(double) * std::max(6 * g->n_free * (6 * g->n_free + 1), 1)));
    HIP_OR_FAIL(g, g->d_n_src.ensure(sizeof(int) * N));
    HIP_OR_FAIL(g, g->d_pair_base.ensure(sizeof(int) * (P + 1)));
    if (g->pruned) {
        const size_t NHW = (size_t)N * g->HW;
        HIP_OR_FAIL(g, g->d_psrc_nz.ensure(sizeof(float4) * NHW));
        HIP_OR_FAIL(g, g->d_psrc_uv.ensure(sizeof(uint32_t) * NHW));
        HIP_OR_FAIL(g, g->d_score.ensure(sizeof(unsigned int) * NHW));
        HIP_OR_FAIL(g, g->d_n_drop.ensure(sizeof(int) * N));
        HIP_OR_FAIL(g, hipMemcpyAsync(g->d_n_drop.p, g->n_drop.data(), sizeof(int) * N, hipMemcpyHostToDevice,
                                      g->stream));
    }
    if (g->n_sets)
        HIP_OR_FAIL(g, hipMemcpyAsync(g->d_fsets.p, g->fsets.data(), sizeof(int4) * g->n_sets,
                                      hipMemcpyHostToDevice, g->stream));
    HIP_OR_FAIL(g, hipMemcpyAsync(g->d_set_of.p, set_of.data(), sizeof(int) * N * N, hipMemcpyHostToDevice,
                                  g->stream));
    if (g->n_free)
        HIP_OR_FAIL(g, hipMemcpyAsync(g->d_free_ids.p, free_ids.data(), sizeof(int) * g->n_free,
                                      hipMemcpyHostToDevice, g->stream));
    std::vector<int> free_pos(N, -1);
    for (int k = 0; k < g->n_free; ++k)
        free_pos[free_ids[k]] = k;
    HIP_OR_FAIL(g, hipMemcpyAsync(g->d_free_pos.p, free_pos.data(), sizeof(int) * N, hipMemcpyHostToDevice,
                                  g->stream));
    HIP_OR_FAIL(g, hipMemcpyAsync(g->d_n_src.p, g->n_src.data(), sizeof(int) * N, hipMemcpyHostToDevice,
                                  g->stream));
    HIP_OR_FAIL(g, hipMemcpyAsync(g->d_pair_base.p, g->pair_base.data(), sizeof(int) * (P + 1),
                                  hipMemcpyHostToDevice, g->stream));
    // the host copies above read pageable host vectors that stay alive; make
    // sure they completed before the vectors may change
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    g->tables_version = g->version;
    return PG_OK;
}

GraphDev make_dev(pg_graph* g)
{
    GraphDev d;
    memset(&d, 0, sizeof(d));
    d.W = g->cam.width;
    d.H = g->cam.height;
    d.HW = g->HW;
    d.n_frames = g->n_frames;
    d.fx = (float)g->cam.fx;
    d.fy = (float)g->cam.fy;
    d.cx = (float)g->cam.cx;
    d.cy = (float)g->cam.cy;
    d.fx64 = g->cam.fx;
    d.fy64 = g->cam.fy;
    d.cx64 = g->cam.cx;
    d.cy64 = g->cam.cy;
    d.ifx = (float)(1.0 / g->cam.fx);
    d.ify = (float)(1.0 / g->cam.fy);
    d.lambda_f = (float)g->cfg.lambda_f;
    d.lambda_g = (float)g->cfg.lambda_g;
    d.huber_f = (float)g->cfg.huber_f_m;
    d.huber_g = (float)g->cfg.huber_g_m;
    d.gate_d2 = (float)(g->cfg.gate_dist_m * g->cfg.gate_dist_m);
    d.gate_cos = (float)cos(g->cfg.gate_normal_rad);
    d.n_sets = g->n_sets;
    d.n_free = g->n_free;
    d.precision = g->cfg.precision;
    d.weighting = g->cfg.weighting;
    d.solver = g->solver;
    d.pcg_max_iters = g->cfg.pcg_max_iters;
    d.pcg_rel_tol = g->cfg.pcg_rel_tol;
    d.maps = g->maps.as<float4>();
    d.src_nz = g->src_nz.as<float4>();
    d.src_uv = g->src_uv.as<uint32_t>();
    d.n_src = g->d_n_src.as<int>();
    d.pair_base = g->d_pair_base.as<int>();
    d.partials = g->d_partials.as<float>();
    d.fpartials = g->d_fpartials.as<double>();
    d.fpts = g->d_fpts.as<float4>();
    d.fsets = g->d_fsets.as<int4>();
    d.set_of = g->d_set_of.as<int>();
    d.xf32 = g->d_xf32.as<float>();
    d.xf64 = g->d_xf64.as<double>();
    d.tinv64 = g->d_tinv64.as<double>();
    d.maxdiag = g->d_maxdiag.as<unsigned long long>();
    d.poses = g->dev_poses();
    d.poses_in = g->h_up;
    d.Hm = g->d_H.as<double>();
    d.grad = g->d_grad.as<double>();
    d.node_stats = g->d_node_stats.as<double>();
    d.free_ids = g->d_free_ids.as<int>();
    d.free_pos = g->d_free_pos.as<int>();
    d.Hff = g->d_Hff.as<double>();
    d.status = g->dev_status();
    d.iters_done = g->dev_iters();
    d.iter_stats = g->dev_iter_stats();
    d.mlp = g->d_mlp.as<__half>();
    d.mlp32 = g->has_mlp ? g->d_mlp32.as<float>() : nullptr;
    d.gate_dist = (float)g->cfg.gate_dist_m;
    d.inv_halfdiag = (float)(1.0 / sqrt(0.25 * d.W * d.W + 0.25 * d.H * d.H));
    d.inv_iters = (float)(1.0 / std::max(g->cfg.gn_iters - 1, 1));
    if (g->learned) {
        d.psrc_nz = g->pruned ? g->d_psrc_nz.as<float4>() : g->src_nz.as<float4>();
        d.psrc_uv = g->pruned ? g->d_psrc_uv.as<uint32_t>() : g->src_uv.as<uint32_t>();
        d.score = g->pruned ? g->d_score.as<unsigned int>() : nullptr;
        d.n_drop = g->pruned ? g->d_n_drop.as<int>() : nullptr;
    }
    return d;
}

pg_status upload_poses(pg_graph* g)
{
    // the start kernel (solve_kernel, mode 1) reads the poses straight from
    // this pinned staging buffer (no copy launch).  The host mirror equals
    // the device poses after every optimize, so the buffer always gets the
    // mirror; it is rewritten only once the previous start kernel reading it
    // has completed (the entry points synchronise their stream, the one that
    // does not records up_done)
    HIP_OR_FAIL(g, hipEventSynchronize(g->up_done));
    memcpy(g->h_up, g->poses.data(), sizeof(double) * 16 * g->n_frames);
    g->poses_dirty = false;
    return PG_OK;
}

// Build a schedule (device tables of all graphs) for one graph or a batch.
pg_status build_schedule(const std::vector<pg_graph*>& gs, Schedule& s)
{
    pg_graph* g0 = gs[0];
    s.graphs = gs;
    s.versions.clear();
    s.max_src = 0;
    std::vector<GraphDev> devs;
    std::vector<WorkItem> items;
    std::vector<int2> fitems, nbs, pframes;
    std::vector<WorkItem> pitems;
    size_t lds = 0;
    int ppt = 4;
    for (size_t k = 0; k < gs.size(); ++k) {
        pg_graph* g = gs[k];
        pg_status st = prepare_graph(g);
        if (st != PG_OK)
            return st;
        s.versions.push_back(g->version);
        int p;
        pick_tile(g, &p);
        if (k == 0) {
            ppt = p;
            s.precision = g->cfg.precision;
            s.learned = g->learned;
        } else if (g->learned != s.learned) {
            return fail(g0, PG_ERR_INVALID_ARG, "graphs of a batch must use one weighting");
        } else if (g->cfg.precision != s.precision) {
            return fail(g0, PG_ERR_INVALID_ARG, "graphs of a batch must use one precision");
        } else if ((g->cfg.persistent != 0) != (g0->cfg.persistent != 0)) {
            return fail(g0, PG_ERR_INVALID_ARG, "graphs of a batch must share the persistent setting");
        }
        ppt = std::max(ppt, p);
        devs.push_back(make_dev(g));
        for (const WorkItem& w : g->items) {
            WorkItem v = w;
            v.gij |= (int)k << 16;
            items.push_back(v);
        }
        for (int t = 0; t < g->n_sets; ++t)
            fitems.push_back(make_int2((int)k, t));
        for (const WorkItem& w : g->pitems) {
            WorkItem v = w;
            v.gij |= (int)k << 16;
            pitems.push_back(v);
        }
        if (g->pruned)
            for (int f = 0; f < g->n_frames; ++f) {
                pframes.push_back(make_int2((int)k, f));
                s.max_src = std::max(s.max_src, g->n_src[f]);
            }
        for (int I = 0; I < g->n_frames; ++I)
            for (int J = 0; J <= I; ++J)
                nbs.push_back(make_int2((int)k, I | (J << 8)));
        lds = std::max(lds, solve_lds_bytes(g->n_free, g->n_frames));
    }
    // one solve kernel for the whole schedule: the matrix-core kernel when
    // every graph resolved to LDL^T or Gauss-Jordan (each graph keeps its own,
    // so a batched graph's step is its single run's bit for bit), else the
    // LDS Cholesky/PCG kernel (those graphs then use Cholesky, which gives the
    // same step up to rounding)
    s.gj = true;
    s.mf = true;
    s.gj_slots = 1;
    s.mf_lds = 0;
    for (pg_graph* g : gs) {
        s.gj = s.gj && (g->solver == kSolverGaussJordan || g->solver == kSolverLDL);
        s.mf = s.mf && g->solver == kSolverPcgMatrixFree;
        if (g->solver == kSolverGaussJordan)
            s.gj_slots = std::max(s.gj_slots, gj_slots(g->n_free));
        s.mf_lds = std::max(s.mf_lds, mf_lds_bytes(g->n_frames, g->n_sets));
    }
    if (s.mf) {
        if (s.mf_lds > (size_t)g0->lds_limit)
            return fail(g0, PG_ERR_CAPACITY, "matrix-free PCG needs %zu B of LDS", s.mf_lds);
        HIP_OR_FAIL(g0, mf_set_max_lds(s.mf_lds));
    }
    if (!s.gj && !s.mf)
        for (GraphDev& d : devs)
            if (d.solver == kSolverGaussJordan || d.solver == kSolverLDL || d.solver == kSolverPcgMatrixFree)
                d.solver = kSolverCholesky;
    // items of all graphs are concatenated; the XCD mapping of the association
    // kernel hands each XCD a contiguous run of them
    s.n_items = (int)items.size();
    s.n_fitems = (int)fitems.size();
    s.n_nbs = (int)nbs.size();
    s.n_pitems = (int)pitems.size();
    s.n_pframes = (int)pframes.size();
    s.lds = lds;
    s.ppt = ppt;
    HIP_OR_FAIL(g0, s.gds.ensure(sizeof(GraphDev) * devs.size()));
    HIP_OR_FAIL(g0, s.items.ensure(sizeof(WorkItem) * std::max<size_t>(items.size(), 1)));
    HIP_OR_FAIL(g0, s.fitems.ensure(sizeof(int2) * std::max<size_t>(fitems.size(), 1)));
    HIP_OR_FAIL(g0, s.nbs.ensure(sizeof(int2) * std::max<size_t>(nbs.size(), 1)));
    HIP_OR_FAIL(g0, s.pitems.ensure(sizeof(WorkItem) * std::max<size_t>(pitems.size(), 1)));
    HIP_OR_FAIL(g0, s.pframes.ensure(sizeof(int2) * std::max<size_t>(pframes.size(), 1)));
    hipStream_t st = g0->stream;
    // persistent association: as many blocks as stay resident, counters
    // zeroed here once (the kernel clears them after every launch)
    s.persistent = g0->cfg.persistent != 0;
    if (s.persistent) {
        s.persist_bpx = assoc_persistent_blocks(ppt, s.precision, s.learned);
        if (s.persist_bpx <= 0)
            s.persist_bpx = 32;
        HIP_OR_FAIL(g0, s.ctr.ensure(sizeof(unsigned) * 9));
        HIP_OR_FAIL(g0, hipMemsetAsync(s.ctr.p, 0, sizeof(unsigned) * 9, st));
    }
    HIP_OR_FAIL(g0, hipMemcpyAsync(s.gds.p, devs.data(), sizeof(GraphDev) * devs.size(), hipMemcpyHostToDevice, st));
    if (!items.empty())
        HIP_OR_FAIL(g0, hipMemcpyAsync(s.items.p, items.data(), sizeof(WorkItem) * items.size(),
                                       hipMemcpyHostToDevice, st));
    if (!fitems.empty())
        HIP_OR_FAIL(g0, hipMemcpyAsync(s.fitems.p, fitems.data(), sizeof(int2) * fitems.size(),
                                       hipMemcpyHostToDevice, st));
    if (!nbs.empty())
        HIP_OR_FAIL(g0, hipMemcpyAsync(s.nbs.p, nbs.data(), sizeof(int2) * nbs.size(), hipMemcpyHostToDevice, st));
    if (!pitems.empty())
        HIP_OR_FAIL(g0, hipMemcpyAsync(s.pitems.p, pitems.data(), sizeof(WorkItem) * pitems.size(),
                                       hipMemcpyHostToDevice, st));
    if (!pframes.empty())
        HIP_OR_FAIL(g0, hipMemcpyAsync(s.pframes.p, pframes.data(), sizeof(int2) * pframes.size(),
                                       hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(g0, hipStreamSynchronize(st));
    if (s.exec) {
        (void)hipGraphExecDestroy(s.exec);
        s.exec = nullptr;
    }
    return PG_OK;
}

// Enqueue the whole optimisation: prepare (and the pruning pass of the
// learned weighting), then per iteration the four phases on one stream.  The
// feature term runs first: it is independent of the association, and as a
// forked graph branch its fork and join cost more than it does.  With events
// (1 + 5 per iteration), each launch is bracketed on the stream.
hipError_t enqueue_iters(const Schedule& s, int iters, hipStream_t st, const std::vector<hipEvent_t>* ev)
{
    const GraphDev* gds = s.gds.as<GraphDev>();
    const int ng = (int)s.graphs.size();
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord((*ev)[0], st)) != hipSuccess)
        return e;
    launch_solve(gds, ng, s.lds, 1, st);
    launch_prune(gds, s.pitems.as<WorkItem>(), s.n_pitems, s.pframes.as<int2>(), s.n_pframes, s.max_src, st);
    for (int it = 0; it < iters; ++it) {
        const hipEvent_t* m = ev ? ev->data() + 1 + 5 * it : nullptr;
        if (m && (e = hipEventRecord(m[0], st)) != hipSuccess)
            return e;
        // the feature match sets run in the first blocks of the association
        // launch (the timing slot of the features stays empty)
        if (m && (e = hipEventRecord(m[1], st)) != hipSuccess)
            return e;
        launch_assoc(gds, s.items.as<WorkItem>(), s.n_items, s.ppt, s.precision, s.learned, it,
                     s.fitems.as<int2>(), s.n_fitems, s.persistent ? s.ctr.as<unsigned>() : nullptr,
                     s.persist_bpx, st);
        if (m && (e = hipEventRecord(m[2], st)) != hipSuccess)
            return e;
        if (!s.mf)
            launch_assemble(gds, s.nbs.as<int2>(), s.n_nbs, st);
        if (m && (e = hipEventRecord(m[3], st)) != hipSuccess)
            return e;
        if (s.mf)
            launch_mf_pcg(gds, ng, s.mf_lds, st);
        else if (s.gj)
            launch_mfma_solve(gds, ng, s.gj_slots, st);
        else
            launch_solve(gds, ng, s.lds, 0, st);
        if (m && (e = hipEventRecord(m[4], st)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

pg_status run_schedule(Schedule& s, int iters, bool use_graph, bool timing, std::vector<pg_stats*>& stats)
{
    pg_graph* g0 = s.graphs[0];
    hipStream_t st = g0->stream;
    for (pg_graph* g : s.graphs) {
        pg_status r = upload_poses(g);
        if (r != PG_OK)
            return r;
    }
    if (timing && s.events.size() != (size_t)(1 + 5 * iters)) {
        for (hipEvent_t e : s.events)
            (void)hipEventDestroy(e);
        s.events.assign(1 + 5 * iters, nullptr);
        for (auto& e : s.events)
            HIP_OR_FAIL(g0, hipEventCreate(&e));
    }
    const std::vector<hipEvent_t>* ev = timing ? &s.events : nullptr;
    // events recorded inside a captured graph cannot be queried for elapsed
    // time, so timing runs the same launches directly on the stream
    if (use_graph && !timing) {
        if (!s.exec || s.iters != iters) {
            if (s.exec) {
                (void)hipGraphExecDestroy(s.exec);
                s.exec = nullptr;
            }
            hipStream_t cs = g0->capture_stream;
            HIP_OR_FAIL(g0, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t ce = enqueue_iters(s, iters, cs, nullptr);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &graph);
            if (ce != hipSuccess || e != hipSuccess) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return fail(g0, PG_ERR_HIP, "graph capture failed: %s",
                            hipGetErrorString(ce != hipSuccess ? ce : e));
            }
            e = hipGraphInstantiate(&s.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                s.exec = nullptr;
                return fail(g0, PG_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
            }
            s.iters = iters;
        }
        HIP_OR_FAIL(g0, hipGraphLaunch(s.exec, st));
    } else {
        HIP_OR_FAIL(g0, enqueue_iters(s, iters, st, ev));
    }
    // read back poses and statistics of every graph
    for (pg_graph* g : s.graphs) {
        HIP_OR_FAIL(g0, hipMemcpyAsync(g->h_status, g->d_result.p, g->result_bytes(), hipMemcpyDeviceToHost, st));
    }
    HIP_OR_FAIL(g0, hipStreamSynchronize(st));
    float ms[5] = {0, 0, 0, 0, 0};   // assoc, feature, assemble, solve, total
    int n_assoc = 0;
    if (timing) {
        const int slot[4] = {1, 0, 2, 3};   // event intervals: feature, assoc, assemble, solve
        for (int it = 0; it < iters; ++it)
            for (int k = 0; k < 4; ++k) {
                float t = 0.f;
                HIP_OR_FAIL(g0, hipEventElapsedTime(&t, s.events[1 + 5 * it + k], s.events[2 + 5 * it + k]));
                ms[slot[k]] += t;
            }
        HIP_OR_FAIL(g0, hipEventElapsedTime(&ms[4], s.events[0], s.events[5 * iters]));
        n_assoc = s.n_items > 0 ? iters : 0;
    }
    pg_status ret = PG_OK;
    for (size_t k = 0; k < s.graphs.size(); ++k) {
        pg_graph* g = s.graphs[k];
        memcpy(g->poses.data(), g->h_poses, sizeof(double) * 16 * g->n_frames);
        pg_status r = PG_OK;
        if (*g->h_status & kStatusSingular)
            r = fail(g, PG_ERR_SINGULAR, "normal equations not positive definite at iteration %d", *g->h_iters);
        else if (*g->h_status & kStatusNonFinite)
            r = fail(g, PG_ERR_NONFINITE, "non-finite update at iteration %d", *g->h_iters);
        if (ret == PG_OK)
            ret = r;
        pg_stats* out = stats[k];
        if (out) {
            memset(out, 0, sizeof(*out));
            out->iters_done = *g->h_iters;
            const int rec = std::min(iters, *g->h_iters + (r != PG_OK ? 1 : 0));
            for (int it = 0; it < rec && it < PG_MAX_ITERS; ++it) {
                out->energy_f[it] = g->h_iter_stats[kIterRecord * it + 0];
                out->energy_g[it] = g->h_iter_stats[kIterRecord * it + 1];
                out->n_valid_g[it] = (long long)g->h_iter_stats[kIterRecord * it + 2];
                out->n_valid_f[it] = (long long)g->h_iter_stats[kIterRecord * it + 3];
                out->n_target_reads[it] = (long long)g->h_iter_stats[kIterRecord * it + 4];
                out->pcg_iters[it] = (g->solver == kSolverPCG || g->solver == kSolverPcgMatrixFree)
                                         ? (int)g->h_iter_stats[kIterRecord * it + 5]
                                         : 0;
            }
            out->status_bits = *g->h_status;
            long long sp = 0;
            for (int f = 0; f < g->n_frames; ++f)
                sp += (long long)g->n_eff[f] * (g->n_frames - 1);
            out->src_pixels = sp;
            out->n_assoc_launches = n_assoc;
            out->ms_assoc = ms[0];
            out->ms_feature = ms[1];
            out->ms_reduce = ms[2];
            out->ms_solve = ms[3];
            out->ms_total = ms[4];
        }
    }
    return ret;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

void pg_config_default(pg_config* c)
{
    if (!c)
        return;
    memset(c, 0, sizeof(*c));
    c->max_frames = 16;
    c->gn_iters = 7;
    c->lambda_f = 1.0;
    c->lambda_g = 1.0;
    c->huber_f_m = 0.005;
    c->huber_g_m = 0.005;
    c->gate_dist_m = 0.01;
    c->gate_normal_rad = 30.0 * M_PI / 180.0;
    c->solver = PG_SOLVER_AUTO;
    c->pcg_max_iters = 500;
    c->pcg_rel_tol = 1e-12;
    c->weighting = PG_WEIGHT_HUBER;
    c->precision = PG_PREC_FP32;
    // direct launches: measured faster than replaying the 22-node graph
    c->use_graph = 0;
    c->timing = 0;
    c->tile_pixels = 0;
    c->prune_frac = 0.25;
}

pg_status pose_graph_create(const pg_config* cfg, const pg_camera* cam, void* hip_stream, pg_graph** out)
{
    if (!out)
        return fail(nullptr, PG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || !cam)
        return fail(nullptr, PG_ERR_INVALID_ARG, "cfg and cam are required");
    if (cam->width < 3 || cam->height < 3 || cam->width > 8192 || cam->height > 8192)
        return fail(nullptr, PG_ERR_INVALID_ARG, "image size %dx%d out of range", cam->width, cam->height);
    if (!(cam->fx > 0 && cam->fy > 0 && isfinite(cam->fx) && isfinite(cam->fy) && isfinite(cam->cx) &&
          isfinite(cam->cy)))
        return fail(nullptr, PG_ERR_INVALID_ARG, "bad intrinsics");
    if (cfg->max_frames < 2 || cfg->max_frames > PG_MAX_FRAMES_LIMIT)
        return fail(nullptr, PG_ERR_INVALID_ARG, "max_frames %d out of [2, %d]", cfg->max_frames,
                    PG_MAX_FRAMES_LIMIT);
    if (cfg->gn_iters < 0 || cfg->gn_iters > PG_MAX_ITERS)
        return fail(nullptr, PG_ERR_INVALID_ARG, "gn_iters %d out of [0, %d]", cfg->gn_iters, PG_MAX_ITERS);
    if (!(cfg->huber_f_m > 0 && cfg->huber_g_m > 0 && cfg->gate_dist_m > 0 && cfg->gate_normal_rad > 0 &&
          cfg->gate_normal_rad <= M_PI && cfg->lambda_f >= 0 && cfg->lambda_g >= 0))
        return fail(nullptr, PG_ERR_INVALID_ARG, "bad method parameters");
    if (cfg->solver < PG_SOLVER_AUTO || cfg->solver > PG_SOLVER_PCG_MATRIX_FREE)
        return fail(nullptr, PG_ERR_INVALID_ARG, "unknown solver");
    if (cfg->weighting != PG_WEIGHT_HUBER && cfg->weighting != PG_WEIGHT_LEARNED)
        return fail(nullptr, PG_ERR_INVALID_ARG, "unknown weighting");
    if (cfg->precision != PG_PREC_FP32 && cfg->precision != PG_PREC_BF16X3)
        return fail(nullptr, PG_ERR_INVALID_ARG, "unknown precision");
    if (cfg->tile_pixels < 0 || cfg->tile_pixels > kTileMaxPixels)
        return fail(nullptr, PG_ERR_INVALID_ARG, "tile_pixels out of range");
    if (cfg->persistent != 0 && cfg->persistent != 1)
        return fail(nullptr, PG_ERR_INVALID_ARG, "persistent must be 0 or 1");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(nullptr, PG_ERR_NO_DEVICE, "no HIP device");
    }
    pg_graph* g = new (std::nothrow) pg_graph();
    if (!g)
        return fail(nullptr, PG_ERR_OUT_OF_MEMORY, "host allocation failed");
    g->cfg = *cfg;
    g->cam = *cam;
    g->stream = (hipStream_t)hip_stream;
    g->HW = cam->width * cam->height;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(nullptr, PG_ERR_NO_DEVICE, "hipGetDevice failed");
    }
    // LDS of the solve for a window of max_frames nodes with one fixed: the
    // packed Cholesky layout must fit; Gauss-Jordan is used where it fits
    int lds_max = 0;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device);
    g->lds_limit = lds_max - kSolveStaticLds;
    const size_t need = solve_lds_bytes(cfg->max_frames - 1, cfg->max_frames);
    if (need > (size_t)g->lds_limit ||
        (cfg->solver == PG_SOLVER_GAUSS_JORDAN && 6 * (cfg->max_frames - 1) > kGjMaxN) ||
        (cfg->solver == PG_SOLVER_LDL && 6 * (cfg->max_frames - 1) > kLdlMaxN) ||
        (cfg->solver == PG_SOLVER_PCG_MATRIX_FREE && cfg->max_frames > kMfMaxFrames)) {
        delete g;
        return fail(nullptr, PG_ERR_CAPACITY, "max_frames %d needs %zu B of LDS for the solve, device has %d",
                    cfg->max_frames, need, lds_max);
    }
    if (g->lds_limit > 65536 - kSolveStaticLds && solve_set_max_lds(g->lds_limit) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return fail(nullptr, PG_ERR_CAPACITY, "cannot raise the solve kernel's LDS limit to %d B", g->lds_limit);
    }
    const size_t M = cfg->max_frames, HW = g->HW;
    hipError_t e = hipSuccess;
    if ((e = g->depth.ensure(sizeof(float) * M * HW)) != hipSuccess ||
        (e = g->mask.ensure(M * HW)) != hipSuccess || (e = g->maps.ensure(sizeof(float4) * M * HW)) != hipSuccess ||
        (e = g->src_nz.ensure(sizeof(float4) * M * HW)) != hipSuccess ||
        (e = g->src_uv.ensure(sizeof(uint32_t) * M * HW)) != hipSuccess || (e = g->flag.ensure(HW)) != hipSuccess ||
        (e = g->rowcnt.ensure(sizeof(int) * cam->height)) != hipSuccess ||
        (e = g->total.ensure(sizeof(int))) != hipSuccess ||
        (e = g->d_result.ensure(sizeof(int) * 2 + sizeof(double) * (kIterRecord * kMaxIters + 16 * M))) !=
            hipSuccess ||
        (e = g->d_mlp.ensure(2 * 1320)) != hipSuccess ||
        (e = hipHostMalloc((void**)&g->h_status, sizeof(int) * 2 + sizeof(double) * (kIterRecord * kMaxIters + 32 * M))) !=
            hipSuccess) {
        pose_graph_destroy(g);
        return fail(nullptr, e == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP, "allocation: %s",
                    hipGetErrorString(e));
    }
    g->h_iters = g->h_status + 1;
    g->h_iter_stats = (double*)(g->h_status + 2);
    g->h_poses = g->h_iter_stats + kIterRecord * kMaxIters;
    g->h_up = g->h_poses + 16 * M;
    if ((e = hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&g->up_done, hipEventDisableTiming)) != hipSuccess) {
        pose_graph_destroy(g);
        return fail(nullptr, PG_ERR_HIP, "stream: %s", hipGetErrorString(e));
    }
    if ((e = hipMemsetAsync(g->d_result.p, 0, sizeof(int) * 2, g->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(g->stream)) != hipSuccess) {
        pose_graph_destroy(g);
        return fail(nullptr, PG_ERR_HIP, "init: %s", hipGetErrorString(e));
    }
    *out = g;
    return PG_OK;
}

pg_status pose_graph_add_frame(pg_graph* g, const float* depth_m, const uint8_t* mask, const double T[16], int fixed,
                               int* out_id)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (!depth_m || !mask || !T)
        return fail(g, PG_ERR_INVALID_ARG, "depth, mask and pose are required");
    if (!finite_pose(T))
        return fail(g, PG_ERR_INVALID_ARG, "pose is not a rigid transform");
    if (g->n_frames >= g->cfg.max_frames)
        return fail(g, PG_ERR_CAPACITY, "graph holds max_frames = %d frames", g->cfg.max_frames);
    const int f = g->n_frames;
    const size_t HW = g->HW;
    float* d = g->depth.as<float>() + f * HW;
    uint8_t* m = g->mask.as<uint8_t>() + f * HW;
    HIP_OR_FAIL(g, copy_in(d, depth_m, sizeof(float) * HW, g->stream));
    HIP_OR_FAIL(g, copy_in(m, mask, HW, g->stream));
    launch_preprocess(d, m, g->cam.width, g->cam.height, (float)g->cam.cx, (float)g->cam.cy, (float)(1.0 / g->cam.fx),
                      (float)(1.0 / g->cam.fy), g->maps.as<float4>() + f * HW, g->flag.as<uint8_t>(),
                      g->rowcnt.as<int>(), g->total.as<int>(), g->src_nz.as<float4>() + f * HW,
                      g->src_uv.as<uint32_t>() + f * HW, g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    int nv = 0;
    HIP_OR_FAIL(g, hipMemcpyAsync(&nv, g->total.p, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    g->n_frames = f + 1;
    g->fixed.push_back(fixed ? 1 : 0);
    g->n_src.push_back(nv);
    g->poses.insert(g->poses.end(), T, T + 16);
    g->poses_dirty = true;
    g->version++;
    if (out_id)
        *out_id = f;
    return PG_OK;
}

pg_status pose_graph_add_matches(pg_graph* g, int id_i, int id_j, const float* uv_i, const float* uv_j, int n)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (id_i < 0 || id_j < 0 || id_i >= g->n_frames || id_j >= g->n_frames || id_i == id_j)
        return fail(g, PG_ERR_INVALID_ARG, "bad node pair (%d, %d)", id_i, id_j);
    if (n < 0 || (n > 0 && (!uv_i || !uv_j)))
        return fail(g, PG_ERR_INVALID_ARG, "bad match arrays");
    if (id_i > id_j) {
        std::swap(id_i, id_j);
        std::swap(uv_i, uv_j);
    }
    const auto key = std::make_pair(id_i, id_j);
    g->version++;
    if (n == 0) {
        g->msets.erase(key);
        return PG_OK;
    }
    MatchSetHost& ms = g->msets[key];
    ms.i = id_i;
    ms.j = id_j;
    ms.n = n;
    DevBuf uvbuf;
    HIP_OR_FAIL(g, uvbuf.ensure(sizeof(float) * 4 * n));
    HIP_OR_FAIL(g, ms.pts.ensure(sizeof(float4) * 2 * n));
    float* ui = uvbuf.as<float>();
    float* uj = ui + 2 * n;
    HIP_OR_FAIL(g, copy_in(ui, uv_i, sizeof(float) * 2 * n, g->stream));
    HIP_OR_FAIL(g, copy_in(uj, uv_j, sizeof(float) * 2 * n, g->stream));
    const size_t HW = g->HW;
    launch_match_points(g->depth.as<float>() + id_i * HW, g->mask.as<uint8_t>() + id_i * HW,
                        g->depth.as<float>() + id_j * HW, g->mask.as<uint8_t>() + id_j * HW, g->cam.width,
                        g->cam.height, ui, uj, n, ms.pts.as<float4>(), g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    return PG_OK;
}

pg_status pose_graph_set_pose(pg_graph* g, int id, const double T[16])
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (id < 0 || id >= g->n_frames || !T)
        return fail(g, PG_ERR_INVALID_ARG, "bad node id %d", id);
    if (!finite_pose(T))
        return fail(g, PG_ERR_INVALID_ARG, "pose is not a rigid transform");
    memcpy(g->poses.data() + 16 * id, T, sizeof(double) * 16);
    g->poses_dirty = true;
    return PG_OK;
}

pg_status pose_graph_set_poses(pg_graph* g, int n, const double* T)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (n != g->n_frames || !T)
        return fail(g, PG_ERR_INVALID_ARG, "expected %d poses", g->n_frames);
    for (int k = 0; k < n; ++k)
        if (!finite_pose(T + 16 * k))
            return fail(g, PG_ERR_INVALID_ARG, "pose %d is not a rigid transform", k);
    memcpy(g->poses.data(), T, sizeof(double) * 16 * n);
    g->poses_dirty = true;
    return PG_OK;
}

pg_status pose_graph_get_pose(const pg_graph* g, int id, double T[16])
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (id < 0 || id >= g->n_frames || !T)
        return fail(const_cast<pg_graph*>(g), PG_ERR_INVALID_ARG, "bad node id %d", id);
    memcpy(T, g->poses.data() + 16 * id, sizeof(double) * 16);
    return PG_OK;
}

int pose_graph_num_frames(const pg_graph* g) { return g ? g->n_frames : 0; }

pg_status pose_graph_optimize(pg_graph* g, pg_stats* stats)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (!g->sched)
        g->sched.reset(new (std::nothrow) Schedule());
    if (!g->sched)
        return fail(g, PG_ERR_OUT_OF_MEMORY, "host allocation failed");
    pg_status r = prepare_graph(g);
    if (r != PG_OK)
        return r;
    if (g->sched->versions.empty() || g->sched->versions[0] != g->version) {
        r = build_schedule({g}, *g->sched);
        if (r != PG_OK)
            return r;
    }
    std::vector<pg_stats*> st{stats};
    return run_schedule(*g->sched, g->cfg.gn_iters, g->cfg.use_graph != 0, g->cfg.timing != 0, st);
}

pg_status pose_graph_optimize_batch(pg_graph* const* graphs, int n_graphs, pg_stats* stats)
{
    if (!graphs || n_graphs < 1)
        return fail(nullptr, PG_ERR_INVALID_ARG, "no graphs");
    std::vector<pg_graph*> gs(graphs, graphs + n_graphs);
    for (pg_graph* g : gs)
        if (!g)
            return fail(nullptr, PG_ERR_INVALID_ARG, "NULL graph in batch");
    pg_graph* g0 = gs[0];
    for (pg_graph* g : gs) {
        if (g->stream != g0->stream || g->device != g0->device)
            return fail(g0, PG_ERR_INVALID_ARG, "graphs of a batch must share one device and stream");
        if (g->cfg.gn_iters != g0->cfg.gn_iters)
            return fail(g0, PG_ERR_INVALID_ARG, "graphs of a batch must share gn_iters");
    }
    std::lock_guard<std::mutex> lk(g_batch_mutex);
    Schedule* s = nullptr;
    for (auto& c : g_batch_cache)
        if (c->graphs == gs) {
            s = c.get();
            break;
        }
    if (!s) {
        g_batch_cache.emplace_back(new Schedule());
        s = g_batch_cache.back().get();
        s->graphs = gs;
    }
    bool stale = s->versions.size() != gs.size();
    for (size_t k = 0; !stale && k < gs.size(); ++k)
        stale = s->versions[k] != gs[k]->version;
    if (stale) {
        pg_status r = build_schedule(gs, *s);
        if (r != PG_OK)
            return r;
    }
    std::vector<pg_stats*> st(gs.size(), nullptr);
    if (stats)
        for (int k = 0; k < n_graphs; ++k)
            st[k] = stats + k;
    return run_schedule(*s, g0->cfg.gn_iters, g0->cfg.use_graph != 0, g0->cfg.timing != 0, st);
}

pg_status pose_graph_linearize(pg_graph* g, double* H, double* grad, pg_stats* stats)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (!g->sched)
        g->sched.reset(new (std::nothrow) Schedule());
    pg_status r = prepare_graph(g);
    if (r != PG_OK)
        return r;
    if (g->sched->versions.empty() || g->sched->versions[0] != g->version) {
        r = build_schedule({g}, *g->sched);
        if (r != PG_OK)
            return r;
    }
    r = upload_poses(g);
    if (r != PG_OK)
        return r;
    Schedule& s = *g->sched;
    const GraphDev* gds = s.gds.as<GraphDev>();
    hipStream_t st = g->stream;
    launch_solve(gds, 1, s.lds, 1, st);
    launch_prune(gds, s.pitems.as<WorkItem>(), s.n_pitems, s.pframes.as<int2>(), s.n_pframes, s.max_src, st);
    launch_assoc(gds, s.items.as<WorkItem>(), s.n_items, s.ppt, s.precision, s.learned, 0, s.fitems.as<int2>(),
                 s.n_fitems, s.persistent ? s.ctr.as<unsigned>() : nullptr, s.persist_bpx, st);
    launch_assemble(gds, s.nbs.as<int2>(), s.n_nbs, st);
    HIP_OR_FAIL(g, hipGetLastError());
    const int N = g->n_frames;
    std::vector<double> ns(kNodeStats * N);
    if (H)
        HIP_OR_FAIL(g, hipMemcpyAsync(H, g->d_H.p, sizeof(double) * 36 * N * N, hipMemcpyDeviceToHost, st));
    if (grad)
        HIP_OR_FAIL(g, hipMemcpyAsync(grad, g->d_grad.p, sizeof(double) * 6 * N, hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(g, hipMemcpyAsync(ns.data(), g->d_node_stats.p, sizeof(double) * kNodeStats * N,
                                  hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(g, hipStreamSynchronize(st));
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        double ef = 0, eg = 0, cf = 0, cg = 0, rd = 0;
        for (int k = 0; k < N; ++k) {
            eg += ns[kNodeStats * k + 0];
            ef += ns[kNodeStats * k + 1];
            cg += ns[kNodeStats * k + 2];
            cf += ns[kNodeStats * k + 3];
            rd += ns[kNodeStats * k + 4];
        }
        stats->n_target_reads[0] = (long long)rd;
        stats->energy_f[0] = ef;
        stats->energy_g[0] = eg;
        stats->n_valid_g[0] = (long long)cg;
        stats->n_valid_f[0] = (long long)cf;
        long long sp = 0;
        for (int f = 0; f < N; ++f)
            sp += (long long)g->n_eff[f] * (N - 1);
        stats->src_pixels = sp;
    }
    return PG_OK;
}

pg_status pose_graph_associate(pg_graph* g, int i, int j, int32_t* target, float* r, float* uv)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (i < 0 || j < 0 || i >= g->n_frames || j >= g->n_frames || i == j)
        return fail(g, PG_ERR_INVALID_ARG, "bad node pair (%d, %d)", i, j);
    if (!g->sched)
        g->sched.reset(new (std::nothrow) Schedule());
    pg_status rc = prepare_graph(g);
    if (rc != PG_OK)
        return rc;
    if (g->sched->versions.empty() || g->sched->versions[0] != g->version) {
        rc = build_schedule({g}, *g->sched);
        if (rc != PG_OK)
            return rc;
    }
    rc = upload_poses(g);
    if (rc != PG_OK)
        return rc;
    Schedule& s = *g->sched;
    const size_t HW = g->HW;
    DevBuf out;
    HIP_OR_FAIL(g, out.ensure(HW * (sizeof(int) + 3 * sizeof(float))));
    int* dt = out.as<int>();
    float* dr = (float*)(dt + HW);
    float* duv = dr + HW;
    launch_solve(s.gds.as<GraphDev>(), 1, s.lds, 1, g->stream);
    launch_assoc_debug(s.gds.as<GraphDev>(), (int)HW, i, j, 0, dt, dr, duv, nullptr, nullptr, g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    if (target)
        HIP_OR_FAIL(g, hipMemcpyAsync(target, dt, HW * sizeof(int), hipMemcpyDeviceToHost, g->stream));
    if (r)
        HIP_OR_FAIL(g, hipMemcpyAsync(r, dr, HW * sizeof(float), hipMemcpyDeviceToHost, g->stream));
    if (uv)
        HIP_OR_FAIL(g, hipMemcpyAsync(uv, duv, 2 * HW * sizeof(float), hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    return PG_OK;
}

// tables and transforms of a single-graph schedule at the current poses
static pg_status ready_single(pg_graph* g)
{
    if (!g->sched)
        g->sched.reset(new (std::nothrow) Schedule());
    if (!g->sched)
        return fail(g, PG_ERR_OUT_OF_MEMORY, "host allocation failed");
    pg_status rc = prepare_graph(g);
    if (rc != PG_OK)
        return rc;
    if (g->sched->versions.empty() || g->sched->versions[0] != g->version) {
        rc = build_schedule({g}, *g->sched);
        if (rc != PG_OK)
            return rc;
    }
    rc = upload_poses(g);
    if (rc != PG_OK)
        return rc;
    launch_solve(g->sched->gds.as<GraphDev>(), 1, g->sched->lds, 1, g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    HIP_OR_FAIL(g, hipEventRecord(g->up_done, g->stream));   // the staging buffer is read until then
    return PG_OK;
}

pg_status pose_graph_pair_features(pg_graph* g, int i, int j, int iteration, float* features, float* sigma,
                                   int32_t* target)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (i < 0 || j < 0 || i >= g->n_frames || j >= g->n_frames || i == j)
        return fail(g, PG_ERR_INVALID_ARG, "bad node pair (%d, %d)", i, j);
    if (iteration < 0 || iteration >= PG_MAX_ITERS)
        return fail(g, PG_ERR_INVALID_ARG, "iteration %d out of [0, %d)", iteration, PG_MAX_ITERS);
    if (sigma && !g->has_mlp)
        return fail(g, PG_ERR_INVALID_ARG, "network weights need the parameters (pose_graph_set_mlp)");
    pg_status rc = ready_single(g);
    if (rc != PG_OK)
        return rc;
    const size_t HW = g->HW;
    // device outputs are written in place, host outputs through a staging buffer
    DevBuf stage;
    HIP_OR_FAIL(g, stage.ensure(HW * 8 * sizeof(float)));
    float* sf = stage.as<float>();
    float* ss = sf + 6 * HW;
    int* st = (int*)(ss + HW);
    float* df = features ? (is_device_ptr(features) ? features : sf) : nullptr;
    float* ds = sigma ? (is_device_ptr(sigma) ? sigma : ss) : nullptr;
    int* dt = target ? (is_device_ptr(target) ? (int*)target : st) : nullptr;
    launch_assoc_debug(g->sched->gds.as<GraphDev>(), (int)HW, i, j, iteration, dt, nullptr, nullptr, df, ds,
                       g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    if (features && df == sf)
        HIP_OR_FAIL(g, hipMemcpyAsync(features, sf, 6 * HW * sizeof(float), hipMemcpyDeviceToHost, g->stream));
    if (sigma && ds == ss)
        HIP_OR_FAIL(g, hipMemcpyAsync(sigma, ss, HW * sizeof(float), hipMemcpyDeviceToHost, g->stream));
    if (target && dt == st)
        HIP_OR_FAIL(g, hipMemcpyAsync(target, st, HW * sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    return PG_OK;
}

pg_status pg_set_tile_table(const int* entries, int n_entries)
{
    if (n_entries < 0 || n_entries > kTileTableMax || (n_entries > 0 && !entries))
        return fail(nullptr, PG_ERR_INVALID_ARG, "tile table: 0..%d entries of 5 ints", kTileTableMax);
    std::vector<TileClass> t;
    for (int k = 0; k < n_entries; ++k) {
        const int* e = entries + 5 * k;
        const TileClass c{e[0], e[1], e[2], e[3], e[4]};
        if (c.width <= 0 || c.height <= 0 || c.lo < 1 || c.hi < c.lo || c.tile < kAssocThreads ||
            c.tile > kTileMaxPixels || c.tile % kAssocThreads != 0)
            return fail(nullptr, PG_ERR_INVALID_ARG, "tile table entry %d invalid", k);
        t.push_back(c);
    }
    std::lock_guard<std::mutex> lk(g_tile_mutex);
    g_tile_table.swap(t);
    return PG_OK;
}

pg_status pose_graph_time_assoc(pg_graph* g, int reps, double* ms_per_launch)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (reps < 1 || reps > 10000 || !ms_per_launch)
        return fail(g, PG_ERR_INVALID_ARG, "reps must be 1..10000 and ms_per_launch non-NULL");
    pg_status rc = ready_single(g);
    if (rc != PG_OK)
        return rc;
    Schedule& s = *g->sched;
    const GraphDev* gds = s.gds.as<GraphDev>();
    launch_prune(gds, s.pitems.as<WorkItem>(), s.n_pitems, s.pframes.as<int2>(), s.n_pframes, s.max_src, g->stream);
    // one untimed launch, then reps back-to-back launches between two events
    launch_assoc(gds, s.items.as<WorkItem>(), s.n_items, s.ppt, s.precision, s.learned, 0, s.fitems.as<int2>(),
                 s.n_fitems, s.persistent ? s.ctr.as<unsigned>() : nullptr, s.persist_bpx, g->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OR_FAIL(g, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess)
        e = hipEventRecord(e0, g->stream);
    for (int k = 0; k < reps && e == hipSuccess; ++k) {
        launch_assoc(gds, s.items.as<WorkItem>(), s.n_items, s.ppt, s.precision, s.learned, 0, s.fitems.as<int2>(),
                     s.n_fitems, s.persistent ? s.ctr.as<unsigned>() : nullptr, s.persist_bpx, g->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, g->stream);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    HIP_OR_FAIL(g, e);
    *ms_per_launch = (double)ms / reps;
    return PG_OK;
}

pg_status pose_graph_prune(pg_graph* g, float* score, uint8_t* keep)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (g->cfg.weighting != PG_WEIGHT_LEARNED || !(g->cfg.prune_frac > 0.0))
        return fail(g, PG_ERR_INVALID_ARG, "pruning needs learned weighting and prune_frac > 0");
    pg_status rc = ready_single(g);
    if (rc != PG_OK)
        return rc;
    Schedule& s = *g->sched;
    launch_prune(s.gds.as<GraphDev>(), s.pitems.as<WorkItem>(), s.n_pitems, s.pframes.as<int2>(), s.n_pframes,
                 s.max_src, g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    const int N = g->n_frames;
    const size_t HW = g->HW, NHW = (size_t)N * HW;
    std::vector<uint32_t> uv(NHW), puv(NHW), sc(NHW);
    HIP_OR_FAIL(g, hipMemcpyAsync(uv.data(), g->src_uv.p, sizeof(uint32_t) * NHW, hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(g, hipMemcpyAsync(puv.data(), g->d_psrc_uv.p, sizeof(uint32_t) * NHW, hipMemcpyDeviceToHost,
                                  g->stream));
    HIP_OR_FAIL(g, hipMemcpyAsync(sc.data(), g->d_score.p, sizeof(uint32_t) * NHW, hipMemcpyDeviceToHost,
                                  g->stream));
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    const int W = g->cam.width;
    for (int f = 0; f < N; ++f) {
        const size_t b = (size_t)f * HW;
        if (score)
            for (size_t x = 0; x < HW; ++x)
                score[b + x] = -1.0f;
        if (keep)
            memset(keep + b, 0, HW);
        for (int k = 0; k < g->n_src[f]; ++k) {
            const uint32_t e = uv[b + k];
            const size_t x = (size_t)(e >> 16) * W + (e & 0xffffu);
            float v;
            memcpy(&v, &sc[b + k], sizeof(float));
            if (score)
                score[b + x] = v;
        }
        if (keep)
            for (int k = 0; k < g->n_eff[f]; ++k) {
                const uint32_t e = puv[b + k];
                keep[b + (size_t)(e >> 16) * W + (e & 0xffffu)] = 1;
            }
    }
    return PG_OK;
}

pg_status pose_graph_frame_info(pg_graph* g, int id, float* map, int* n_valid)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (id < 0 || id >= g->n_frames)
        return fail(g, PG_ERR_INVALID_ARG, "bad node id %d", id);
    if (n_valid)
        *n_valid = g->n_src[id];
    if (map) {
        HIP_OR_FAIL(g, hipMemcpyAsync(map, g->maps.as<float4>() + (size_t)id * g->HW, sizeof(float4) * g->HW,
                                      hipMemcpyDeviceToHost, g->stream));
        HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    }
    return PG_OK;
}

pg_status pose_graph_set_mlp(pg_graph* g, const void* params, size_t n_bytes)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (!params || n_bytes != 2626)
        return fail(g, PG_ERR_INVALID_ARG, "expected 1313 fp16 parameters (2626 bytes), got %zu bytes", n_bytes);
    HIP_OR_FAIL(g, copy_in(g->d_mlp.p, params, n_bytes, g->stream));
    HIP_OR_FAIL(g, g->d_mlp32.ensure(sizeof(float) * 1320));
    launch_mlp_to_float(g->d_mlp.as<__half>(), g->d_mlp32.as<float>(), g->stream);
    HIP_OR_FAIL(g, hipGetLastError());
    HIP_OR_FAIL(g, hipStreamSynchronize(g->stream));
    if (!g->has_mlp)
        g->version++;   // the parameter pointer enters the schedule's tables
    g->has_mlp = true;
    return PG_OK;
}

pg_status pose_graph_ransac(pg_graph* g, int n_pairs, const int* pi, const int* pj, const int* match_off,
                            const float* uv_i, const float* uv_j, int n_hyp, const int* samples, double delta_m,
                            double alpha_rad, int install, int* best, int* score, double* T, uint8_t* inlier)
{
    if (!g)
        return PG_ERR_INVALID_ARG;
    if (n_pairs < 1 || !pi || !pj || !match_off || !samples || !best || !T)
        return fail(g, PG_ERR_INVALID_ARG, "pairs, match offsets, samples, best and T are required");
    if (n_hyp < 1 || n_hyp > PG_RANSAC_MAX_HYP)
        return fail(g, n_hyp < 1 ? PG_ERR_INVALID_ARG : PG_ERR_CAPACITY, "n_hyp %d outside 1..%d", n_hyp,
                    PG_RANSAC_MAX_HYP);
    if (!(delta_m > 0.0) || !isfinite(delta_m) || !(alpha_rad > 0.0) || !(alpha_rad < M_PI))
        return fail(g, PG_ERR_INVALID_ARG, "delta must be positive and alpha in (0, pi)");
    std::vector<int4> pairs(n_pairs);
    for (int q = 0; q < n_pairs; ++q) {
        if (pi[q] < 0 || pj[q] < 0 || pi[q] >= g->n_frames || pj[q] >= g->n_frames || pi[q] == pj[q])
            return fail(g, PG_ERR_INVALID_ARG, "pair %d: bad node pair (%d, %d)", q, pi[q], pj[q]);
        const int n = match_off[q + 1] - match_off[q];
        if (match_off[q] < 0 || n < 0)
            return fail(g, PG_ERR_INVALID_ARG, "match offsets must be non-negative and non-decreasing");
        if (n > PG_RANSAC_MAX_MATCHES)
            return fail(g, PG_ERR_CAPACITY, "pair %d has %d matches, more than %d", q, n, PG_RANSAC_MAX_MATCHES);
        pairs[q] = make_int4(pi[q], pj[q], match_off[q], n);
    }
    const int total = match_off[n_pairs];
    if (total > 0 && (!uv_i || !uv_j))
        return fail(g, PG_ERR_INVALID_ARG, "match coordinates are required");
    const size_t nh = (size_t)n_pairs * n_hyp;
    DevBuf d_pairs, d_uv, d_samples, d_score, d_T, d_best, d_Tbest, d_inl;
    HIP_OR_FAIL(g, d_pairs.ensure(sizeof(int4) * n_pairs));
    HIP_OR_FAIL(g, d_uv.ensure(sizeof(float) * 4 * (size_t)std::max(total, 1)));
    HIP_OR_FAIL(g, d_samples.ensure(sizeof(int) * 3 * nh));
    HIP_OR_FAIL(g, d_score.ensure(sizeof(int) * nh));
    HIP_OR_FAIL(g, d_T.ensure(sizeof(double) * 12 * nh));
    HIP_OR_FAIL(g, d_best.ensure(sizeof(int) * n_pairs));
    HIP_OR_FAIL(g, d_Tbest.ensure(sizeof(double) * 16 * n_pairs));
    HIP_OR_FAIL(g, d_inl.ensure((size_t)std::max(total, 1)));
    hipStream_t st = g->stream;
    float* ui = d_uv.as<float>();
    float* uj = ui + 2 * (size_t)std::max(total, 1);
    HIP_OR_FAIL(g, hipMemcpyAsync(d_pairs.p, pairs.data(), sizeof(int4) * n_pairs, hipMemcpyHostToDevice, st));
    if (total > 0) {
        HIP_OR_FAIL(g, copy_in(ui, uv_i, sizeof(float) * 2 * total, st));
        HIP_OR_FAIL(g, copy_in(uj, uv_j, sizeof(float) * 2 * total, st));
    }
    HIP_OR_FAIL(g, copy_in(d_samples.p, samples, sizeof(int) * 3 * nh, st));
    HIP_OR_FAIL(g, launch_ransac(g->maps.as<float4>(), g->cam.width, g->cam.height, g->cam.fx, g->cam.fy,
                                 g->cam.cx, g->cam.cy, d_pairs.as<int4>(), n_pairs, ui, uj, d_samples.as<int>(),
                                 n_hyp, delta_m, cos(alpha_rad), d_score.as<int>(), d_T.as<double>(),
                                 d_best.as<int>(), d_Tbest.as<double>(), d_inl.as<unsigned char>(), st));
    std::vector<uint8_t> inl((size_t)std::max(total, 1));
    HIP_OR_FAIL(g, hipMemcpyAsync(best, d_best.p, sizeof(int) * n_pairs, hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(g, hipMemcpyAsync(T, d_Tbest.p, sizeof(double) * 16 * n_pairs, hipMemcpyDeviceToHost, st));
    if (score)
        HIP_OR_FAIL(g, hipMemcpyAsync(score, d_score.p, sizeof(int) * nh, hipMemcpyDeviceToHost, st));
    if (total > 0)
        HIP_OR_FAIL(g, hipMemcpyAsync(inl.data(), d_inl.p, total, hipMemcpyDeviceToHost, st));
    HIP_OR_FAIL(g, hipStreamSynchronize(st));
    if (inlier && total > 0)
        memcpy(inlier, inl.data(), total);
    if (install) {
        // the inlier coordinates, read back from the device copies (the
        // caller's arrays may be device memory)
        std::vector<float> hu(2 * (size_t)std::max(total, 1)), hv(2 * (size_t)std::max(total, 1));
        if (total > 0) {
            HIP_OR_FAIL(g, hipMemcpy(hu.data(), ui, sizeof(float) * 2 * total, hipMemcpyDeviceToHost));
            HIP_OR_FAIL(g, hipMemcpy(hv.data(), uj, sizeof(float) * 2 * total, hipMemcpyDeviceToHost));
        }
        for (int q = 0; q < n_pairs; ++q) {
            if (best[q] < 0)
                continue;
            std::vector<float> a, b;
            for (int m = match_off[q]; m < match_off[q + 1]; ++m)
                if (inl[m]) {
                    a.insert(a.end(), {hu[2 * m], hu[2 * m + 1]});
                    b.insert(b.end(), {hv[2 * m], hv[2 * m + 1]});
                }
            const pg_status r = pose_graph_add_matches(g, pi[q], pj[q], a.data(), b.data(), (int)(a.size() / 2));
            if (r != PG_OK)
                return r;
        }
    }
    return PG_OK;
}

const char* pose_graph_last_error(const pg_graph* g)
{
    return g ? g->err.c_str() : g_create_error.c_str();
}

void pose_graph_destroy(pg_graph* g)
{
    if (!g)
        return;
    {
        std::lock_guard<std::mutex> lk(g_batch_mutex);
        g_batch_cache.erase(std::remove_if(g_batch_cache.begin(), g_batch_cache.end(),
                                           [g](const std::unique_ptr<Schedule>& s) {
                                               return std::find(s->graphs.begin(), s->graphs.end(), g) !=
                                                      s->graphs.end();
                                           }),
                            g_batch_cache.end());
    }
    (void)hipStreamSynchronize(g->stream);
    g->sched.reset();
    if (g->capture_stream)
        (void)hipStreamDestroy(g->capture_stream);
    if (g->up_done)
        (void)hipEventDestroy(g->up_done);
    if (g->h_status)
        (void)hipHostFree(g->h_status);
    delete g;
}

}  // extern "C"
