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
#include "pg_frontend.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <mutex>
#include <string>

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

const char* pg_frontend_last_error(void) { return g_frontend_error.c_str(); }

}  // extern "C"
