// HIP kernels (gfx950) of the per-iteration linearisation of BundleTrack's
// online pose-graph optimisation (Wen & Bekris, IROS 2021), Sec. IV-D.
//
//   preprocess       per-frame vertex/normal map and the compact list of
//                    valid source pixels;
//   assoc_kernel     dense projective association, point-to-plane residual of
//                    Eq. (3), Jacobian, Huber IRLS weight and the per-item sum of
//                    w J_i^T J_i, w r J_i, energy, count and target reads (30 values);
//   feature_set      feature residual of Eq. (2): weighted second moments of
//                    (1, p_m, p_n) per match set, expanded exactly into the
//                    12x12 block and gradient of its 3x12 Jacobian (FP64), in
//                    the first blocks of the association launch;
//   prune_*          pruning of source pixels by the learned weight.
//
// The dense residual depends on the two poses only through A = T_i T_j^-1, so
// its Jacobian w.r.t. a left perturbation of T_j is minus the Jacobian w.r.t.
// T_i times the adjoint of A.  Each pixel-pair therefore only accumulates the
// 6x6 block w J_i^T J_i (21 unique values), w r J_i, rho and a count; the
// (i,j), (j,i) and (j,j) blocks follow in FP64 when the normal equations are
// assembled.
#include "pg_device.hpp"
#include "pg_mlp.hpp"
#include "pg_util.hpp"

#include <math.h>

namespace pg {

// ------------------------------------------------------------------ helpers

// nearest pixel with ties to the upper pixel, floor(x + 1/2) without the
// rounding of the addition
__device__ __forceinline__ float round_half_up(float x)
{
    const float f = floorf(x);
    return (x - f >= 0.5f) ? f + 1.0f : f;
}

__device__ __forceinline__ bool depth_ok(float z, uint8_t m) { return m != 0 && isfinite(z) && z > 0.0f; }

// ---------------------------------------------------- per-frame preprocessing

// Validity, back-projection pi_D^-1 at the pixel centre and the normal by
// central differences of the vertex map, oriented towards the camera.  A pixel
// is a source/target only with a valid normal (all four neighbours valid,
// not on the border).  Output: packed {nx, ny, nz, z}, zero when invalid.
__global__ void preprocess_map_kernel(const float* __restrict__ depth, const uint8_t* __restrict__ mask,
                                      int W, int H, float cx, float cy, float ifx, float ify,
                                      float4* __restrict__ map, uint8_t* __restrict__ flag)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= W || v >= H)
        return;
    const int x = v * W + u;
    const float z = depth[x];
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    uint8_t ok = 0;
    if (depth_ok(z, mask[x]) && u > 0 && v > 0 && u < W - 1 && v < H - 1) {
        const float zl = depth[x - 1], zr = depth[x + 1], zu = depth[x - W], zd = depth[x + W];
        if (depth_ok(zl, mask[x - 1]) && depth_ok(zr, mask[x + 1]) && depth_ok(zu, mask[x - W]) &&
            depth_ok(zd, mask[x + W])) {
            const float xu = (u - cx) * ifx, yv = (v - cy) * ify;
            const float xl = (u - 1 - cx) * ifx, xr = (u + 1 - cx) * ifx;
            const float yu = (v - 1 - cy) * ify, yd = (v + 1 - cy) * ify;
            // d/du: V(u+1,v) - V(u-1,v); d/dv: V(u,v+1) - V(u,v-1)
            const float ax = zr * xr - zl * xl, ay = zr * yv - zl * yv, az = zr - zl;
            const float bx = zd * xu - zu * xu, by = zd * yd - zu * yu, bz = zd - zu;
            float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
            const float len2 = nx * nx + ny * ny + nz * nz;
            if (len2 > 0.0f) {
                const float len = sqrtf(len2);
                nx /= len;
                ny /= len;
                nz /= len;
                if (nx * (z * xu) + ny * (z * yv) + nz * z > 0.0f) {
                    nx = -nx;
                    ny = -ny;
                    nz = -nz;
                }
                out = make_float4(nx, ny, nz, z);
                ok = 1;
            }
        }
    }
    map[x] = out;
    flag[x] = ok;
}

__global__ void row_count_kernel(const uint8_t* __restrict__ flag, int W, int* __restrict__ row_cnt)
{
    __shared__ int part[4];
    const int v = blockIdx.x;
    int c = 0;
    for (int u = threadIdx.x; u < W; u += blockDim.x)
        c += flag[v * W + u];
    for (int o = 32; o > 0; o >>= 1)
        c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        row_cnt[v] = part[0] + part[1] + part[2] + part[3];
}

// Exclusive prefix sum of v over the block (up to 1024 threads) and the block total.
__device__ __forceinline__ int block_excl_scan_int(int v, int* wave_sums, int& total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += o;
    }
    if (lane == 63)
        wave_sums[wv] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        const int c = wave_sums[w];
        off += (w < wv) ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;   // rows per thread: up to 8192 rows

// Exclusive prefix sum of the per-row counts (in place) and their total.
__global__ __launch_bounds__(kScanThreads) void row_scan_kernel(int* __restrict__ row_cnt, int H,
                                                                  int* __restrict__ total)
{
    __shared__ int wave_sums[kScanThreads / 64];
    const int r0 = threadIdx.x * kScanPer;
    int c[kScanPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        c[q] = (r0 + q < H) ? row_cnt[r0 + q] : 0;
        sum += c[q];
    }
    int tot;
    int off = block_excl_scan_int(sum, wave_sums, tot);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (r0 + q < H)
            row_cnt[r0 + q] = off;
        off += c[q];
    }
    if (threadIdx.x == 0)
        *total = tot;
}

// row-major compaction of the valid pixels: the source list of a frame
__global__ void row_scatter_kernel(const float4* __restrict__ map, const uint8_t* __restrict__ flag,
                                   const int* __restrict__ row_off, int W, float4* __restrict__ src_nz,
                                   uint32_t* __restrict__ src_uv)
{
    __shared__ int wave_cnt[4];
    const int v = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int base = row_off[v];
    for (int u0 = 0; u0 < W; u0 += 256) {
        const int u = u0 + threadIdx.x;
        const bool f = (u < W) && flag[v * W + u];
        const unsigned long long bal = __ballot(f);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0)
            wave_cnt[wv] = __popcll(bal);
        __syncthreads();
        int off = base, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wv)
                off += wave_cnt[w];
            tot += wave_cnt[w];
        }
        if (f) {
            src_nz[off + pre] = map[v * W + u];
            src_uv[off + pre] = (uint32_t)u | ((uint32_t)v << 16);
        }
        __syncthreads();
        base += tot;
    }
}

// ------------------------------------------------------------ feature points

__device__ __forceinline__ bool match_point(const float* __restrict__ depth, const uint8_t* __restrict__ mask,
                                            int W, int H, float u, float v, float4& p)
{
    const float ui = round_half_up(u), vi = round_half_up(v);
    p = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!(ui >= 0.f && ui < (float)W && vi >= 0.f && vi < (float)H))
        return false;
    const int x = (int)vi * W + (int)ui;
    const float z = depth[x];
    if (!depth_ok(z, mask[x]))
        return false;
    p = make_float4(ui, vi, z, 1.0f);
    return true;
}

// Endpoints of each match: the nearest pixel and its depth, {u, v, z, valid};
// valid = 1 when both endpoints have depth, else the match is inert.  The
// feature kernel back-projects them in FP64.
__global__ void match_points_kernel(const float* __restrict__ depth_i, const uint8_t* __restrict__ mask_i,
                                    const float* __restrict__ depth_j, const uint8_t* __restrict__ mask_j,
                                    int W, int H, const float* __restrict__ uv_i, const float* __restrict__ uv_j,
                                    int n, float4* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    float4 pm, pn;
    const bool a = match_point(depth_i, mask_i, W, H, uv_i[2 * k], uv_i[2 * k + 1], pm);
    const bool b = match_point(depth_j, mask_j, W, H, uv_j[2 * k], uv_j[2 * k + 1], pn);
    const float ok = (a && b) ? 1.0f : 0.0f;
    pm.w = ok;
    pn.w = ok;
    out[2 * k] = pm;
    out[2 * k + 1] = pn;
}

// one feature match set by one block (defined with the feature residuals);
// the association kernels run it in their first blocks
__device__ __forceinline__ void feature_set(const GraphDev* __restrict__ gds, int2 fi);

// ------------------------------------------------------ dense association

// Project source point p (frame-i camera) into frame j with B = T_j T_i^-1:
// returns the nearest target pixel packed as u | v << 16, or -2 (behind the
// camera) / -3 (outside the image); (uf, vf) is the continuous projection.
template <typename Cam>
__device__ __forceinline__ int project_px(const float (&B)[12], float px, float py, float pz, const Cam& gd,
                                          float& uf, float& vf)
{
    const float qx = fmaf(B[0], px, fmaf(B[1], py, fmaf(B[2], pz, B[3])));
    const float qy = fmaf(B[4], px, fmaf(B[5], py, fmaf(B[6], pz, B[7])));
    const float qz = fmaf(B[8], px, fmaf(B[9], py, fmaf(B[10], pz, B[11])));
    uf = __builtin_nanf("");
    vf = uf;
    if (!(qz > 0.0f))
        return -2;
    const float iz = 1.0f / qz;
    uf = fmaf(gd.fx * qx, iz, gd.cx);
    vf = fmaf(gd.fy * qy, iz, gd.cy);
    const float ui = round_half_up(uf), vi = round_half_up(vf);
    if (!(ui >= 0.0f && ui < (float)gd.W && vi >= 0.0f && vi < (float)gd.H))
        return -3;
    return (int)ui | ((int)vi << 16);
}

// loads through the global address space (global_load instead of flat_load)
// The graph constants of the per-pixel projection and gating, read once into
// scalar registers (the same names as in GraphDev, so the helpers above take
// either): kept as opaque values, they are not reloaded under every pixel's
// branch.
struct PixelConsts {
    float fx, fy, cx, cy, ifx, ify, gate_cos, gate_d2;
    int W, H;
};

__device__ __forceinline__ PixelConsts pixel_consts(const GraphDev& gd)
{
    PixelConsts c{gd.fx, gd.fy, gd.cx, gd.cy, gd.ifx, gd.ify, gd.gate_cos, gd.gate_d2, gd.W, gd.H};
    asm volatile("" : "+s"(c.fx), "+s"(c.fy), "+s"(c.cx), "+s"(c.cy), "+s"(c.ifx), "+s"(c.ify));
    asm volatile("" : "+s"(c.gate_cos), "+s"(c.gate_d2), "+s"(c.W), "+s"(c.H));
    return c;
}

// row-major index of a packed pixel (u | v << 16)
__device__ __forceinline__ int px_index(int pk, int W) { return (pk >> 16) * W + (pk & 0xffff); }

// Finish the association with the gathered target t = {n_q, z_q} of the
// packed pixel pk: -4 invalid target, -5 distance gate, -6 normal gate; else
// returns pk with the residual r = n . (A q - p) and J_i = [n, s x n] (s = A q).
template <typename Cam>
__device__ __forceinline__ int finish_px(const float (&A)[12], float px, float py, float pz, float nx, float ny,
                                         float nz, int pk, float4 t, const Cam& gd, float& r,
                                         float (&J)[6], float& d2_out, float& c_out, float& sn_out)
{
    if (!(t.w > 0.0f))
        return -4;
    const int ui = pk & 0xffff, vi = pk >> 16;
    const float qz = t.w;
    const float qx = qz * (((float)ui - gd.cx) * gd.ifx);
    const float qy = qz * (((float)vi - gd.cy) * gd.ify);
    const float sx = fmaf(A[0], qx, fmaf(A[1], qy, fmaf(A[2], qz, A[3])));
    const float sy = fmaf(A[4], qx, fmaf(A[5], qy, fmaf(A[6], qz, A[7])));
    const float sz = fmaf(A[8], qx, fmaf(A[9], qy, fmaf(A[10], qz, A[11])));
    const float dx = sx - px, dy = sy - py, dz = sz - pz;
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    d2_out = d2;
    c_out = 0.0f;
    sn_out = 0.0f;
    if (!(d2 < gd.gate_d2))
        return -5;
    const float rnx = fmaf(A[0], t.x, fmaf(A[1], t.y, A[2] * t.z));
    const float rny = fmaf(A[4], t.x, fmaf(A[5], t.y, A[6] * t.z));
    const float rnz = fmaf(A[8], t.x, fmaf(A[9], t.y, A[10] * t.z));
    const float c = fmaf(nx, rnx, fmaf(ny, rny, nz * rnz));
    c_out = c;
    {
        // |n x R n_q|: with the cosine, the angle between the normals as atan2
        // (well conditioned near 0, unlike acos of the cosine)
        const float ex = ny * rnz - nz * rny, ey = nz * rnx - nx * rnz, ez = nx * rny - ny * rnx;
        sn_out = sqrtf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
    }
    if (!(c > gd.gate_cos))
        return -6;
    r = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
    J[0] = nx;
    J[1] = ny;
    J[2] = nz;
    J[3] = sy * nz - sz * ny;
    J[4] = sz * nx - sx * nz;
    J[5] = sx * ny - sy * nx;
    return pk;
}

// ------------------------------------------------ learned weighting network

// Features of a gated-in pixel-pair: r / huber_g, normal angle / 30 deg
// (from its cosine c and sine sn), source depth / 0.8 m, pixel radius /
// half-diagonal, |s - p| / gate_dist, iteration / (iterations - 1).
__device__ __forceinline__ void learned_features(const GraphDev& gd, float r, float d2, float c, float sn, float z,
                                                 uint32_t uv, int iteration, float (&f)[6])
{
    const float u = (float)(uv & 0xffffu) - gd.cx, v = (float)(uv >> 16) - gd.cy;
    f[0] = r / gd.huber_g;
    f[1] = atan2f(sn, c) * (6.0f / 3.14159265358979f);
    f[2] = z * (1.0f / 0.8f);
    f[3] = sqrtf(u * u + v * v) * gd.inv_halfdiag;
    f[4] = sqrtf(d2) / gd.gate_dist;
    f[5] = (float)iteration * gd.inv_iters;
}


// Value of v held by the partner lane across lane bit B (partner = lane ^
// (1 << B)): DPP quad permutations for bits 0 and 1, a row rotation by 8 for
// bit 3, bit-mask swizzles for bits 2 and 4, a permute for bit 5.
template <int B>
__device__ __forceinline__ float lane_swap_f32(float v)
{
    const int x = __float_as_int(v);
    if constexpr (B == 0)
        return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));    // quad_perm [1, 0, 3, 2]
    else if constexpr (B == 1)
        return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));    // quad_perm [2, 3, 0, 1]
    else if constexpr (B == 3)
        return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false));   // row_ror 8
    else if constexpr (B == 2 || B == 4)
        return __int_as_float(__builtin_amdgcn_ds_swizzle(x, 0x1F | ((1 << B) << 10)));
    else
        return __shfl_xor(v, 1 << B);
}

// One recursive-halving level over lane bit B (lanes with the bit clear keep
// values [0, HALF), the others [HALF, 2 HALF), moved to acc[0, HALF)).
template <int HALF, int B>
__device__ __forceinline__ void halve_bit_f32(float (&acc)[32], int lane)
{
    const bool up = (lane >> B) & 1;
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        const float send = up ? acc[q] : acc[q + HALF];
        const float keep = up ? acc[q + HALF] : acc[q];
        acc[q] = keep + lane_swap_f32<B>(send);
    }
}

// Sum acc[0..31] over the wave: lane l < 32 ends with the total of value
// 16 b0 + 8 b1 + 4 b3 + 2 b2 + b4 (b the bits of l) in acc[0].
__device__ __forceinline__ int wave_sum32_f32(float (&acc)[32], int lane)
{
    halve_bit_f32<16, 0>(acc, lane);
    halve_bit_f32<8, 1>(acc, lane);
    halve_bit_f32<4, 3>(acc, lane);
    halve_bit_f32<2, 2>(acc, lane);
    halve_bit_f32<1, 4>(acc, lane);
    acc[0] += lane_swap_f32<5>(acc[0]);
    return 16 * (lane & 1) + 8 * ((lane >> 1) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) + ((lane >> 4) & 1);
}

// One work item per block: PPT source pixels per thread of one frame-i tile,
// associated into frame j.  Blocks are mapped so that each XCD (blockIdx mod
// 8) walks a contiguous run of the item list, which is ordered source tile
// first: the items that re-read one source tile share an L2.
template <int PPT, bool LEARNED>
__device__ __forceinline__ void assoc_item(const GraphDev* __restrict__ gds, const WorkItem it, int iteration)
{
    const int gid = it.gij >> 16, i = it.gij & 0xff, j = (it.gij >> 8) & 0xff;
    const GraphDev& gd = gds[gid];
    // the graph status is loaded with the first reads and tested before the
    // sums are reduced (one memory round trip fewer ahead of the source
    // loads); every read below is in bounds whatever it holds
    const int status = *gd.status;
    const int p = pair_index(i, j, gd.n_frames);
    float A[12], B[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        A[k] = gd.xf32[p * 24 + k];
        B[k] = gd.xf32[p * 24 + 12 + k];
    }
    const float4* __restrict__ src_nz = (LEARNED ? gd.psrc_nz : gd.src_nz) + (size_t)i * gd.HW;
    const uint32_t* __restrict__ src_uv = (LEARNED ? gd.psrc_uv : gd.src_uv) + (size_t)i * gd.HW;
    const float4* __restrict__ tmap = gd.maps + (size_t)j * gd.HW;
    const float huber = gd.huber_g;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // learned weighting: network operands (registers) and output-layer constants (LDS)
    __shared__ __attribute__((aligned(16))) float s_tail[kMlpTail];
    MlpFrags M;   // loaded after the source records are in flight (one memory round trip)

    float acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k)
        acc[k] = 0.0f;

    // phase 1: source records; phase 2: projections and target gathers;
    // phase 3: residuals and accumulation (loads of all PPT pixels in flight)
    float4 s[PPT];
    float px[PPT], py[PPT];
    int y[PPT];
    uint32_t uvs[PPT];
    const int end = it.start + it.count;   // count >= 1
    // every source load in flight before the first projection: unconditional
    // loads from a clamped (in-bounds) index, the pixels past the end dropped
    // afterwards (a load under the per-pixel branch would wait for the
    // previous pixel's projection)
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int k = it.start + threadIdx.x + m * kAssocThreads;
        const int kc = (k < end) ? k : end - 1;
        s[m] = ld_global(src_nz + kc);
        uvs[m] = ld_global(src_uv + kc);
    }
    if (LEARNED) {
        mlp_tail_load(gd.mlp32, s_tail);
        mlp_frags_load(gd.mlp32, M, lane);
        __syncthreads();
    }
    const PixelConsts pc = pixel_consts(gd);   // after the loads are issued
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int k = it.start + threadIdx.x + m * kAssocThreads;
        y[m] = -1;
        px[m] = py[m] = 0.f;
        if (k >= end) {
            s[m] = make_float4(0.f, 0.f, 0.f, 0.f);
            uvs[m] = 0;
        } else {
            const uint32_t uv = uvs[m];
            const float z = s[m].w;
            px[m] = z * (((float)(uv & 0xffffu) - pc.cx) * pc.ifx);
            py[m] = z * (((float)(uv >> 16) - pc.cy) * pc.ify);
            float uf, vf;
            y[m] = project_px(B, px[m], py[m], z, pc, uf, vf);
        }
    }
    float4 t[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        t[m] = (y[m] >= 0) ? ld_global(tmap + px_index(y[m], pc.W)) : make_float4(0.f, 0.f, 0.f, 0.f);
        acc[29] += (y[m] >= 0) ? 1.0f : 0.0f;
    }
    if constexpr (LEARNED) {
        // the network runs wave-wide on the wave's gated-in pixel-pairs only:
        // their features are packed in LDS (in pixel order), evaluated 64 at a
        // time, and each pair's output read back from its slot.  A sample's
        // output does not depend on the others of its batch, so packing
        // changes no result.
        __shared__ float s_feat[kAssocThreads / 64][kMlpIn][64 * PPT];
        __shared__ float s_sig[kAssocThreads / 64][64 * PPT];
        float rr[PPT], JJ[PPT][6];
        int slot[PPT];
        int nw = 0;   // gated-in pixel-pairs of the wave so far (uniform)
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            float d2 = 0.f, cg = 0.f, sn = 0.f;
            rr[m] = 0.f;
#pragma unroll
            for (int a = 0; a < 6; ++a)
                JJ[m][a] = 0.f;
            bool gated = false;
            if (y[m] >= 0)
                gated = finish_px(A, px[m], py[m], s[m].w, s[m].x, s[m].y, s[m].z, y[m], t[m], pc, rr[m], JJ[m], d2,
                                  cg, sn) >= 0;
            const unsigned long long bal = __ballot(gated);
            slot[m] = gated ? nw + __popcll(bal & below) : -1;
            if (gated) {
                float f[kMlpIn];
                learned_features(gd, rr[m], d2, cg, sn, s[m].w, uvs[m], iteration, f);
#pragma unroll
                for (int k = 0; k < kMlpIn; ++k)
                    s_feat[wave][k][slot[m]] = f[k];
            }
            nw += __popcll(bal);
        }
        // the wave reads back its own LDS writes (in order within a wavefront)
        asm volatile("" ::: "memory");
        for (int b0 = 0; b0 < nw; b0 += 64) {
            const int q = b0 + lane;
            float f[kMlpIn];
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k)
                f[k] = (q < nw) ? s_feat[wave][k][q] : 0.f;
            const float sgv = mlp_sigma_wave(M, s_tail, f, lane);
            if (q < nw)
                s_sig[wave][q] = sgv;
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            if (slot[m] < 0)
                continue;
            const float sg = s_sig[wave][slot[m]];
            const float r = rr[m];
            const float ar = fabsf(r);
            const float w = ((ar <= huber) ? 1.0f : huber * __builtin_amdgcn_rcpf(ar)) * sg;
            const float e = ((ar <= huber) ? 0.5f * ar * ar : huber * (ar - 0.5f * huber)) * sg;
            float wJ[6];
#pragma unroll
            for (int a = 0; a < 6; ++a)
                wJ[a] = w * JJ[m][a];
            int q = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a)
#pragma unroll
                for (int c = a; c < 6; ++c)
                    acc[q++] += wJ[a] * JJ[m][c];
#pragma unroll
            for (int a = 0; a < 6; ++a)
                acc[21 + a] += wJ[a] * r;
            acc[27] += e;
            acc[28] += 1.0f;
        }
    } else {
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        float r = 0.f, J[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, d2 = 0.f, cg = 0.f, sn = 0.f;
        bool gated = false;
        if (y[m] >= 0)
            gated = finish_px(A, px[m], py[m], s[m].w, s[m].x, s[m].y, s[m].z, y[m], t[m], pc, r, J, d2, cg, sn) >= 0;
        float sg = 1.0f;
        if (!gated)
            continue;
        const float ar = fabsf(r);
        const float w = ((ar <= huber) ? 1.0f : huber * __builtin_amdgcn_rcpf(ar)) * sg;
        const float e = ((ar <= huber) ? 0.5f * ar * ar : huber * (ar - 0.5f * huber)) * sg;
        float wJ[6];
#pragma unroll
        for (int a = 0; a < 6; ++a)
            wJ[a] = w * J[a];
        int q = 0;
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int c = a; c < 6; ++c)
                acc[q++] += wJ[a] * J[c];
#pragma unroll
        for (int a = 0; a < 6; ++a)
            acc[21 + a] += wJ[a] * r;
        acc[27] += e;
        acc[28] += 1.0f;
    }
    }
    if (status)   // uniform over the block
        return;

    const int vidx = wave_sum32_f32(acc, lane);
    __shared__ float red[kAssocThreads / 64][32];
    if (lane < 32)
        red[wave][vidx] = acc[0];
    __syncthreads();
    if (threadIdx.x < 32) {
        float v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kAssocThreads / 64; ++w)
            v += red[w][threadIdx.x];
        gd.partials[(size_t)it.slot * kDenseStride + threadIdx.x] = v;
    }
}

template <int PPT, bool LEARNED>
__global__ __launch_bounds__(kAssocThreads) void assoc_kernel(const GraphDev* __restrict__ gds,
                                                              const WorkItem* __restrict__ items, int n_items,
                                                              int per_xcd, int iteration,
                                                              const int2* __restrict__ fitems, int n_fitems)
{
    // the first blocks (a multiple of 8) take the feature match sets
    const int nf8 = (n_fitems + 7) & ~7;
    if ((int)blockIdx.x < nf8) {
        if ((int)blockIdx.x < n_fitems)
            feature_set(gds, fitems[blockIdx.x]);
        return;
    }
    const int b = blockIdx.x - nf8;
    const int L = (b & 7) * per_xcd + (b >> 3);
    if (L >= n_items)
        return;
    assoc_item<PPT, LEARNED>(gds, items[L], iteration);
}

// ------------------------------------------- BF16x3 split-precision MFMA form

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Same association, residual and weight as assoc_kernel; the 6x6 sums
// w J_i^T J_i and w r J_i come from matrix cores instead: each pixel's
// x = sqrt(w) [J_i, r] (padded to 16) is split into bf16 hi = rn(x) and
// lo = rn(x - hi), a wave's 64 pixels are transposed through LDS, and
// v_mfma_f32_16x16x32_bf16 accumulates X_hi^T X_hi + X_hi^T X_lo + X_lo^T X_hi
// in FP32 (the dropped X_lo^T X_lo term and the two splits bound the relative
// error of each product by about 3 * 2^-16).  For X^T X the A and B operands
// of the instruction coincide: lane l holds feature l % 16 of the 8 pixels
// 8 (l / 16) .. 8 (l / 16) + 7 of a 32-pixel half.  Energy and counts stay on
// the VALU.  The partial record has the same layout as assoc_kernel's.
template <int PPT, bool LEARNED>
__device__ __forceinline__ void assoc_bf16x3_item(const GraphDev* __restrict__ gds, const WorkItem it, int iteration)
{
    const int gid = it.gij >> 16, i = it.gij & 0xff, j = (it.gij >> 8) & 0xff;
    const GraphDev& gd = gds[gid];
    // the graph status is loaded with the first reads and tested before the
    // sums are reduced (one memory round trip fewer ahead of the source
    // loads); every read below is in bounds whatever it holds
    const int status = *gd.status;
    const int p = pair_index(i, j, gd.n_frames);
    float A[12], B[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        A[k] = gd.xf32[p * 24 + k];
        B[k] = gd.xf32[p * 24 + 12 + k];
    }
    const float4* __restrict__ src_nz = (LEARNED ? gd.psrc_nz : gd.src_nz) + (size_t)i * gd.HW;
    const uint32_t* __restrict__ src_uv = (LEARNED ? gd.psrc_uv : gd.src_uv) + (size_t)i * gd.HW;
    const float4* __restrict__ tmap = gd.maps + (size_t)j * gd.HW;
    const float huber = gd.huber_g;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // learned weighting: network operands (registers) and output-layer constants (LDS)
    __shared__ __attribute__((aligned(16))) float s_tail[kMlpTail];
    MlpFrags M;   // loaded after the source records are in flight (one memory round trip)
    // per wave: [hi, lo][16 features][64 pixels]
    __shared__ __attribute__((aligned(16))) __bf16 stage[kAssocThreads / 64][2][16][64];
    for (int e = lane; e < 2 * 9 * 64; e += 64)
        stage[wave][e / (9 * 64)][7 + (e / 64) % 9][e % 64] = (__bf16)0.0f;

    float4 s[PPT];
    float px[PPT], py[PPT];
    int y[PPT];
    uint32_t uvs[PPT];
    const int end = it.start + it.count;   // count >= 1
    // every source load in flight before the first projection: unconditional
    // loads from a clamped (in-bounds) index, the pixels past the end dropped
    // afterwards (a load under the per-pixel branch would wait for the
    // previous pixel's projection)
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int k = it.start + threadIdx.x + m * kAssocThreads;
        const int kc = (k < end) ? k : end - 1;
        s[m] = ld_global(src_nz + kc);
        uvs[m] = ld_global(src_uv + kc);
    }
    if (LEARNED) {
        mlp_tail_load(gd.mlp32, s_tail);
        mlp_frags_load(gd.mlp32, M, lane);
        __syncthreads();
    }
    const PixelConsts pc = pixel_consts(gd);   // after the loads are issued
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int k = it.start + threadIdx.x + m * kAssocThreads;
        y[m] = -1;
        px[m] = py[m] = 0.f;
        if (k >= end) {
            s[m] = make_float4(0.f, 0.f, 0.f, 0.f);
            uvs[m] = 0;
        } else {
            const uint32_t uv = uvs[m];
            const float z = s[m].w;
            px[m] = z * (((float)(uv & 0xffffu) - pc.cx) * pc.ifx);
            py[m] = z * (((float)(uv >> 16) - pc.cy) * pc.ify);
            float uf, vf;
            y[m] = project_px(B, px[m], py[m], z, pc, uf, vf);
        }
    }
    float4 t[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m)
        t[m] = (y[m] >= 0) ? ld_global(tmap + px_index(y[m], pc.W)) : make_float4(0.f, 0.f, 0.f, 0.f);

    float energy = 0.f, count = 0.f, reads = 0.f;
    f32x4 C = {0.f, 0.f, 0.f, 0.f};
    // learned weighting: the network on the wave's gated-in pixel-pairs only,
    // packed in LDS and evaluated 64 at a time before the contraction (as in
    // the FP32 association)
    float rr[PPT], JJ[PPT][6];
    int slot[PPT];
    __shared__ float s_feat[kAssocThreads / 64][kMlpIn][64 * PPT];   // learned only
    if constexpr (LEARNED) {
        int nw = 0;
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            float d2 = 0.f, cg = 0.f, sn = 0.f;
            rr[m] = 0.f;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                JJ[m][q] = 0.f;
            bool gated = false;
            if (y[m] >= 0) {
                reads += 1.0f;
                gated = finish_px(A, px[m], py[m], s[m].w, s[m].x, s[m].y, s[m].z, y[m], t[m], pc, rr[m], JJ[m], d2,
                                  cg, sn) >= 0;
            }
            const unsigned long long bal = __ballot(gated);
            slot[m] = gated ? nw + __popcll(bal & below) : -1;
            if (gated) {
                float f[kMlpIn];
                learned_features(gd, rr[m], d2, cg, sn, s[m].w, uvs[m], iteration, f);
#pragma unroll
                for (int k = 0; k < kMlpIn; ++k)
                    s_feat[wave][k][slot[m]] = f[k];
            }
            nw += __popcll(bal);
        }
        // the wave reads back its own LDS writes (in order within a wavefront);
        // each output goes to the slot of its features
        asm volatile("" ::: "memory");
        for (int b0 = 0; b0 < nw; b0 += 64) {
            const int q = b0 + lane;
            float f[kMlpIn];
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k)
                f[k] = (q < nw) ? s_feat[wave][k][q] : 0.f;
            const float sgv = mlp_sigma_wave(M, s_tail, f, lane);
            if (q < nw)
                s_feat[wave][0][q] = sgv;
        }
        asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        float x[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float r = 0.f, J[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, d2 = 0.f, cg = 0.f, sn = 0.f;
        bool gated = false;
        float sg = 1.0f;
        if constexpr (LEARNED) {
            gated = slot[m] >= 0;
            r = rr[m];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                J[q] = JJ[m][q];
            if (gated)
                sg = s_feat[wave][0][slot[m]];
        } else if (y[m] >= 0) {
            reads += 1.0f;
            gated = finish_px(A, px[m], py[m], s[m].w, s[m].x, s[m].y, s[m].z, y[m], t[m], pc, r, J, d2, cg, sn) >= 0;
        }
        if (gated) {
            const float ar = fabsf(r);
            const float w = ((ar <= huber) ? 1.0f : huber * __builtin_amdgcn_rcpf(ar)) * sg;
            energy += ((ar <= huber) ? 0.5f * ar * ar : huber * (ar - 0.5f * huber)) * sg;
            count += 1.0f;
            const float sw = sqrtf(w);
#pragma unroll
            for (int a = 0; a < 6; ++a)
                x[a] = sw * J[a];
            x[6] = sw * r;
        }
#pragma unroll
        for (int f = 0; f < 7; ++f) {
            const __bf16 hi = (__bf16)x[f];
            stage[wave][0][f][lane] = hi;
            stage[wave][1][f][lane] = (__bf16)(x[f] - (float)hi);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int f = lane & 15, p0 = 32 * c + 8 * (lane >> 4);
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&stage[wave][0][f][p0]);
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(&stage[wave][1][f][p0]);
            C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ah, C, 0, 0, 0);
            C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, al, C, 0, 0, 0);
            C = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, ah, C, 0, 0, 0);
        }
    }
    if (status)   // uniform over the block
        return;
    for (int o = 32; o > 0; o >>= 1) {
        energy += __shfl_xor(energy, o);
        count += __shfl_xor(count, o);
        reads += __shfl_xor(reads, o);
    }
    __shared__ float red[kAssocThreads / 64][32];
    // lane l holds D[4 (l / 16) + r][l % 16] in C[r]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ii = 4 * (lane >> 4) + r, jj = lane & 15;
        if (ii <= jj && jj < 6)
            red[wave][upper_index(ii, jj, 6)] = C[r];
        else if (jj == 6 && ii < 6)
            red[wave][21 + ii] = C[r];
    }
    if (lane == 0) {
        red[wave][27] = energy;
        red[wave][28] = count;
        red[wave][29] = reads;
        red[wave][30] = 0.f;
        red[wave][31] = 0.f;
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        float v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kAssocThreads / 64; ++w)
            v += red[w][threadIdx.x];
        gd.partials[(size_t)it.slot * kDenseStride + threadIdx.x] = v;
    }
}

template <int PPT, bool LEARNED>
__global__ __launch_bounds__(kAssocThreads) void assoc_bf16x3_kernel(const GraphDev* __restrict__ gds,
                                                                     const WorkItem* __restrict__ items,
                                                                     int n_items, int per_xcd, int iteration,
                                                                     const int2* __restrict__ fitems, int n_fitems)
{
    // the first blocks (a multiple of 8) take the feature match sets
    const int nf8 = (n_fitems + 7) & ~7;
    if ((int)blockIdx.x < nf8) {
        if ((int)blockIdx.x < n_fitems)
            feature_set(gds, fitems[blockIdx.x]);
        return;
    }
    const int b = blockIdx.x - nf8;
    const int L = (b & 7) * per_xcd + (b >> 3);
    if (L >= n_items)
        return;
    assoc_bf16x3_item<PPT, LEARNED>(gds, items[L], iteration);
}

// Persistent form: a fixed grid of association blocks (bpx for each of the 8
// runs of the item list, after the feature blocks) drains the work table.
// Block b of run x = b mod 8 first takes item b / 8 of its run, then claims
// the run's later items one at a time from the run's counter (which starts at
// bpx); each claim is issued when the block starts its current item, so its
// round trip overlaps the item's work.  Which block runs an item does not
// change its result (each item writes its own partial record, summed later in
// a fixed order); the last block to finish clears the counters for the next
// launch, so a captured graph replays it with no memory set.  ctr: 8 run
// counters and a count of finished blocks, zero at launch.
template <int PPT, bool LEARNED, bool BF16>
__global__ __launch_bounds__(kAssocThreads) void assoc_persistent_kernel(
    const GraphDev* __restrict__ gds, const WorkItem* __restrict__ items, int n_items, int per_xcd,
    int iteration, const int2* __restrict__ fitems, int n_fitems, unsigned* __restrict__ ctr, int n_blocks)
{
    const int nf8 = (n_fitems + 7) & ~7;
    if ((int)blockIdx.x < nf8) {
        if ((int)blockIdx.x < n_fitems)
            feature_set(gds, fitems[blockIdx.x]);
        return;
    }
    const int b = (int)blockIdx.x - nf8;
    const int x = b & 7, bpx = n_blocks / 8;
    __shared__ int s_next;
    int k = b >> 3;   // index within the run of this block's current item
    for (;;) {
        const int L = x * per_xcd + k;
        if (k >= per_xcd || L >= n_items)
            break;
        if (threadIdx.x == 0)
            s_next = bpx + (int)atomicAdd(ctr + x, 1u);   // the next claim, in flight during the item
        if constexpr (BF16)
            assoc_bf16x3_item<PPT, LEARNED>(gds, items[L], iteration);
        else
            assoc_item<PPT, LEARNED>(gds, items[L], iteration);
        __syncthreads();
        k = s_next;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(ctr + 8, 1u) == (unsigned)(n_blocks - 1))
            for (int q = 0; q < 9; ++q)
                atomicExch(ctr + q, 0u);
    }
}

// Association decisions of one ordered pair for inspection: the same
// projection and gating code as the association kernel, one thread per pixel.
__global__ __launch_bounds__(256) void assoc_debug_kernel(const GraphDev* __restrict__ gds, int i, int j,
                                                          int iteration, int* __restrict__ target,
                                                          float* __restrict__ res, float* __restrict__ uv,
                                                          float* __restrict__ feat, float* __restrict__ sigma)
{
    const GraphDev& gd = gds[0];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = x < gd.HW;
    const int lane = threadIdx.x & 63;
    const bool want_sigma = sigma != nullptr && gd.mlp32 != nullptr;   // uniform
    __shared__ __attribute__((aligned(16))) float s_tail[kMlpTail];
    MlpFrags M;
    if (want_sigma) {
        mlp_tail_load(gd.mlp32, s_tail);
        mlp_frags_load(gd.mlp32, M, lane);
        __syncthreads();
    }
    const int p = pair_index(i, j, gd.n_frames);
    float A[12], B[12];
    for (int k = 0; k < 12; ++k) {
        A[k] = gd.xf32[p * 24 + k];
        B[k] = gd.xf32[p * 24 + 12 + k];
    }
    const float4 s = live ? gd.maps[(size_t)i * gd.HW + x] : make_float4(0.f, 0.f, 0.f, 0.f);
    int code = -1;
    float r = 0.f, uf = __builtin_nanf(""), vf = uf;
    float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (s.w > 0.f) {
        const int u = x % gd.W, v = x / gd.W;
        const float px = s.w * (((float)u - gd.cx) * gd.ifx);
        const float py = s.w * (((float)v - gd.cy) * gd.ify);
        code = project_px(B, px, py, s.w, gd, uf, vf);
        if (code >= 0) {
            float J[6], rr, d2, c, sn;
            const int yi = px_index(code, gd.W);
            const float4 t = gd.maps[(size_t)j * gd.HW + yi];
            code = finish_px(A, px, py, s.w, s.x, s.y, s.z, code, t, gd, rr, J, d2, c, sn);
            if (code >= 0)
                code = yi;   // the target pixel's row-major index
            if (code >= 0) {
                r = rr;
                learned_features(gd, rr, d2, c, sn, s.w, (uint32_t)u | ((uint32_t)v << 16), iteration, f);
            }
        }
    }
    // the network as the association kernels evaluate it (wave-wide)
    float sg = 0.f;
    if (want_sigma && __ballot(code >= 0)) {
        const float o = mlp_sigma_wave(M, s_tail, f, lane);
        sg = (code >= 0) ? o : 0.f;
    }
    if (!live)
        return;
    if (target)
        target[x] = code;
    if (res)
        res[x] = r;
    if (uv) {
        uv[2 * x] = uf;
        uv[2 * x + 1] = vf;
    }
    if (feat)
        for (int k = 0; k < 6; ++k)
            feat[6 * (size_t)x + k] = f[k];
    if (sigma)
        sigma[x] = sg;
}

// ------------------------------------------------ pruning of source pixels

// Score of every source pixel at the poses of the start of an optimize: the
// largest network weight over the target frames it is gated in with
// (iteration feature 0), 0 when it is gated in nowhere.  One thread per
// source-list entry, looping over the target frames (no atomics: the score is
// a per-thread maximum).  Items: gij = frame | graph << 16, start, count <= 256.
constexpr int kPruneThreads = 256;

__global__ __launch_bounds__(kPruneThreads) void prune_score_kernel(const GraphDev* __restrict__ gds,
                                                                    const WorkItem* __restrict__ items)
{
    const WorkItem it = items[blockIdx.x];
    const GraphDev& gd = gds[it.gij >> 16];
    const int i = it.gij & 0xff;
    const int lane = threadIdx.x & 63;
    __shared__ __attribute__((aligned(16))) float s_tail[kMlpTail];
    // every lane stays to the end: the network runs wave-wide
    const bool live = (int)threadIdx.x < it.count;
    const size_t e = (size_t)i * gd.HW + it.start + (live ? threadIdx.x : 0);
    const float4 s = gd.src_nz[e];
    const uint32_t uv = gd.src_uv[e];
    // the network parameters, loaded while the source record is in flight
    MlpFrags M;
    mlp_tail_load(gd.mlp32, s_tail);
    mlp_frags_load(gd.mlp32, M, lane);
    __syncthreads();
    const float px = s.w * (((float)(uv & 0xffffu) - gd.cx) * gd.ifx);
    const float py = s.w * (((float)(uv >> 16) - gd.cy) * gd.ify);
    // the network runs wave-wide on the gated-in (pixel, target) samples of a
    // group of kPruneGroup targets, packed in LDS and evaluated 64 at a time;
    // each output goes back to its pixel's lane (the maximum is exact, so the
    // grouping changes no score)
    constexpr int kPruneGroup = 4;
    __shared__ float s_feat[kPruneThreads / 64][kMlpIn][64 * kPruneGroup];
    __shared__ float s_sig[kPruneThreads / 64][64 * kPruneGroup];
    const int wave = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    float best = 0.0f;
    for (int j0 = 0; j0 < gd.n_frames; j0 += kPruneGroup) {
        int slot[kPruneGroup];
        int nw = 0;   // gated-in samples of the wave in this group (uniform)
#pragma unroll
        for (int g = 0; g < kPruneGroup; ++g) {
            const int j = j0 + g;
            slot[g] = -1;
            if (j >= gd.n_frames || j == i)   // uniform
                continue;
            const int p = pair_index(i, j, gd.n_frames);
            float A[12], B[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                A[k] = gd.xf32[p * 24 + k];
                B[k] = gd.xf32[p * 24 + 12 + k];
            }
            bool gated = false;
            float f[kMlpIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (live) {
                float uf, vf;
                const int y = project_px(B, px, py, s.w, gd, uf, vf);
                if (y >= 0) {
                    const float4 t = gd.maps[(size_t)j * gd.HW + px_index(y, gd.W)];
                    float r, J[6], d2, c, sn;
                    if (finish_px(A, px, py, s.w, s.x, s.y, s.z, y, t, gd, r, J, d2, c, sn) >= 0) {
                        gated = true;
                        learned_features(gd, r, d2, c, sn, s.w, uv, 0, f);
                    }
                }
            }
            const unsigned long long bal = __ballot(gated);
            if (gated) {
                slot[g] = nw + __popcll(bal & below);
#pragma unroll
                for (int k = 0; k < kMlpIn; ++k)
                    s_feat[wave][k][slot[g]] = f[k];
            }
            nw += __popcll(bal);
        }
        // the wave reads back its own LDS writes (in order within a wavefront)
        asm volatile("" ::: "memory");
        for (int b0 = 0; b0 < nw; b0 += 64) {
            const int q = b0 + lane;
            float f[kMlpIn];
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k)
                f[k] = (q < nw) ? s_feat[wave][k][q] : 0.f;
            const float sgv = mlp_sigma_wave(M, s_tail, f, lane);
            if (q < nw)
                s_sig[wave][q] = sgv;
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int g = 0; g < kPruneGroup; ++g)
            if (slot[g] >= 0)
                best = fmaxf(best, s_sig[wave][slot[g]]);
        // the next group's writes after every lane has read this group's
        // outputs (in order within a wavefront)
        asm volatile("" ::: "memory");
    }
    if (live)
        gd.score[e] = __float_as_uint(best);
}

// Inclusive prefix sum over the 64 lanes of a wave by DPP (row shifts within
// the four 16-lane rows, then the row totals broadcast to the rows above): no
// LDS traffic.
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return x;
}

__device__ __forceinline__ int wave_sum(int x) { return __builtin_amdgcn_readlane(wave_incl_scan(x), 63); }

// The select kernel's block-wide scans: 16 waves, the wave values through LDS
// (read back in one unrolled pass) and one barrier; each call site has its
// own wave_vals buffer, so none is rewritten while a wave may still read it.
constexpr int kSelectThreads = 1024;
constexpr int kSelectWaves = kSelectThreads / 64;

// Exclusive prefix over the waves of one value per wave (every lane of a wave
// passes the same v) and the block total.
__device__ __forceinline__ int select_wave_excl(int v, int* wave_vals, int& total)
{
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        wave_vals[wv] = v;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSelectWaves; ++w) {
        const int c = wave_vals[w];
        off += (w < wv) ? c : 0;
        tot += c;
    }
    total = tot;
    return off;
}

// Exclusive prefix of one value per thread over the block, and the total.
__device__ __forceinline__ int select_thread_excl(int v, int* wave_vals, int& total)
{
    const int incl = wave_incl_scan(v);
    return select_wave_excl(__builtin_amdgcn_readlane(incl, 63), wave_vals, total) + incl - v;
}

// Block totals of two per-thread counts a and b, and the exclusive prefix over
// the waves of one value per wave c (every lane of a wave passes the same c).
__device__ __forceinline__ void select_counts(int a, int b, int c, int* wave_vals, int& ta, int& tb, int& c_off)
{
    const int wv = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        wave_vals[3 * wv] = a;
        wave_vals[3 * wv + 1] = b;
        wave_vals[3 * wv + 2] = c;
    }
    __syncthreads();
    ta = tb = c_off = 0;
#pragma unroll
    for (int w = 0; w < kSelectWaves; ++w) {
        ta += wave_vals[3 * w];
        tb += wave_vals[3 * w + 1];
        c_off += (w < wv) ? wave_vals[3 * w + 2] : 0;
    }
}

// Histograms of one digit of the keys k < n: LDS atomics of integer counts,
// so a histogram does not depend on which thread counts a key or in which
// order.  The whole slices of T keys (one per thread) go through a short
// sequence of compares into lane masks (inline assembly: the compiler's own
// form of these branches cost several times the instructions): a key costs a
// few vector instructions, and an LDS atomic is issued only when a lane of the
// wave has a key to add; the last, partial slice takes plain code with a
// bounds test.
constexpr int kSelectDom = 3;
constexpr int kSelectDomRounds = 16;

// The counting of select_hist_top with dominant bins bd0..bd2 (ZERO: bd2 is
// bin 0 and counts only keys equal to zero, their total also added to
// *zeros).
template <bool ZERO, typename KeyAt>
__device__ __forceinline__ void select_top_sweep(KeyAt key_at, int n, int* h, int bd0, int bd1, int bd2, int* zeros)
{
    constexpr int T = kSelectThreads, P = 8;
    const int tid = threadIdx.x, lane = tid & 63;
    // per-lane counts of the dominant bins
    int c0 = 0, c1 = 0, c2 = 0;
    const unsigned int hb = (unsigned int)(uintptr_t)(const __attribute__((address_space(3))) int*)h;
    // whole slices of T keys: compares into lane masks, counts by
    // add-with-carry, and the LDS atomic of the other lanes with the
    // execution mask narrowed to them (skipped when there are none; the mask
    // is restored before the block ends)
    auto whole = [&](unsigned int key) {
        unsigned int bin, addr;
        unsigned long long m0, m1, m2, co, sv;
        if constexpr (ZERO) {
            asm volatile(
                "v_lshrrev_b32 %[bin], 20, %[key]\n\t"
                "v_cmp_eq_u32 %[m0], %[b0], %[bin]\n\t"
                "v_cmp_eq_u32 %[m1], %[b1], %[bin]\n\t"
                "v_cmp_eq_u32 %[m2], 0, %[key]\n\t"
                "v_addc_co_u32 %[c0], %[co], 0, %[c0], %[m0]\n\t"
                "v_addc_co_u32 %[c1], %[co], 0, %[c1], %[m1]\n\t"
                "v_addc_co_u32 %[c2], %[co], 0, %[c2], %[m2]\n\t"
                "s_or_b64 %[m0], %[m0], %[m1]\n\t"
                "s_or_b64 %[m0], %[m0], %[m2]\n\t"
                "s_mov_b64 %[sv], exec\n\t"
                "s_andn2_b64 exec, exec, %[m0]\n\t"
                "s_cbranch_execz .Lsel_topz_skip%=\n\t"
                "v_lshl_add_u32 %[addr], %[bin], 2, %[hb]\n\t"
                "ds_add_u32 %[addr], %[one]\n\t"
                ".Lsel_topz_skip%=:\n\t"
                "s_mov_b64 exec, %[sv]"
                : [bin] "=&v"(bin), [addr] "=&v"(addr), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2),
                  [co] "=&s"(co), [sv] "=&s"(sv), [c0] "+v"(c0), [c1] "+v"(c1), [c2] "+v"(c2)
                : [key] "v"(key), [b0] "s"(bd0), [b1] "s"(bd1), [hb] "s"(hb), [one] "v"(1)
                : "memory", "scc");
        } else {
            asm volatile(
                "v_lshrrev_b32 %[bin], 20, %[key]\n\t"
                "v_cmp_eq_u32 %[m0], %[b0], %[bin]\n\t"
                "v_cmp_eq_u32 %[m1], %[b1], %[bin]\n\t"
                "v_cmp_eq_u32 %[m2], %[b2], %[bin]\n\t"
                "v_addc_co_u32 %[c0], %[co], 0, %[c0], %[m0]\n\t"
                "v_addc_co_u32 %[c1], %[co], 0, %[c1], %[m1]\n\t"
                "v_addc_co_u32 %[c2], %[co], 0, %[c2], %[m2]\n\t"
                "s_or_b64 %[m0], %[m0], %[m1]\n\t"
                "s_or_b64 %[m0], %[m0], %[m2]\n\t"
                "s_mov_b64 %[sv], exec\n\t"
                "s_andn2_b64 exec, exec, %[m0]\n\t"
                "s_cbranch_execz .Lsel_top_skip%=\n\t"
                "v_lshl_add_u32 %[addr], %[bin], 2, %[hb]\n\t"
                "ds_add_u32 %[addr], %[one]\n\t"
                ".Lsel_top_skip%=:\n\t"
                "s_mov_b64 exec, %[sv]"
                : [bin] "=&v"(bin), [addr] "=&v"(addr), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2),
                  [co] "=&s"(co), [sv] "=&s"(sv), [c0] "+v"(c0), [c1] "+v"(c1), [c2] "+v"(c2)
                : [key] "v"(key), [b0] "s"(bd0), [b1] "s"(bd1), [b2] "s"(bd2), [hb] "s"(hb), [one] "v"(1)
                : "memory", "scc");
        }
    };
    const int full = (n / T) * T;
    int k0 = 0;
    for (; k0 + T * P <= full; k0 += T * P) {
        unsigned int kk[P];
#pragma unroll
        for (int q = 0; q < P; ++q)
            kk[q] = key_at(k0 + q * T + tid);
#pragma unroll
        for (int q = 0; q < P; ++q)
            whole(kk[q]);
    }
    if (k0 < full) {   // the other whole slices, loaded together
        const int ns = (full - k0) / T;
        unsigned int kk[P - 1];
#pragma unroll
        for (int q = 0; q < P - 1; ++q)
            if (q < ns)
                kk[q] = key_at(k0 + q * T + tid);
#pragma unroll
        for (int q = 0; q < P - 1; ++q)
            if (q < ns)
                whole(kk[q]);
        k0 = full;
    }
    if (k0 < n && k0 + tid < n) {   // the last, partial slice
        const unsigned int key = key_at(k0 + tid);
        const int bin = (int)(key >> 20);
        if (bin == bd0)
            ++c0;
        else if (bin == bd1)
            ++c1;
        else if (ZERO ? key == 0u : bin == bd2)
            ++c2;
        else
            atomicAdd(&h[bin], 1);
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    if (lane == 0) {
        if (c0 > 0)
            atomicAdd(&h[bd0], c0);
        if (c1 > 0)
            atomicAdd(&h[bd1], c1);
        if (c2 > 0) {
            atomicAdd(&h[bd2], c2);
            if (ZERO)
                atomicAdd(zeros, c2);
        }
    }
}

// First digit, bits 20..31 of every key.  Each wave first takes the
// kSelectDom most frequent bins of 64 keys spread over the list (at most
// kSelectDomRounds distinct bins looked at) as its dominant bins and counts
// the keys in those in registers, added with one atomic each at the end (the
// first digit of the scores falls in a few bins: mostly one, and zero for
// sources gated in nowhere; lanes of a wave that hit one address would
// serialise their atomics); every other key is one LDS atomic.  *zeros
// receives the count of keys equal to zero when bin 0 is a dominant bin (else
// it is left as it is).
template <typename KeyAt>
__device__ __forceinline__ void select_hist_top(KeyAt key_at, int n, int* h, int* zeros)
{
    constexpr int T = kSelectThreads, P = 8;
    const int tid = threadIdx.x, lane = tid & 63;
    if (n <= 0)
        return;
    int bd[kSelectDom], cnt[kSelectDom];
#pragma unroll
    for (int e = 0; e < kSelectDom; ++e) {
        bd[e] = -1;
        cnt[e] = 0;
    }
    {
        const int b = (int)(key_at((int)(((long long)lane * n) >> 6)) >> 20);
        unsigned long long left = ~0ull;
        for (int r = 0; r < kSelectDomRounds && left != 0ull; ++r) {
            const int cb = __builtin_amdgcn_readlane(b, __ffsll((long long)left) - 1);
            const unsigned long long same = __ballot(b == cb);
            left &= ~same;
            int c = __popcll(same), bb = cb;
#pragma unroll
            for (int e = 0; e < kSelectDom; ++e)   // insertion into the descending list
                if (c > cnt[e]) {
                    const int tc = cnt[e], tb = bd[e];
                    cnt[e] = c;
                    bd[e] = bb;
                    c = tc;
                    bb = tb;
                }
        }
    }
    // bin 0 (zero and subnormal scores) among them: that slot counts only the
    // exact zeros (the others fall to the atomics), so that a threshold at
    // zero is recognised without the later digits (a tie of many keys)
    if (bd[0] == 0) {
        bd[0] = bd[2];
        bd[2] = 0;
    } else if (bd[1] == 0) {
        bd[1] = bd[2];
        bd[2] = 0;
    }
    if (bd[2] == 0)
        select_top_sweep<true>(key_at, n, h, bd[0], bd[1], 0, zeros);
    else
        select_top_sweep<false>(key_at, n, h, bd[0], bd[1], bd[2], zeros);
}

// A later digit, (key >> shift) & dmask of the keys with (key & mask) == prefix.
// AGG (a prefix shared by many equal keys: zero, the score of sources gated in
// nowhere): the lanes in the bin of the first counted lane add with one
// atomic of their count, as equal keys would serialise on one address.
template <bool AGG, typename KeyAt>
__device__ __forceinline__ void select_hist_low(KeyAt key_at, int n, int shift, unsigned int dmask,
                                                unsigned int mask, unsigned int prefix, int* h)
{
    constexpr int T = kSelectThreads, P = 8;
    const int tid = threadIdx.x;
    const unsigned int hb = (unsigned int)(uintptr_t)(const __attribute__((address_space(3))) int*)h;
    // whole slices of T keys
    auto whole = [&](unsigned int key) {
        if constexpr (!AGG) {
            // the LDS atomic with the execution mask narrowed to the lanes
            // whose key has the prefix (skipped when there are none; the
            // mask is restored before the block ends)
            unsigned int t, addr;
            unsigned long long m, sv;
            asm volatile(
                "v_and_b32 %[t], %[mask], %[key]\n\t"
                "v_cmp_eq_u32 %[m], %[prefix], %[t]\n\t"
                "s_mov_b64 %[sv], exec\n\t"
                "s_and_b64 exec, exec, %[m]\n\t"
                "s_cbranch_execz .Lsel_low_skip%=\n\t"
                "v_lshrrev_b32 %[t], %[shift], %[key]\n\t"
                "v_and_b32 %[t], %[dmask], %[t]\n\t"
                "v_lshl_add_u32 %[addr], %[t], 2, %[hb]\n\t"
                "ds_add_u32 %[addr], %[one]\n\t"
                ".Lsel_low_skip%=:\n\t"
                "s_mov_b64 exec, %[sv]"
                : [t] "=&v"(t), [addr] "=&v"(addr), [m] "=&s"(m), [sv] "=&s"(sv)
                : [key] "v"(key), [mask] "s"(mask), [prefix] "s"(prefix), [shift] "s"(shift),
                  [dmask] "s"(dmask), [hb] "s"(hb), [one] "v"(1)
                : "memory", "scc");
        } else {
            // of the lanes whose key has the prefix, those in the bin of the
            // first of them add with one atomic of their count, the others
            // with one atomic each, the execution mask narrowed to them (all
            // skipped when no lane has the prefix; the mask is restored
            // before the block ends)
            unsigned int t, addr, vc;
            unsigned long long m, same, one_lane, sv;
            unsigned int fl, b0, cnt;
            asm volatile(
                "v_and_b32 %[t], %[mask], %[key]\n\t"
                "v_cmp_eq_u32 %[m], %[prefix], %[t]\n\t"
                "s_cmp_eq_u64 %[m], 0\n\t"
                "s_cbranch_scc1 .Lsel_low_none%=\n\t"
                "v_lshrrev_b32 %[t], %[shift], %[key]\n\t"
                "v_and_b32 %[t], %[dmask], %[t]\n\t"
                "s_ff1_i32_b64 %[fl], %[m]\n\t"
                "s_nop 4\n\t"
                "v_readlane_b32 %[b0], %[t], %[fl]\n\t"
                "v_cmp_eq_u32 %[same], %[b0], %[t]\n\t"
                "s_and_b64 %[same], %[same], %[m]\n\t"
                "s_andn2_b64 %[m], %[m], %[same]\n\t"
                "s_bcnt1_i32_b64 %[cnt], %[same]\n\t"
                "s_lshl_b64 %[one], 1, %[fl]\n\t"
                "s_mov_b64 %[sv], exec\n\t"
                "s_mov_b64 exec, %[one]\n\t"
                "v_mov_b32 %[vc], %[cnt]\n\t"
                "v_lshl_add_u32 %[addr], %[t], 2, %[hb]\n\t"
                "ds_add_u32 %[addr], %[vc]\n\t"
                "s_and_b64 exec, %[sv], %[m]\n\t"
                "s_cbranch_execz .Lsel_low_restore%=\n\t"
                "v_lshl_add_u32 %[addr], %[t], 2, %[hb]\n\t"
                "ds_add_u32 %[addr], %[onev]\n\t"
                ".Lsel_low_restore%=:\n\t"
                "s_mov_b64 exec, %[sv]\n\t"
                ".Lsel_low_none%=:"
                : [t] "=&v"(t), [addr] "=&v"(addr), [vc] "=&v"(vc), [m] "=&s"(m), [same] "=&s"(same),
                  [one] "=&s"(one_lane), [sv] "=&s"(sv), [fl] "=&s"(fl), [b0] "=&s"(b0), [cnt] "=&s"(cnt)
                : [key] "v"(key), [mask] "s"(mask), [prefix] "s"(prefix), [shift] "s"(shift),
                  [dmask] "s"(dmask), [hb] "s"(hb), [onev] "v"(1)
                : "memory", "scc");
        }
    };
    const int full = (n / T) * T;
    int k0 = 0;
    for (; k0 + T * P <= full; k0 += T * P) {
        unsigned int kk[P];
#pragma unroll
        for (int q = 0; q < P; ++q)
            kk[q] = key_at(k0 + q * T + tid);
#pragma unroll
        for (int q = 0; q < P; ++q)
            whole(kk[q]);
    }
    if (k0 < full) {   // the other whole slices, loaded together
        const int ns = (full - k0) / T;
        unsigned int kk[P - 1];
#pragma unroll
        for (int q = 0; q < P - 1; ++q)
            if (q < ns)
                kk[q] = key_at(k0 + q * T + tid);
#pragma unroll
        for (int q = 0; q < P - 1; ++q)
            if (q < ns)
                whole(kk[q]);
        k0 = full;
    }
    if (k0 < n && k0 + tid < n) {   // the last, partial slice
        const unsigned int key = key_at(k0 + tid);
        if ((key & mask) == prefix)
            atomicAdd(&h[(key >> shift) & dmask], 1);
    }
}

// The bin holding the entry of 0-based rank 'rank' in histogram h (PER
// consecutive bins per thread of the 1024): out = {bin, rank within the bin},
// visible to the block on return.
template <int PER>
__device__ __forceinline__ void select_bin(const int* h, int rank, int* wave_vals, int* out)
{
    int c[PER], sum = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        c[e] = h[PER * threadIdx.x + e];
        sum += c[e];
    }
    int tot;
    const int excl = select_thread_excl(sum, wave_vals, tot);
    if (excl <= rank && rank < excl + sum) {
        int r = rank - excl, bin = -1;
#pragma unroll
        for (int e = 0; e < PER; ++e)
            if (bin < 0) {
                if (r < c[e])
                    bin = e;
                else
                    r -= c[e];
            }
        out[0] = PER * (int)threadIdx.x + bin;
        out[1] = r;
    }
    __syncthreads();
}

// Per frame, bpf >= kSelectBlocks blocks of 1024 threads: drop the n_drop
// source pixels of lowest score, ties by position in the row-major source
// list, and compact the kept ones in order into the pruned lists.  Every block
// finds the n_drop-th smallest key itself (the same computation on the same
// data, so all agree): an MSB-first radix select over three digits (bits
// 20..31, 10..19, 0..9) with LDS histograms of integer counts, so the result
// does not depend on the order of the atomics.  STAGED (at most kSelectStageKeys sources): the frame's keys are loaded into
// LDS once, every load in flight together, and the passes read them there;
// otherwise they are read from global memory.  Block b then compacts its own segment of the list: its output
// offset and its rank among the keys equal to the threshold come from
// counting the keys before the segment.  Within the segment each wave takes a
// contiguous run in slices of 64 consecutive entries (ranks by ballot, wave
// offsets by a scan over the waves), so the loads of the source records and
// the stores of the kept ones are coalesced; staged, the run's records are
// loaded at the start, in flight during the select.
constexpr int kSelectBlocks = 8;          // blocks per frame, at least
constexpr int kSelectMaxSlices = 64;      // 64-entry slices of one wave's run (bits of a mask)
constexpr int kSelectPer = 8;             // keys per thread and step of a histogram pass
constexpr int kSelectStagePer = 32;       // keys per thread when staged
constexpr int kSelectStageKeys = kSelectStagePer * kSelectThreads;
constexpr int kSelectGroup = 4;           // slices whose records are loaded together
constexpr int kSelectBinsA = 4096;       // digit A: key bits 20..31
constexpr int kSelectBinsB = 1024;       // digits B, C: bits 10..19 and 0..9
// staged, a wave's run is at most kSelectGroup slices (one load group)
static_assert(kSelectStageKeys / kSelectBlocks <= kSelectWaves * 64 * kSelectGroup, "staged runs");

template <bool STAGED>
__global__ __launch_bounds__(kSelectThreads) void prune_select_kernel(const GraphDev* __restrict__ gds,
                                                                      const int2* __restrict__ frames, int bpf)
{
    __shared__ __attribute__((aligned(16))) unsigned int s_key[STAGED ? kSelectStageKeys : 4];
    // the three digits' histograms (cleared together), one wave-value buffer
    // per scan and one result per digit, so no buffer is rewritten before
    // every wave has passed a barrier after its last read
    __shared__ __attribute__((aligned(16))) int hist[kSelectBinsA + 2 * kSelectBinsB];
    __shared__ int wave_vals[5][3 * kSelectWaves];
    __shared__ int s_sel[3][2];
    __shared__ int s_zeros;   // keys equal to zero, when counted by the first digit
    const int2 fr = frames[blockIdx.x / bpf];
    const int seg = blockIdx.x % bpf;
    const GraphDev& gd = gds[fr.x];
    const int i = fr.y;
    const int V = ld_global(gd.n_src + i);
    const int drop = ld_global(gd.n_drop + i);
    const size_t base = (size_t)i * gd.HW;
    const unsigned int* key = gd.score + base;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;

    // this block's segment [s0, s1) of the list and this wave's run [r0, r1)
    // of it: n_slices <= kSelectMaxSlices (the launch sizes bpf for that)
    const int s0 = (int)(((long long)V * seg) / bpf);
    const int s1 = (int)(((long long)V * (seg + 1)) / bpf);
    const int run = (s1 - s0 + kSelectWaves * 64 - 1) / (kSelectWaves * 64) * 64;
    const int r0 = min(s0 + wv * run, s1), r1 = min(r0 + run, s1);
    const int n_slices = (r1 - r0 + 63) / 64;

    float4 pnz[kSelectGroup];
    uint32_t puv[kSelectGroup];
    if constexpr (STAGED) {
        // the run's source records and every key of the frame, all in flight
        // together
#pragma unroll
        for (int d = 0; d < kSelectGroup; ++d) {
            const int k = r0 + 64 * d + lane;
            pnz[d] = make_float4(0.f, 0.f, 0.f, 0.f);
            puv[d] = 0u;
            if (k < r1) {
                pnz[d] = ld_global(gd.src_nz + base + k);
                puv[d] = ld_global(gd.src_uv + base + k);
            }
        }
        // (the slots past the list, never read, hold all ones).  Rows of a
        // multiple of 4 pixels: 4 keys per load (16-byte aligned; a group past
        // the list start stays inside the frame, whose size is a multiple of 4)
        if ((gd.HW & 3) == 0) {
            typedef unsigned int u4v __attribute__((ext_vector_type(4)));
            u4v kv[kSelectStagePer / 4];
#pragma unroll
            for (int q = 0; q < kSelectStagePer / 4; ++q) {
                const int k = 4 * (q * kSelectThreads + tid);
                kv[q] = (u4v){0u, 0u, 0u, 0u};
                if (k < V)
                    kv[q] = *(const __attribute__((address_space(1))) u4v*)(key + k);
            }
#pragma unroll
            for (int q = 0; q < kSelectStagePer / 4; ++q) {
                const int k = 4 * (q * kSelectThreads + tid);
                u4v w = kv[q];
                w.x = (k < V) ? w.x : 0xffffffffu;
                w.y = (k + 1 < V) ? w.y : 0xffffffffu;
                w.z = (k + 2 < V) ? w.z : 0xffffffffu;
                w.w = (k + 3 < V) ? w.w : 0xffffffffu;
                *(u4v*)(s_key + k) = w;
            }
        } else {
            unsigned int kk[kSelectStagePer];
#pragma unroll
            for (int q = 0; q < kSelectStagePer; ++q)
                kk[q] = (V > 0) ? ld_global(key + min(q * kSelectThreads + tid, V - 1)) : 0u;
#pragma unroll
            for (int q = 0; q < kSelectStagePer; ++q)
                s_key[q * kSelectThreads + tid] = (q * kSelectThreads + tid < V) ? kk[q] : 0xffffffffu;
        }
    }
    if (STAGED && drop <= 0)
        __syncthreads();   // the staging ends (with drop > 0, at the histogram clear)
    auto key_at = [&](int k) -> unsigned int {
        if constexpr (STAGED)
            return s_key[k];
        else
            return ld_global(key + k);
    };

    unsigned int tau = 0;   // key of the last dropped entry in (key, position) order
    int need = 0;           // entries equal to tau that are dropped (lowest positions first)
    if (drop > 0) {
        for (int q = tid; q < kSelectBinsA + 2 * kSelectBinsB; q += kSelectThreads)
            hist[q] = 0;
        if (tid == 0)
            s_zeros = 0;
        __syncthreads();   // (also ends the staging)
        // digit A: key bits 20..31
        select_hist_top(key_at, V, hist, &s_zeros);
        __syncthreads();
        select_bin<kSelectBinsA / kSelectThreads>(hist, drop - 1, wave_vals[0], s_sel[0]);
        if (s_sel[0][0] == 0 && hist[0] == s_zeros) {
            // the entry sought is a zero and its bin holds zeros only: a tie
            // of many keys, resolved without the later digits
            tau = 0u;
            need = s_sel[0][1] + 1;
        } else {
            unsigned int prefix = (unsigned int)s_sel[0][0] << 20;
            // digit B: bits 10..19 of the keys with that digit A
            int* const histB = hist + kSelectBinsA;
            // (ties at zero: the aggregating form)
            const bool zero = s_sel[0][0] == 0;
            if (zero)
                select_hist_low<true>(key_at, V, 10, kSelectBinsB - 1, 0xfff00000u, prefix, histB);
            else
                select_hist_low<false>(key_at, V, 10, kSelectBinsB - 1, 0xfff00000u, prefix, histB);
            __syncthreads();
            select_bin<kSelectBinsB / kSelectThreads>(histB, s_sel[0][1], wave_vals[1], s_sel[1]);
            prefix |= (unsigned int)s_sel[1][0] << 10;
            // digit C: bits 0..9 of the keys with those digits A and B
            int* const histC = histB + kSelectBinsB;
            if (zero)
                select_hist_low<true>(key_at, V, 0, kSelectBinsB - 1, 0xfffffc00u, prefix, histC);
            else
                select_hist_low<false>(key_at, V, 0, kSelectBinsB - 1, 0xfffffc00u, prefix, histC);
            __syncthreads();
            select_bin<kSelectBinsB / kSelectThreads>(histC, s_sel[1][1], wave_vals[2], s_sel[2]);
            tau = prefix | (unsigned int)s_sel[2][0];
            need = s_sel[2][1] + 1;
        }
    }
    // keys before the segment (the output offset and the rank among the keys
    // equal to tau) and the entries equal to tau in this wave's run, in one
    // exchange over the waves
    int n_lt = 0, n_eq = 0, eq_w = 0;
    if (drop > 0) {
        for (int k0 = 0; k0 < s0; k0 += kSelectThreads * kSelectPer) {
            unsigned int kk[kSelectPer];
#pragma unroll
            for (int q = 0; q < kSelectPer; ++q)
                kk[q] = key_at(min(k0 + q * kSelectThreads + tid, V - 1));
#pragma unroll
            for (int q = 0; q < kSelectPer; ++q) {
                const bool in = k0 + q * kSelectThreads + tid < s0;
                n_lt += (in && kk[q] < tau) ? 1 : 0;
                n_eq += (in && kk[q] == tau) ? 1 : 0;
            }
        }
        for (int c = 0; c < n_slices; ++c) {
            const int k = r0 + 64 * c + lane;
            eq_w += __popcll(__ballot(k < r1 && key_at(k) == tau));
        }
    }
    int lt_before, eq_before, eq_off;
    select_counts(n_lt, n_eq, eq_w, wave_vals[3], lt_before, eq_before, eq_off);
    int eq_rank = eq_before + eq_off;
    // keep decisions of the run in order: entry k is kept unless key < tau,
    // or key == tau and it is among the first 'need' entries equal to tau
    unsigned long long keep = 0ull;   // bit c: this lane's entry of slice c is kept
    int kept_w = 0;
    for (int c = 0; c < n_slices; ++c) {
        const int k = r0 + 64 * c + lane;
        const bool live = k < r1;
        const unsigned int kv = live ? key_at(k) : 0u;
        const bool eq = live && drop > 0 && kv == tau;
        const unsigned long long be = __ballot(eq);
        const bool kq = live && (drop == 0 || kv > tau || (eq && eq_rank + __popcll(be & below) >= need));
        eq_rank += __popcll(be);
        keep |= (kq ? 1ull : 0ull) << c;
        kept_w += __popcll(__ballot(kq));
    }
    int kept_tot;
    int pos = s0 - lt_before - min(need, eq_before) + select_wave_excl(kept_w, wave_vals[4], kept_tot);
    // the kept records at their ranks, kSelectGroup slices loaded together
    for (int c0 = 0; c0 < n_slices; c0 += kSelectGroup) {
        float4 nz[kSelectGroup];
        uint32_t uv[kSelectGroup];
#pragma unroll
        for (int d = 0; d < kSelectGroup; ++d) {
            if constexpr (STAGED) {   // a single group, loaded at the start
                nz[d] = pnz[d];
                uv[d] = puv[d];
            } else {
                const int k = r0 + 64 * (c0 + d) + lane;
                nz[d] = make_float4(0.f, 0.f, 0.f, 0.f);
                uv[d] = 0u;
                if (k < r1) {
                    nz[d] = ld_global(gd.src_nz + base + k);
                    uv[d] = ld_global(gd.src_uv + base + k);
                }
            }
        }
#pragma unroll
        for (int d = 0; d < kSelectGroup; ++d) {
            const int c = c0 + d;
            const bool kq = c < n_slices && ((keep >> c) & 1ull);
            const unsigned long long bk = __ballot(kq);
            if (kq) {
                const int at = pos + __popcll(bk & below);
                st_global(gd.psrc_nz + base + at, nz[d]);
                st_global(gd.psrc_uv + base + at, uv[d]);
            }
            pos += __popcll(bk);
        }
    }
}

// -------------------------------------------------------- feature residuals

// One block per match set, in FP64 (the residual is a millimetre difference
// of object-frame points; the whole term is a few thousand matches):
// e = T_i^-1 p_m - T_j^-1 p_n (Eq. 2), Huber weight w.  Every entry of the
// Jacobian [-R_i^T, R_i^T [p_m]x | R_j^T, -R_j^T [p_n]x] and of e is linear in
// u = (1, p_m, p_n), so the sums of w J^T J and w J^T e over a set follow
// exactly from the weighted second moments S = sum w u u^T (28 values): with
// J_r = B_r u and e_r = A_r . u per residual row r,
//   sum w J^T J [a][c] = sum_r B_r[a]^T S B_r[c],  sum w J^T e [a] = sum_r B_r[a]^T S A_r.
// Per thread: S, the Huber energy and the count (30 values) in registers,
// a recursive-halving wave reduction, a fixed-order sum over the waves, then
// the 12x12 upper triangle, the 12 gradient entries, energy and count
// expanded from S in FP64, one output per thread.
constexpr int kFeatThreads = 256;
static_assert(kFeatThreads == kAssocThreads, "feature sets run in association blocks");

template <int HALF, int OFF, typename T, int L>
__device__ __forceinline__ void halve_at(T (&acc)[L], int lane)
{
    const bool up = (lane & (2 * HALF)) != 0;
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        const T send = up ? acc[OFF + q] : acc[OFF + q + HALF];
        const T keep = up ? acc[OFF + q + HALF] : acc[OFF + q];
        acc[OFF + q] = keep + __shfl_xor(send, 2 * HALF);
    }
}

// reduce the 32 values acc[OFF..OFF+31] over the wave: lane l ends with the
// total of value OFF + (l >> 1) in acc[OFF]
template <int OFF, typename T, int L>
__device__ __forceinline__ void wave_reduce32(T (&acc)[L], int lane)
{
    halve_at<16, OFF>(acc, lane);
    halve_at<8, OFF>(acc, lane);
    halve_at<4, OFF>(acc, lane);
    halve_at<2, OFF>(acc, lane);
    halve_at<1, OFF>(acc, lane);
    acc[OFF] += __shfl_xor(acc[OFF], 1);
}

// Value of v held by the partner lane across lane bit B (the partner is
// lane ^ (1 << B)): DPP quad permutations for bits 0 and 1, a row rotation by
// 8 for bit 3, a bit-mask swizzle for bits 2 and 4, a permute for bit 5.
template <int B>
__device__ __forceinline__ double lane_swap(double v)
{
    const long long x = __double_as_longlong(v);
    int lo = (int)x, hi = (int)(x >> 32);
    if constexpr (B == 0) {
        lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
        hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
    } else if constexpr (B == 1) {
        lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
        hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
    } else if constexpr (B == 3) {
        lo = __builtin_amdgcn_mov_dpp(lo, 0x128, 0xF, 0xF, false);  // row_ror 8 (within 16 lanes)
        hi = __builtin_amdgcn_mov_dpp(hi, 0x128, 0xF, 0xF, false);
    } else if constexpr (B == 2 || B == 4) {
        constexpr int kSwz = 0x1F | ((1 << B) << 10);                // and 0x1f, xor 1 << B
        lo = __builtin_amdgcn_ds_swizzle(lo, kSwz);
        hi = __builtin_amdgcn_ds_swizzle(hi, kSwz);
    } else {
        return __shfl_xor(v, 1 << B);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One recursive-halving level over lane bit B: the lanes with the bit clear
// keep values [0, HALF) of acc, the others [HALF, 2 HALF), each adding its
// partner's copy; the kept half moves to acc[0, HALF).
template <int HALF, int B, int L>
__device__ __forceinline__ void halve_bit(double (&acc)[L], int lane)
{
    const bool up = (lane >> B) & 1;
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        const double send = up ? acc[q] : acc[q + HALF];
        const double keep = up ? acc[q + HALF] : acc[q];
        acc[q] = keep + lane_swap<B>(send);
    }
}

// Sum the 32 values acc[0..31] over the wave: on return acc[0] of lane l
// holds the total of value wave_sum32_index(l).
template <int L>
__device__ __forceinline__ void wave_sum32(double (&acc)[L], int lane)
{
    halve_bit<16, 0>(acc, lane);
    halve_bit<8, 1>(acc, lane);
    halve_bit<4, 3>(acc, lane);
    halve_bit<2, 2>(acc, lane);
    halve_bit<1, 4>(acc, lane);
    acc[0] += lane_swap<5>(acc[0]);
}

__device__ __forceinline__ int wave_sum32_index(int lane)
{
    return 16 * (lane & 1) + 8 * ((lane >> 1) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) +
           ((lane >> 4) & 1);
}

// Non-zero coefficients of u = (1, p_m, p_n) in Jacobian column a of residual
// row r (rho = row r of R_i^T, sig = row r of R_j^T): J[r][a] = c0 u_i0 + c1 u_i1.
__device__ __forceinline__ void feat_jac_sparse(const double* __restrict__ rho, const double* __restrict__ sig,
                                                int a, int& i0, double& c0, int& i1, double& c1)
{
    const int q = a % 3, q1 = (q + 1) % 3, q2 = (q + 2) % 3;
    if (a < 3) {            // -R_i^T
        i0 = 0; c0 = -rho[q]; i1 = 0; c1 = 0.0;
    } else if (a < 6) {     // R_i^T [p_m]x: row r is rho x p_m
        i0 = 1 + q2; c0 = rho[q1]; i1 = 1 + q1; c1 = -rho[q2];
    } else if (a < 9) {     // R_j^T
        i0 = 0; c0 = sig[q]; i1 = 0; c1 = 0.0;
    } else {                // -R_j^T [p_n]x
        i0 = 4 + q2; c0 = -sig[q1]; i1 = 4 + q1; c1 = sig[q2];
    }
}

// Sum 16 values acc[0..15] over the wave: on return acc[0] of lane l < 16
// holds the total of value wave_sum16_index(l).
template <int L>
__device__ __forceinline__ void wave_sum16(double (&acc)[L], int lane)
{
    halve_bit<8, 0>(acc, lane);
    halve_bit<4, 1>(acc, lane);
    halve_bit<2, 3>(acc, lane);
    halve_bit<1, 2>(acc, lane);
    acc[0] += lane_swap<4>(acc[0]);
    acc[0] += lane_swap<5>(acc[0]);
}

__device__ __forceinline__ int wave_sum16_index(int lane)
{
    return 8 * (lane & 1) + 4 * ((lane >> 1) & 1) + 2 * ((lane >> 3) & 1) + ((lane >> 2) & 1);
}

// Values 16 PASS .. 16 PASS + 15 of one match's 30 (the 28 weighted moments
// w u_a u_c, a <= c, row-major, then the Huber energy and the count) added to
// acc; false when the match is invalid.
// a value equal on every lane, moved to scalar registers
__device__ __forceinline__ double uniform_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int PASS>
__device__ __forceinline__ bool feature_match_values(const GraphDev& gd, const double (&A)[12], float4 qm,
                                                     float4 qn, double ifx, double ify, double (&acc)[16])
{
    if (!(qm.w > 0.f))
        return false;
    const double huber = (double)gd.huber_f;
    const double zm = qm.z, zn = qn.z;
    const double u[7] = {1.0,
                         zm * (((double)qm.x - gd.cx64) * ifx), zm * (((double)qm.y - gd.cy64) * ify), zm,
                         zn * (((double)qn.x - gd.cx64) * ifx), zn * (((double)qn.y - gd.cy64) * ify), zn};
    // |e| = |R_i^T (p_m - A p_n)| = |p_m - A p_n| with A = T_i T_j^-1
    double ne2 = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double d = u[1 + r] - (A[4 * r] * u[4] + A[4 * r + 1] * u[5] + A[4 * r + 2] * u[6] + A[4 * r + 3]);
        ne2 = fma(d, d, ne2);
    }
    // |e| and the Huber weight through 1/|e| (hardware reciprocal square root
    // and two Newton steps)
    const double x = fmax(ne2, 1e-300);
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    y = y * fma(-0.5 * x, y * y, 1.5);
    const double ne = ne2 * y;
    const double w = (ne <= huber) ? 1.0 : huber * y;
    int q = 0;
#pragma unroll
    for (int a = 0; a < 7; ++a)
#pragma unroll
        for (int c = a; c < 7; ++c, ++q)
            if (q >= 16 * PASS && q < 16 * PASS + 16)
                acc[q - 16 * PASS] += (w * u[a]) * u[c];
    if (PASS == 1) {
        acc[28 - 16] += (ne <= huber) ? 0.5 * ne * ne : huber * (ne - 0.5 * huber);
        acc[29 - 16] += 1.0;
    }
    return true;
}

// One match set (fi = {graph, set}) by one block of kFeatThreads threads: the
// 30 sums in two passes of 16 (few registers, so the association kernels can
// run it in some of their blocks), fixed-order wave and cross-wave sums, then
// the expansion to the 92 outputs.
__device__ __forceinline__ void feature_set(const GraphDev* __restrict__ gds, int2 fi)
{
    const GraphDev& gd = gds[fi.x];
    if (*gd.status)
        return;
    const int4 S = gd.fsets[fi.y];
    __shared__ double Tinv[2][12];
    __shared__ double red[kFeatThreads / 64][32];
    __shared__ double Sm[7][8];  // the moments as a full symmetric matrix; [0][7], [1][7]: energy, count
    // T^-1 of both frames: uniform reads (scalar registers) in the match loop,
    // an LDS copy for the expansion
    const double* __restrict__ Ti_g = gd.tinv64 + 12 * S.x;
    const double* __restrict__ Tj_g = gd.tinv64 + 12 * S.y;
    if (threadIdx.x < 24)
        Tinv[threadIdx.x / 12][threadIdx.x % 12] = (threadIdx.x < 12 ? Ti_g : Tj_g)[threadIdx.x % 12];
    // A = T_i T_j^-1 of the ordered pair (i, j), in scalar registers
    const double* __restrict__ A_g = gd.xf64 + 12 * pair_index(S.x, S.y, gd.n_frames);
    double A[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        A[k] = uniform_f64(A_g[k]);
    const double ifx = 1.0 / gd.fx64, ify = 1.0 / gd.fy64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        double acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            acc[q] = 0.0;
#pragma unroll 1
        for (int k = threadIdx.x; k < S.w; k += kFeatThreads) {
            const float4 qm = gd.fpts[2 * (S.z + k)];
            const float4 qn = gd.fpts[2 * (S.z + k) + 1];
            if (pass == 0)
                feature_match_values<0>(gd, A, qm, qn, ifx, ify, acc);
            else
                feature_match_values<1>(gd, A, qm, qn, ifx, ify, acc);
        }
        wave_sum16(acc, lane);
        if (lane < 16)
            red[wave][16 * pass + wave_sum16_index(lane)] = acc[0];
        __builtin_amdgcn_sched_barrier(0);   // the passes do not overlap (registers)
    }
    __syncthreads();
    if (threadIdx.x < 30) {
        double v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kFeatThreads / 64; ++w)
            v += red[w][threadIdx.x];
        if (threadIdx.x >= 28) {
            Sm[threadIdx.x - 28][7] = v;
        } else {
            int k = 0, rem = threadIdx.x;   // (k, l), k <= l, of the upper index
            while (rem >= 7 - k) {
                rem -= 7 - k;
                ++k;
            }
            Sm[k][k + rem] = v;
            Sm[k + rem][k] = v;
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= kFeatFields)
        return;
    double v;
    if (t >= 90) {
        v = Sm[t - 90][7];   // energy, count
    } else {
        int a, c = -1;
        if (t < 78) {
            // upper index of (a, c) in a 12 x 12 upper triangle, row-major
            a = 0;
            int rem = t;
            while (rem >= 12 - a) {
                rem -= 12 - a;
                ++a;
            }
            c = a + rem;
        } else {
            a = t - 78;
        }
        v = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double* Ti = Tinv[0] + 4 * r;
            const double* Tj = Tinv[1] + 4 * r;
            int ia0, ia1;
            double ca0, ca1;
            feat_jac_sparse(Ti, Tj, a, ia0, ca0, ia1, ca1);
            if (c >= 0) {
                int ic0, ic1;
                double cc0, cc1;
                feat_jac_sparse(Ti, Tj, c, ic0, cc0, ic1, cc1);
                v += ca0 * (cc0 * Sm[ia0][ic0] + cc1 * Sm[ia0][ic1]) + ca1 * (cc0 * Sm[ia1][ic0] + cc1 * Sm[ia1][ic1]);
            } else {
                // e_r = (t'_i - t'_j)_r + rho . p_m - sig . p_n
                const double ar[7] = {Ti[3] - Tj[3], Ti[0], Ti[1], Ti[2], -Tj[0], -Tj[1], -Tj[2]};
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int l = 0; l < 7; ++l) {
                    s0 += Sm[ia0][l] * ar[l];
                    s1 += Sm[ia1][l] * ar[l];
                }
                v += ca0 * s0 + ca1 * s1;
            }
        }
    }
    gd.fpartials[(size_t)fi.y * kFeatStride + t] = v;
}

// ------------------------------------------------------------ launchers

void launch_preprocess(const float* depth, const uint8_t* mask, int W, int H, float cx, float cy, float ifx,
                       float ify, float4* map, uint8_t* flag, int* row_cnt, int* total, float4* src_nz,
                       uint32_t* src_uv, hipStream_t st)
{
    dim3 blk(32, 8), grd((W + 31) / 32, (H + 7) / 8);
    preprocess_map_kernel<<<grd, blk, 0, st>>>(depth, mask, W, H, cx, cy, ifx, ify, map, flag);
    row_count_kernel<<<H, 256, 0, st>>>(flag, W, row_cnt);
    row_scan_kernel<<<1, kScanThreads, 0, st>>>(row_cnt, H, total);
    row_scatter_kernel<<<H, 256, 0, st>>>(map, flag, row_cnt, W, src_nz, src_uv);
}

void launch_match_points(const float* di, const uint8_t* mi, const float* dj, const uint8_t* mj, int W, int H,
                         const float* uvi, const float* uvj, int n, float4* out, hipStream_t st)
{
    if (n > 0)
        match_points_kernel<<<(n + 255) / 256, 256, 0, st>>>(di, mi, dj, mj, W, H, uvi, uvj, n, out);
}

int assoc_ppt_supported(int ppt) { return ppt == 1 || ppt == 2 || ppt == 4 || ppt == 8; }

template <bool LEARNED>
static void launch_assoc_t(const GraphDev* gds, const WorkItem* items, int n_items, int ppt, int precision,
                           int iteration, const int2* fitems, int n_fitems, unsigned* ctr, int blocks_per_xcd,
                           hipStream_t st)
{
    const int per_xcd = (n_items + 7) / 8;
    const int nf8 = (n_fitems + 7) & ~7;
    if (ctr && n_items > 0) {
        const int bpx = std::max(1, std::min(blocks_per_xcd, per_xcd));
        const int grid = nf8 + 8 * bpx;
#define PG_PERSIST_LAUNCH(P, B)                                                                            \
    assoc_persistent_kernel<P, LEARNED, B><<<grid, kAssocThreads, 0, st>>>(gds, items, n_items, per_xcd,    \
                                                                          iteration, fitems, n_fitems, ctr, \
                                                                          8 * bpx)
        const bool bf = precision == 1;
        switch (ppt) {
        case 1: if (bf) PG_PERSIST_LAUNCH(1, true); else PG_PERSIST_LAUNCH(1, false); break;
        case 2: if (bf) PG_PERSIST_LAUNCH(2, true); else PG_PERSIST_LAUNCH(2, false); break;
        case 8: if (bf) PG_PERSIST_LAUNCH(8, true); else PG_PERSIST_LAUNCH(8, false); break;
        default: if (bf) PG_PERSIST_LAUNCH(4, true); else PG_PERSIST_LAUNCH(4, false); break;
        }
#undef PG_PERSIST_LAUNCH
        return;
    }
    const int grid = nf8 + 8 * per_xcd;
#define PG_ASSOC_LAUNCH(K)                                                                                  \
    switch (ppt) {                                                                                          \
    case 1: K<1, LEARNED><<<grid, kAssocThreads, 0, st>>>(gds, items, n_items, per_xcd, iteration, fitems, n_fitems); break;  \
    case 2: K<2, LEARNED><<<grid, kAssocThreads, 0, st>>>(gds, items, n_items, per_xcd, iteration, fitems, n_fitems); break;  \
    case 8: K<8, LEARNED><<<grid, kAssocThreads, 0, st>>>(gds, items, n_items, per_xcd, iteration, fitems, n_fitems); break;  \
    default: K<4, LEARNED><<<grid, kAssocThreads, 0, st>>>(gds, items, n_items, per_xcd, iteration, fitems, n_fitems); break; \
    }
    if (precision == 1) {
        PG_ASSOC_LAUNCH(assoc_bf16x3_kernel)
    } else {
        PG_ASSOC_LAUNCH(assoc_kernel)
    }
#undef PG_ASSOC_LAUNCH
}

void launch_assoc(const GraphDev* gds, const WorkItem* items, int n_items, int ppt, int precision, bool learned,
                  int iteration, const int2* fitems, int n_fitems, unsigned* ctr, int blocks_per_xcd,
                  hipStream_t st)
{
    if (n_items <= 0 && n_fitems <= 0)
        return;
    if (learned)
        launch_assoc_t<true>(gds, items, n_items, ppt, precision, iteration, fitems, n_fitems, ctr,
                             blocks_per_xcd, st);
    else
        launch_assoc_t<false>(gds, items, n_items, ppt, precision, iteration, fitems, n_fitems, ctr,
                              blocks_per_xcd, st);
}

// Resident blocks per XCD of the persistent association kernel for these
// settings (occupancy x compute units / 8), 0 if unknown.
int assoc_persistent_blocks(int ppt, int precision, bool learned)
{
    const void* k = nullptr;
    const bool bf = precision == 1;
#define PG_K(P)                                                                                               \
    k = learned ? (bf ? (const void*)assoc_persistent_kernel<P, true, true>                                  \
                      : (const void*)assoc_persistent_kernel<P, true, false>)                                \
                : (bf ? (const void*)assoc_persistent_kernel<P, false, true>                                 \
                      : (const void*)assoc_persistent_kernel<P, false, false>)
    switch (ppt) {
    case 1: PG_K(1); break;
    case 2: PG_K(2); break;
    case 8: PG_K(8); break;
    default: PG_K(4); break;
    }
#undef PG_K
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kAssocThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus / 8;
}

void launch_assoc_debug(const GraphDev* gds, int HW, int i, int j, int iteration, int* target, float* r,
                        float* uv, float* feat, float* sigma, hipStream_t st)
{
    assoc_debug_kernel<<<(HW + 255) / 256, 256, 0, st>>>(gds, i, j, iteration, target, r, uv, feat, sigma);
}

__global__ void mlp_to_float_kernel(const __half* __restrict__ p16, float* __restrict__ p32)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < kMlpParams)
        p32[q] = __half2float(p16[q]);
}

void launch_mlp_to_float(const __half* p16, float* p32, hipStream_t st)
{
    mlp_to_float_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(p16, p32);
}

void launch_prune(const GraphDev* gds, const WorkItem* pitems, int n_pitems, const int2* pframes, int n_pframes,
                  int max_src, hipStream_t st)
{
    if (n_pitems > 0)
        prune_score_kernel<<<n_pitems, kPruneThreads, 0, st>>>(gds, pitems);
    if (n_pframes > 0) {
        // blocks per frame: at most kSelectMaxSlices slices per wave run
        const int per_block = kSelectWaves * 64 * kSelectMaxSlices;
        const int bpf = std::max(kSelectBlocks, (max_src + per_block - 1) / per_block);
        if (max_src <= kSelectStageKeys)
            prune_select_kernel<true><<<n_pframes * bpf, kSelectThreads, 0, st>>>(gds, pframes, bpf);
        else
            prune_select_kernel<false><<<n_pframes * bpf, kSelectThreads, 0, st>>>(gds, pframes, bpf);
    }
}

}  // namespace pg
