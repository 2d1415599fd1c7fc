// Tile rasteriser, forward and backward, for gfx950 (wave64).
//
// One wave (64 lanes) owns one screen tile of TW x TH pixels; lane l holds the
// TW*TH/64 pixels of column l % TW, rows l / TW + k * (64 / TW).  The tile's
// depth-sorted Gaussian list is walked in batches of 64 records staged in LDS
// (structure of arrays; every lane reads the same record, a broadcast).
//
// Per (pixel, Gaussian) pair, with u = (ux, uy, 1) the pixel's view-space ray
// and the record (centre h + l, A, v0, mz, K', E'; see vgr_internal.h):
//   d = pixel centre - h - l,  a = A d,  w = v0 + a,  n = v0 x a,
//   num = |n|^2,  qw = |w|^2,  se = (log2 e / 2) mz^2
//   bound test: num > E' qw  =>  alpha < alpha_min, skip (no transcendental)
//   r = 1/sqrt(qw), y = K' |u| r exp2(-se num r^2)        (= log2(e) x, Sec. 4.2)
//   skip if y < tau log2(e); y = min(y, -log2(1 - alpha_max))
//   1 - alpha = exp2(-y); stop the pixel when T (1 - alpha) < T_min, else
//   C += c alpha T, T *= 1 - alpha                          (Sec. 4.1)
// The lane's column shares d_x, A[:,0] d_x and v0 + A[:,0] d_x over its pixels;
// uy[] holds the pixel-centre row coordinates.
// The wave leaves its list as soon as every one of its pixels has stopped.
// X-ray mode sums y over the whole list instead (Sec. 6.2).
//
// The backward walks each pixel's list in reverse from its last blended
// Gaussian, recovering T in front of Gaussian i as T_after / (1 - alpha_i)
// from the stored final transmittance, and the colour behind it as a running
// sum starting at T_final * bg.  The geometric gradient of each pair is kept
// as moments in the Gaussian's L-frame (see the record-gradient layout in
// vgr_internal.h).  Per Gaussian, the 16 partial sums of the wave are reduced
// with a transpose-reduce (17 shuffles) and added with one 16-lane atomic.
#include "vgr_internal.h"

namespace vgr {

namespace {

__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct Rec {
    float hx, hy, lx, ly, A00, A01, A10, A11, A20, A21, v0x, v0y, v0z, mz, K, E, se;
};

__device__ __forceinline__ Rec load_rec(const float4 *g0, const float4 *g1, const float4 *g2,
                                        const float4 *g3, int q)
{
    const float4 a = g0[q], b = g1[q], c = g2[q], d = g3[q];
    Rec r;
    r.hx = a.x; r.hy = a.y; r.lx = a.z; r.ly = a.w;
    r.A00 = b.x; r.A01 = b.y; r.A10 = b.z; r.A11 = b.w;
    r.A20 = c.x; r.A21 = c.y; r.v0x = c.z; r.v0y = c.w;
    r.v0z = d.x; r.mz = d.y; r.K = d.z; r.E = d.w;
    r.se = (0.5f * kLog2e) * r.mz * r.mz;
    return r;
}

// Per-lane column terms shared by the lane's pixels (pxc = px + 0.5).
struct ColTerms {
    float dx, ax0, ax1, ax2, wx0, wx1, wx2;
};

__device__ __forceinline__ ColTerms col_terms(const Rec &r, float pxc)
{
    ColTerms c;
    c.dx = (pxc - r.hx) - r.lx;
    c.ax0 = r.A00 * c.dx;
    c.ax1 = r.A10 * c.dx;
    c.ax2 = r.A20 * c.dx;
    c.wx0 = r.v0x + c.ax0;
    c.wx1 = r.v0y + c.ax1;
    c.wx2 = r.v0z + c.ax2;
    return c;
}

// Geometry of one pair (pyc = py + 0.5).  Returns false when the bound test
// rejects the pair.
struct PairGeom {
    float dy, a0, a1, a2, w0, w1, w2, n0, n1, n2, num, qw;
};

__device__ __forceinline__ bool pair_geom(const Rec &r, const ColTerms &c, float pyc, PairGeom &g)
{
    g.dy = (pyc - r.hy) - r.ly;
    g.a0 = __fmaf_rn(r.A01, g.dy, c.ax0);
    g.a1 = __fmaf_rn(r.A11, g.dy, c.ax1);
    g.a2 = __fmaf_rn(r.A21, g.dy, c.ax2);
    g.w0 = __fmaf_rn(r.A01, g.dy, c.wx0);
    g.w1 = __fmaf_rn(r.A11, g.dy, c.wx1);
    g.w2 = __fmaf_rn(r.A21, g.dy, c.wx2);
    g.n0 = __fmaf_rn(r.v0y, g.a2, -r.v0z * g.a1);
    g.n1 = __fmaf_rn(r.v0z, g.a0, -r.v0x * g.a2);
    g.n2 = __fmaf_rn(r.v0x, g.a1, -r.v0y * g.a0);
    g.num = __fmaf_rn(g.n0, g.n0, __fmaf_rn(g.n1, g.n1, g.n2 * g.n2));
    g.qw = __fmaf_rn(g.w0, g.w0, __fmaf_rn(g.w1, g.w1, g.w2 * g.w2));
    return !(g.num > r.E * g.qw);
}

template <int TW, int TH>
struct TileMap {
    static constexpr int PPL = TW * TH / 64;
    static constexpr int RS = 64 / TW;
    static_assert(TW * TH % 64 == 0 && 64 % TW == 0, "tile shape");
};

__device__ __forceinline__ int find_view(const ViewInfo *views, int n_views, int gt)
{
    int v = 0;
    for (int k = 1; k < n_views; ++k)
        if (views[k].tile_off <= gt) v = k;
    return v;
}

template <int TW, int TH, int MODE, bool COUNT>
__global__ __launch_bounds__(64) void raster_fwd_kernel(RenderParams rp, Buffers b)
{
    constexpr int PPL = TileMap<TW, TH>::PPL;
    constexpr int RS = TileMap<TW, TH>::RS;
    __shared__ float4 s_g0[64], s_g1[64], s_g2[64], s_g3[64], s_c[64];

    const int gt = blockIdx.x;
    const int v = find_view(b.views, rp.n_views, gt);
    const ViewInfo &vi = b.views[v];
    const int lt = gt - vi.tile_off;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * TW + (lane % TW);
    const int py0 = ty * TH + lane / TW;
    const int W = vi.width, H = vi.height;
    const float pxc = (float)px + 0.5f;
    const float ux = (pxc - vi.cx) / vi.fx;

    float uy[PPL], un[PPL], T[PPL], C0[PPL], C1[PPL], C2[PPL];
    int last[PPL];
    bool act[PPL];
    uint32_t c_test = 0, c_full = 0, c_blend = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        uy[k] = (float)py + 0.5f;   // pixel-centre row coordinate
        const float uyn = (uy[k] - vi.cy) / vi.fy;
        un[k] = sqrtf(ux * ux + uyn * uyn + 1.0f);
        act[k] = px < W && py < H;
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        last[k] = -1;
    }
    const uint2 range = b.ranges[gt];
    const float tau2 = rp.tau2, ymax = rp.ymax, Tmin = rp.T_min;

    for (uint32_t bs = range.x; bs < range.y; bs += 64) {
        bool anyact = false;
#pragma unroll
        for (int k = 0; k < PPL; ++k) anyact |= act[k];
        if (!__any(anyact)) break;
        const uint32_t j = bs + lane;
        if (j < range.y) {
            const uint32_t item = b.inst_val[j];
            const float4 *gp = b.geom + (size_t)item * 4;
            s_g0[lane] = gp[0];
            s_g1[lane] = gp[1];
            s_g2[lane] = gp[2];
            s_g3[lane] = gp[3];
            if (MODE == VGR_MODE_COLOR) s_c[lane] = b.color[item];
        }
        __syncthreads();
        const int nb = (int)min(64u, range.y - bs);
        for (int qi = 0; qi < nb; ++qi) {
            if (MODE == VGR_MODE_COLOR) {
                bool a2 = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) a2 |= act[k];
                if (!__any(a2)) break;
            }
            const Rec r = load_rec(s_g0, s_g1, s_g2, s_g3, qi);
            float4 col;
            if (MODE == VGR_MODE_COLOR) col = s_c[qi];
            const ColTerms ct = col_terms(r, pxc);
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                if (!act[k]) continue;
                if (COUNT) ++c_test;
                PairGeom g;
                if (!pair_geom(r, ct, uy[k], g)) continue;
                if (COUNT) ++c_full;
                const float rq = fast_rsq(g.qw);
                const float ex = fast_exp2(-(r.se * g.num * (rq * rq)));
                float y = r.K * un[k] * rq * ex;
                if (y < tau2) continue;
                if (MODE == VGR_MODE_COLOR) {
                    y = fminf(y, ymax);
                    const float om = fast_exp2(-y);
                    const float Tn = T[k] * om;
                    if (Tn < Tmin) {
                        act[k] = false;
                        continue;
                    }
                    const float wgt = (1.0f - om) * T[k];
                    C0[k] = __fmaf_rn(col.x, wgt, C0[k]);
                    C1[k] = __fmaf_rn(col.y, wgt, C1[k]);
                    C2[k] = __fmaf_rn(col.z, wgt, C2[k]);
                    T[k] = Tn;
                    last[k] = (int)(bs + qi);
                } else {
                    C0[k] += y;
                    last[k] += 1;   // number of terms (starts at -1)
                }
                if (COUNT) ++c_blend;
            }
        }
        __syncthreads();
    }

    const int64_t HW = (int64_t)W * H;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        if (px < W && py < H) {
            const int64_t idx = (int64_t)py * W + px;
            const int64_t pidx = vi.pix_off + idx;
            if (MODE == VGR_MODE_COLOR) {
                vi.out[idx] = __fmaf_rn(T[k], rp.bg[0], C0[k]);
                vi.out[HW + idx] = __fmaf_rn(T[k], rp.bg[1], C1[k]);
                vi.out[2 * HW + idx] = __fmaf_rn(T[k], rp.bg[2], C2[k]);
                b.T_final[pidx] = T[k];
                b.last_pos[pidx] = last[k];
                b.last_id[pidx] = last[k] >= 0
                    ? (int32_t)((int64_t)b.inst_val[last[k]] - (int64_t)v * rp.n) : -1;
            } else {
                vi.out[idx] = C0[k] * kLn2;
                b.T_final[pidx] = fast_exp2(-C0[k]);
                b.last_pos[pidx] = (int32_t)range.y - 1;
                b.last_id[pidx] = last[k] + 1;
            }
        }
    }
    if (COUNT) {
        atomicAdd(&b.counters[0], (unsigned long long)c_test);
        atomicAdd(&b.counters[1], (unsigned long long)c_full);
        atomicAdd(&b.counters[2], (unsigned long long)c_blend);
    }
}

// Sum v[0..15] over the 64 lanes.  Afterwards lane l with (l & 3) == 0 holds
// the total of index ((l>>5)&1)*8 + ((l>>4)&1)*4 + ((l>>3)&1)*2 + ((l>>2)&1).
__device__ __forceinline__ float wave_reduce16(float v[16], int lane)
{
    {
        const bool hi = lane & 32;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float send = hi ? v[k] : v[k + 8];
            const float keep = hi ? v[k + 8] : v[k];
            v[k] = keep + __shfl_xor(send, 32, 64);
        }
    }
    {
        const bool hi = lane & 16;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float send = hi ? v[k] : v[k + 4];
            const float keep = hi ? v[k + 4] : v[k];
            v[k] = keep + __shfl_xor(send, 16, 64);
        }
    }
    {
        const bool hi = lane & 8;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float send = hi ? v[k] : v[k + 2];
            const float keep = hi ? v[k + 2] : v[k];
            v[k] = keep + __shfl_xor(send, 8, 64);
        }
    }
    {
        const bool hi = lane & 4;
        const float send = hi ? v[0] : v[1];
        const float keep = hi ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, 4, 64);
    }
    v[0] += __shfl_xor(v[0], 2, 64);
    v[0] += __shfl_xor(v[0], 1, 64);
    return v[0];
}

template <int TW, int TH, int MODE, bool COUNT>
__global__ __launch_bounds__(64) void raster_bwd_kernel(RenderParams rp, Buffers b)
{
    constexpr int PPL = TileMap<TW, TH>::PPL;
    constexpr int RS = TileMap<TW, TH>::RS;
    constexpr int NCH = MODE == VGR_MODE_COLOR ? 3 : 1;
    __shared__ float4 s_g0[64], s_g1[64], s_g2[64], s_g3[64], s_c[64];
    __shared__ uint32_t s_item[64];

    const int gt = blockIdx.x;
    const int v = find_view(b.views, rp.n_views, gt);
    const ViewInfo &vi = b.views[v];
    const int lt = gt - vi.tile_off;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * TW + (lane % TW);
    const int py0 = ty * TH + lane / TW;
    const int W = vi.width, H = vi.height;
    const int64_t HW = (int64_t)W * H;
    const float pxc = (float)px + 0.5f;
    const float ux = (pxc - vi.cx) / vi.fx;
    const uint2 range = b.ranges[gt];

    float uy[PPL], un[PPL], T[PPL], g[PPL][NCH], B[PPL][NCH];
    int last[PPL];
    int maxlast = -1;
    uint32_t c_test = 0, c_full = 0, c_blend = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        uy[k] = (float)py + 0.5f;   // pixel-centre row coordinate
        const float uyn = (uy[k] - vi.cy) / vi.fy;
        un[k] = sqrtf(ux * ux + uyn * uyn + 1.0f);
        const bool inside = px < W && py < H;
        const int64_t idx = (int64_t)py * W + px;
        last[k] = inside ? b.last_pos[vi.pix_off + idx] : -1;
        T[k] = inside ? b.T_final[vi.pix_off + idx] : 1.0f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            g[k][c] = inside ? vi.dL[c * HW + idx] : 0.0f;
            B[k][c] = T[k] * rp.bg[c];
        }
        maxlast = max(maxlast, last[k]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, off, 64));
    if (maxlast < (int)range.x) return;   // uniform: no pixel of this tile blended anything
    const float tau2 = rp.tau2, ymax = rp.ymax;
    float *rg = reinterpret_cast<float *>(b.rgrad);
    const int red_idx = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                        ((lane >> 2) & 1);

    for (int be = maxlast + 1; be > (int)range.x; be -= 64) {
        const int bs = max((int)range.x, be - 64);
        const int j = bs + lane;
        if (j < be) {
            const uint32_t item = b.inst_val[j];
            const float4 *gp = b.geom + (size_t)item * 4;
            s_item[lane] = item;
            s_g0[lane] = gp[0];
            s_g1[lane] = gp[1];
            s_g2[lane] = gp[2];
            s_g3[lane] = gp[3];
            if (MODE == VGR_MODE_COLOR) s_c[lane] = b.color[item];
        }
        __syncthreads();
        for (int qi = be - 1 - bs; qi >= 0; --qi) {
            const int jpos = bs + qi;
            const Rec r = load_rec(s_g0, s_g1, s_g2, s_g3, qi);
            float4 col;
            if (MODE == VGR_MODE_COLOR) col = s_c[qi];
            const ColTerms ct = col_terms(r, pxc);
            float acc[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
            bool touched = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                if (jpos > last[k]) continue;
                if (COUNT) ++c_test;
                PairGeom pg;
                if (!pair_geom(r, ct, uy[k], pg)) continue;
                if (COUNT) ++c_full;
                const float rq = fast_rsq(pg.qw);
                const float rq2 = rq * rq;
                const float ex = fast_exp2(-(r.se * pg.num * rq2));
                const float y = r.K * un[k] * rq * ex;
                if (y < tau2) continue;
                if (COUNT) ++c_blend;
                float dy;
                if (MODE == VGR_MODE_COLOR) {
                    const bool clamped = y > ymax;
                    const float om = fast_exp2(-fminf(y, ymax));
                    const float inv = fast_rcp(om);
                    const float alpha = 1.0f - om;
                    const float Tb = T[k] * inv;
                    const float da = g[k][0] * (col.x * Tb - B[k][0] * inv) +
                                     g[k][1] * (col.y * Tb - B[k][1] * inv) +
                                     g[k][2] * (col.z * Tb - B[k][2] * inv);
                    const float wgt = alpha * Tb;
                    acc[10] = __fmaf_rn(g[k][0], wgt, acc[10]);
                    acc[11] = __fmaf_rn(g[k][1], wgt, acc[11]);
                    acc[12] = __fmaf_rn(g[k][2], wgt, acc[12]);
                    B[k][0] = __fmaf_rn(col.x, wgt, B[k][0]);
                    B[k][1] = __fmaf_rn(col.y, wgt, B[k][1]);
                    B[k][2] = __fmaf_rn(col.z, wgt, B[k][2]);
                    T[k] = Tb;
                    dy = clamped ? 0.0f : da * kLn2 * om;
                } else {
                    dy = g[k][0] * kLn2;
                }
                touched = true;
                // t = dL/d(ln x) = dL/dy * y;  dL/dK' = dy |u| r exp2(-e)
                const float t = dy * y;
                acc[9] = __fmaf_rn(dy, un[k] * rq * ex, acc[9]);
                // z = mz (w x n) / |w|^2 = L (m - gamma u);  w' = w / |w|
                const float cz = r.mz * rq2;
                const float z0 = cz * (pg.w1 * pg.n2 - pg.w2 * pg.n1);
                const float z1 = cz * (pg.w2 * pg.n0 - pg.w0 * pg.n2);
                const float z2 = cz * (pg.w0 * pg.n1 - pg.w1 * pg.n0);
                const float p0 = pg.w0 * rq, p1 = pg.w1 * rq, p2 = pg.w2 * rq;
                acc[6] = __fmaf_rn(t, z0, acc[6]);
                acc[7] = __fmaf_rn(t, z1, acc[7]);
                acc[8] = __fmaf_rn(t, z2, acc[8]);
                acc[0] = __fmaf_rn(t, __fmaf_rn(p0, p0, z0 * z0), acc[0]);
                acc[1] = __fmaf_rn(t, __fmaf_rn(p0, p1, z0 * z1), acc[1]);
                acc[2] = __fmaf_rn(t, __fmaf_rn(p0, p2, z0 * z2), acc[2]);
                acc[3] = __fmaf_rn(t, __fmaf_rn(p1, p1, z1 * z1), acc[3]);
                acc[4] = __fmaf_rn(t, __fmaf_rn(p1, p2, z1 * z2), acc[4]);
                acc[5] = __fmaf_rn(t, __fmaf_rn(p2, p2, z2 * z2), acc[5]);
            }
            if (__any(touched)) {
                const float tot = wave_reduce16(acc, lane);
                if ((lane & 3) == 0) {
                    const uint32_t item = s_item[qi];
                    atomicAdd(rg + (size_t)item * 16 + red_idx, tot);
                }
            }
        }
        __syncthreads();
    }
    if (COUNT) {
        atomicAdd(&b.counters[3], (unsigned long long)c_test);
        atomicAdd(&b.counters[4], (unsigned long long)c_full);
        atomicAdd(&b.counters[5], (unsigned long long)c_blend);
    }
}

template <int TW, int TH>
hipError_t fwd_shape(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    if (rp.mode == VGR_MODE_COLOR) {
        if (count) raster_fwd_kernel<TW, TH, VGR_MODE_COLOR, true><<<grid, block, 0, s>>>(rp, b);
        else raster_fwd_kernel<TW, TH, VGR_MODE_COLOR, false><<<grid, block, 0, s>>>(rp, b);
    } else {
        if (count) raster_fwd_kernel<TW, TH, VGR_MODE_XRAY, true><<<grid, block, 0, s>>>(rp, b);
        else raster_fwd_kernel<TW, TH, VGR_MODE_XRAY, false><<<grid, block, 0, s>>>(rp, b);
    }
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_shape(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    if (rp.mode == VGR_MODE_COLOR) {
        if (count) raster_bwd_kernel<TW, TH, VGR_MODE_COLOR, true><<<grid, block, 0, s>>>(rp, b);
        else raster_bwd_kernel<TW, TH, VGR_MODE_COLOR, false><<<grid, block, 0, s>>>(rp, b);
    } else {
        if (count) raster_bwd_kernel<TW, TH, VGR_MODE_XRAY, true><<<grid, block, 0, s>>>(rp, b);
        else raster_bwd_kernel<TW, TH, VGR_MODE_XRAY, false><<<grid, block, 0, s>>>(rp, b);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.total_tiles <= 0) return hipSuccess;
    if (rp.tile_w == 8 && rp.tile_h == 8) return fwd_shape<8, 8>(rp, b, count, s);
    if (rp.tile_w == 16 && rp.tile_h == 8) return fwd_shape<16, 8>(rp, b, count, s);
    if (rp.tile_w == 32 && rp.tile_h == 8) return fwd_shape<32, 8>(rp, b, count, s);
    return fwd_shape<16, 16>(rp, b, count, s);
}

hipError_t launch_raster_bwd(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.total_tiles <= 0) return hipSuccess;
    if (rp.tile_w == 8 && rp.tile_h == 8) return bwd_shape<8, 8>(rp, b, count, s);
    if (rp.tile_w == 16 && rp.tile_h == 8) return bwd_shape<16, 8>(rp, b, count, s);
    if (rp.tile_w == 32 && rp.tile_h == 8) return bwd_shape<32, 8>(rp, b, count, s);
    return bwd_shape<16, 16>(rp, b, count, s);
}

}  // namespace vgr
