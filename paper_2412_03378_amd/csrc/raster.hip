// Tile rasteriser, forward and backward, for gfx950 (wave64).
//
// One wave (64 lanes) owns one screen tile of TW x TH pixels; lane l holds the
// TW*TH/64 pixels of column l % TW, rows l / TW + k * (64 / TW) ("slot" k).
// Tiles are launched in the order of b.tile_order (heaviest lists first).
// The tile's depth-sorted Gaussian list is walked in batches of B records
// (B = 64 or 32, the block shape the autotuner picks with the tile shape)
// staged in LDS (structure of arrays).  The colour forward (and the X-ray
// forward with one pixel per lane) pre-tests the whole batch with broadcast
// reads and then lets every lane evaluate its own passing records in order
// (per-lane reads), so that an evaluation step is not spent on lanes whose
// pixel the record misses; it keeps each lane's pass mask of the batch for
// the backward.  The X-ray forward with several pixels per lane walks the
// batch together, reading the three float4 of the bound pre-test first and
// the other three only when some pixel of the slot passes.  The backward
// reduces its per-pair gradients per Gaussian, so lanes that share a record
// walk together: on 8x8 tiles in the volumetric colour modes each 4x4
// quarter of the tile (16 lanes) walks the records its own pixels' masks
// name, four records per step; elsewhere the whole wave walks the records
// that the union of the lanes' masks names, or, where the forward kept no
// masks, pre-tests each record as the X-ray forward does.
//
// Per (pixel, Gaussian) pair, with the record (centre h + l, A, v0, mz, K',
// bound form Q, l; see vgr_internal.h) and d = pixel centre - h - l:
//   bound pre-test f(d) = d^T Q d + 2 l^T d - 1 > margin  =>  alpha < alpha_min
//   a = A d,  w = v0 + a,  n = v0 x a,  num = |n|^2,  qw = |w|^2
//   r = 1/sqrt(qw), y = K' |u| r exp2(-se num r^2), se = (log2 e / 2) mz^2
//                                               (y = log2(e) x, Sec. 4.2)
//   skip if y < tau log2(e); y = min(y, -log2(1 - alpha_max))
//   1 - alpha = exp2(-y); stop the pixel when T (1 - alpha) < T_min, else
//   C += c alpha T, T *= 1 - alpha                          (Sec. 4.1)
// The pre-test costs three operations per pixel; everything after it runs
// under one wave-uniform branch per slot (taken when any lane's pixel in the
// slot passes), with per-lane selects instead of nested execution masks.
// The wave leaves its list as soon as every one of its pixels has stopped.
// X-ray mode sums y over the whole list instead (Sec. 6.2).
//
// The backward walks each pixel's list in reverse from its last blended
// Gaussian, recovering T in front of Gaussian i as T_after / (1 - alpha_i)
// from the stored final transmittance, and the colour behind it (through its
// dot product with dL/dC, which is all the replay needs) as a running sum
// starting at T_final * bg.  The geometric gradient of each pair is kept
// as moments in the Gaussian's L-frame (see the record-gradient layout in
// vgr_internal.h).  The partial sums (13, or 16 with the near-plane segment)
// of the lanes on one record are reduced with a transpose-reduce (lane-swap
// and DPP moves, no LDS), after which each lane holds one total, and added
// with one atomic instruction (for all four records of a quarter-walk step).
#include "vgr_internal.h"

namespace vgr {

namespace {

constexpr int kStageVec = 6;   // record float4 the rasteriser uses (g0..g5)

__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Near-plane segment factor Phi(eta) of a flagged record (K' < 0):
// eta = (gamma - t_n) / beta = mz (v0 . w) / |w| - zn |w| for the pixel's
// w = L u, t_n = zn |u| the near-plane crossing of the ray (Sec. 4.2, the
// integral from t_n on).  qw = |w|^2, rq = 1 / |w|.
__device__ __forceinline__ float near_eta(float v0x, float v0y, float v0z, float mz, float w0,
                                          float w1, float w2, float qw, float rq, float zn)
{
    const float vw = __fmaf_rn(v0x, w0, __fmaf_rn(v0y, w1, v0z * w2));
    return __fmaf_rn(mz, vw, -zn * qw) * rq;
}
__device__ __forceinline__ float norm_cdf(float e) { return 0.5f * erfcf(-0.70710678f * e); }

// Profile factor of the line integral at D^2 = se num rq2 (with se from the
// record): exp2(-(log2 e / 2) D^2) for the Gaussian, (1 - D^2)^(3/2) (0 past
// the support) for the Epanechnikov kernel.
template <bool EPAN>
__device__ __forceinline__ float profile(float se, float num, float rq2)
{
    if constexpr (EPAN) {
        const float h2 = fmaxf(1.0f - se * num * rq2, 0.0f);
        return h2 * __builtin_sqrtf(h2);
    } else {
        return fast_exp2(-(se * num * rq2));
    }
}

// Timed runs (b.wg_time set) record for each workgroup the constant-rate
// realtime counter difference between start and end, and a key of the compute unit it ran on (XCC id, then the
// shader engine, array and CU fields of HW_ID), so that the host can sum the
// busy time per compute unit (load balance).
__device__ __forceinline__ uint64_t wg_clock() { return __builtin_amdgcn_s_memrealtime(); }
__device__ __forceinline__ uint32_t cu_key()
{
    const uint32_t hw = __builtin_amdgcn_s_getreg(4 | (31 << 11));    // HW_ID
    const uint32_t xcc = __builtin_amdgcn_s_getreg(20 | (3 << 11));   // XCC_ID[3:0]
    return (xcc << 8) | ((hw >> 8) & 0xFFu);
}

// True if p holds on any active lane: a ballot of the predicate's lane mask,
// which the branch tests directly.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

template <int B>
struct Stage {
    float4 g[kStageVec][B];
    uint32_t item[B];
};

// Word of the kept pre-test mask of lane `lane` for the batch that starts at
// list position bs of global tile gt (layout: raster_keeps_masks).
template <int B>
__device__ __forceinline__ size_t mask_word(uint32_t bs, int gt, int lane)
{
    return (size_t)bs * (64 / B) + 64 * (size_t)gt + lane;
}

// Fields of the bound pre-test (g0..g2) and of the full evaluation (g3..g5).
struct PreRec {
    float hx, hy, lx, ly, Q00, Q01x2, l0x2, l1x2, Q11, A00, A10, A20;
};
struct FullRec {
    float A01, A11, A21, v0x, v0y, v0z, K, se, c0, c1, c2, mz;
};

template <class ST>
__device__ __forceinline__ PreRec load_pre(const ST &st, int q)
{
    const float4 a = st.g[0][q], b = st.g[1][q], c = st.g[2][q];
    PreRec r;
    r.hx = a.x; r.hy = a.y; r.lx = a.z; r.ly = a.w;
    r.Q00 = b.x; r.Q01x2 = b.y; r.l0x2 = b.z; r.l1x2 = b.w;
    r.Q11 = c.x; r.A00 = c.y; r.A10 = c.z; r.A20 = c.w;
    return r;
}

template <class ST>
__device__ __forceinline__ FullRec load_full(const ST &st, int q)
{
    const float4 a = st.g[3][q], b = st.g[4][q], c = st.g[5][q];
    FullRec r;
    r.A01 = a.x; r.A11 = a.y; r.A21 = a.z; r.v0x = a.w;
    r.v0y = b.x; r.v0z = b.y; r.K = b.z; r.se = b.w;
    r.c0 = c.x; r.c1 = c.y; r.c2 = c.z; r.mz = c.w;
    return r;
}

// One staged record in registers, read at a per-lane index.
struct RecRegs {
    float4 g[kStageVec];
};

template <class ST>
__device__ __forceinline__ RecRegs load_regs(const ST &st, int q)
{
    RecRegs r;
#pragma unroll
    for (int v = 0; v < kStageVec; ++v) r.g[v] = st.g[v][q];
    return r;
}

__device__ __forceinline__ PreRec pre_of4(const float4 &a, const float4 &b, const float4 &c)
{
    PreRec r;
    r.hx = a.x; r.hy = a.y; r.lx = a.z; r.ly = a.w;
    r.Q00 = b.x; r.Q01x2 = b.y; r.l0x2 = b.z; r.l1x2 = b.w;
    r.Q11 = c.x; r.A00 = c.y; r.A10 = c.z; r.A20 = c.w;
    return r;
}

__device__ __forceinline__ PreRec pre_of(const RecRegs &x)
{
    return pre_of4(x.g[0], x.g[1], x.g[2]);
}

__device__ __forceinline__ FullRec full_of(const RecRegs &x)
{
    FullRec r;
    r.A01 = x.g[3].x; r.A11 = x.g[3].y; r.A21 = x.g[3].z; r.v0x = x.g[3].w;
    r.v0y = x.g[4].x; r.v0z = x.g[4].y; r.K = x.g[4].z; r.se = x.g[4].w;
    r.c0 = x.g[5].x; r.c1 = x.g[5].y; r.c2 = x.g[5].z; r.mz = x.g[5].w;
    return r;
}

template <class ST>
__device__ __forceinline__ void stage_record(ST &st, const Buffers &b, int lane, uint32_t item)
{
    const float4 *gp = b.geom + (size_t)item * kRecVec;
#pragma unroll
    for (int v = 0; v < kStageVec; ++v) st.g[v][lane] = gp[v];
    st.item[lane] = item;
}

// Per-lane terms of the pre-test shared by the lane's pixels (pxc = px + 0.5).
struct ColTerms {
    float dx, f0, f1;
};

__device__ __forceinline__ ColTerms col_terms(const PreRec &r, float pxc)
{
    ColTerms c;
    c.dx = (pxc - r.hx) - r.lx;
    c.f0 = __fmaf_rn(c.dx, __fmaf_rn(r.Q00, c.dx, r.l0x2), -1.0f);
    c.f1 = __fmaf_rn(r.Q01x2, c.dx, r.l1x2);
    return c;
}

// Bound pre-test of one pixel (pyc = py + 0.5): true if alpha >= alpha_min is
// possible.  Writes the row offset.
__device__ __forceinline__ bool pre_test(const PreRec &r, const ColTerms &c, float pyc, float &dy)
{
    dy = (pyc - r.hy) - r.ly;
    const float f = __fmaf_rn(dy, __fmaf_rn(r.Q11, dy, c.f1), c.f0);
    return !(f > kConicMargin);
}

struct PairGeom {
    float a0, a1, a2, w0, w1, w2, n0, n1, n2, num, qw;
};

__device__ __forceinline__ void pair_geom(const PreRec &p, const FullRec &r, float dx, float dy,
                                          PairGeom &g)
{
    g.a0 = __fmaf_rn(r.A01, dy, p.A00 * dx);
    g.a1 = __fmaf_rn(r.A11, dy, p.A10 * dx);
    g.a2 = __fmaf_rn(r.A21, dy, p.A20 * dx);
    g.w0 = r.v0x + g.a0;
    g.w1 = r.v0y + g.a1;
    g.w2 = r.v0z + g.a2;
    g.n0 = __fmaf_rn(r.v0y, g.a2, -r.v0z * g.a1);
    g.n1 = __fmaf_rn(r.v0z, g.a0, -r.v0x * g.a2);
    g.n2 = __fmaf_rn(r.v0x, g.a1, -r.v0y * g.a0);
    g.num = __fmaf_rn(g.n0, g.n0, __fmaf_rn(g.n1, g.n1, g.n2 * g.n2));
    g.qw = __fmaf_rn(g.w0, g.w0, __fmaf_rn(g.w1, g.w1, g.w2 * g.w2));
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

// Pair counts (per lane) and wave-level visit counts (kept by lane 0): a
// visit is one Gaussian against one slot of the wave's pixels; a full visit
// is one that takes the evaluation branch.
struct Counts {
    uint32_t test = 0, full = 0, blend = 0, visits = 0, visits_full = 0;
};

template <int TW, int TH, int MODE, bool COUNT, int B>
__global__ __launch_bounds__(64) void raster_fwd_kernel(RenderParams rp, Buffers b)
{
    static_assert(B == 32 || B == 64, "records per batch");
    constexpr int PPL = TileMap<TW, TH>::PPL;
    constexpr int RS = TileMap<TW, TH>::RS;
    constexpr bool COLOR = MODE != VGR_MODE_XRAY && MODE != kModeXrayNear && MODE != kModeXrayEpan;
    constexpr bool SPLAT = MODE == kModeSplat;   // colour with the 3DGS splatting alpha
    constexpr bool NEAR = MODE == kModeColorNear || MODE == kModeXrayNear;
    constexpr bool EPAN = MODE == kModeColorEpan || MODE == kModeXrayEpan;
    __shared__ Stage<B> st;

    const bool timed = b.wg_time != nullptr;   // uniform
    const uint64_t t_start = timed ? wg_clock() : 0;
    const int gt = (int)b.tile_order[blockIdx.x];
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

    float pyc[PPL], un[PPL], T[PPL], C0[PPL], C1[PPL], C2[PPL];
    int last[PPL];
    bool act[PPL];
    Counts n;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        pyc[k] = (float)py + 0.5f;
        const float uyn = (pyc[k] - vi.cy) / vi.fy;
        un[k] = sqrtf(ux * ux + uyn * uyn + 1.0f);
        act[k] = px < W && py < H;
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        last[k] = -1;
    }
    const uint2 range = b.ranges[gt];
    const float tau2 = rp.tau2, ymax = rp.ymax, Tmin = rp.T_min;
    const float amin = rp.amin, amax = rp.amax;
    const float zn = vi.znear;

    for (uint32_t bs = range.x; bs < range.y; bs += B) {
        const uint32_t j = bs + lane;
        if (lane < B && j < range.y) stage_record(st, b, lane, b.inst_val[j]);
        __syncthreads();
        const int nb = (int)min((uint32_t)B, range.y - bs);
        if constexpr (PPL == 1 || COLOR) {
            // Phase 1: bound pre-test of the whole batch (broadcast records);
            // bit q of mask[k] marks record q as passing for the lane's slot k.
            // The two 32-record halves fill 32-bit words, each bit set by one
            // select of a wave-uniform constant.
            uint32_t mhalf[2][PPL];
    #pragma unroll
            for (int k = 0; k < PPL; ++k) mhalf[1][k] = 0u;   // B = 32: one half
    #pragma unroll
            for (int h = 0; h < B / 32; ++h) {
    #pragma unroll
                for (int k = 0; k < PPL; ++k) mhalf[h][k] = 0u;
                const int qend = min(nb, 32 * h + 32);
                for (int qi = 32 * h; qi < qend; ++qi) {
                    const float4 g0 = st.g[0][qi], g1 = st.g[1][qi], g2 = st.g[2][qi];
                    const PreRec pr = pre_of4(g0, g1, g2);
                    const ColTerms ct = col_terms(pr, pxc);
                    const uint32_t bit = 1u << (qi & 31);
    #pragma unroll
                    for (int k = 0; k < PPL; ++k) {
                        float dy;
                        const bool pass = act[k] && pre_test(pr, ct, pyc[k], dy);
                        mhalf[h][k] |= pass ? bit : 0u;
                        if (COUNT) {
                            n.test += act[k] ? 1u : 0u;
                            const bool anyl = wave_any(act[k]);
                            n.visits += (lane == 0 && anyl) ? 1u : 0u;
                        }
                    }
                }
            }
            uint64_t mask[PPL];
    #pragma unroll
            for (int k = 0; k < PPL; ++k) mask[k] = ((uint64_t)mhalf[1][k] << 32) | mhalf[0][k];
            // kept for the backward (layout: raster_keeps_masks)
    #pragma unroll
            for (int k = 0; k < PPL; ++k)
                b.pmask[mask_word<B>(bs, gt, lane) * PPL + k] = mask[k];
            // Phase 2: every lane evaluates and blends its own passing records in
            // list order, one per step (records read from LDS at per-lane
            // addresses), so a step does useful work on every lane that still has
            // a record left instead of only on those that pass one shared record.
    #pragma unroll
            for (int k = 0; k < PPL; ++k) {
                uint64_t mk = mask[k];
                bool has = mk != 0 && act[k];
                if (wave_any(has)) do {                          // wave-uniform loop
                    const int qi = has ? (int)__builtin_ctzll(mk) : 0;
                    mk &= mk - 1;
                    if (COUNT) {
                        n.full += has ? 1u : 0u;
                        n.visits_full += lane == 0 ? 1u : 0u;
                    }
                    const RecRegs rr = load_regs(st, qi);
                    const PreRec pr = pre_of(rr);
                    const FullRec fr = full_of(rr);
                    const float dx = (pxc - pr.hx) - pr.lx;
                    const float dy = (pyc[k] - pr.hy) - pr.ly;
                    float y, om, wa;   // log2(e) x (volumetric), 1 - alpha, alpha
                    bool bl;
                    if constexpr (SPLAT) {
                        // alpha = o exp(-1/2 d^T C d) (the 3DGS splat)
                        const float e = __fmaf_rn(dx, __fmaf_rn(fr.A01, dx, fr.A11 * dy),
                                                  fr.A21 * (dy * dy));
                        const float al = fr.K * fast_exp2(-e);
                        bl = has && !(al < amin);
                        wa = al > amax ? amax : al;
                        om = 1.0f - wa;
                        y = 0.0f;
                    } else {
                        PairGeom g;
                        pair_geom(pr, fr, dx, dy, g);
                        const float rq = fast_rsq(g.qw);
                        const float ex = profile<EPAN>(fr.se, g.num, rq * rq);
                        y = (NEAR ? fabsf(fr.K) : fr.K) * un[k] * rq * ex;
                        if constexpr (NEAR) {
                            if (fr.K < 0.0f)
                                y *= norm_cdf(near_eta(fr.v0x, fr.v0y, fr.v0z, fr.mz, g.w0, g.w1,
                                                       g.w2, g.qw, rq, zn));
                        }
                        bl = has && !(y < tau2);
                        om = fast_exp2(-(y > ymax ? ymax : y));
                        wa = 1.0f - om;
                    }
                    if constexpr (COLOR) {
                        const float Tn = T[k] * om;
                        const bool stop = bl && Tn < Tmin;
                        const bool dob = bl && !stop;
                        const float wgt = dob ? wa * T[k] : 0.0f;
                        C0[k] = __fmaf_rn(fr.c0, wgt, C0[k]);
                        C1[k] = __fmaf_rn(fr.c1, wgt, C1[k]);
                        C2[k] = __fmaf_rn(fr.c2, wgt, C2[k]);
                        T[k] = dob ? Tn : T[k];
                        last[k] = dob ? (int)(bs + qi) : last[k];
                        act[k] = act[k] && !stop;
                        if (COUNT) n.blend += dob ? 1u : 0u;
                    } else {
                        C0[k] += bl ? y : 0.0f;
                        last[k] += bl ? 1 : 0;   // number of terms (starts at -1)
                        if (COUNT) n.blend += bl ? 1u : 0u;
                    }
                    has = mk != 0 && act[k];
                } while (wave_any(has));
            }
        } else {
            // X-ray with several pixels per lane: every record of the list is
            // summed (no early stop), and one broadcast read per step is
            // shared by the lane's pixels, which measured faster than a
            // per-lane walk that re-reads the record for each pixel.
            for (int qi = 0; qi < nb; ++qi) {
                if (COLOR) {
                    bool any = false;
    #pragma unroll
                    for (int k = 0; k < PPL; ++k) any |= act[k];
                    if (!wave_any(any)) break;              // every pixel has stopped
                }
                const PreRec pr = load_pre(st, qi);
                const ColTerms ct = col_terms(pr, pxc);
    #pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    float dy;
                    const bool near = pre_test(pr, ct, pyc[k], dy);   // always evaluated: sets dy
                    const bool pass = act[k] && near;
                    const bool anyp = wave_any(pass);
                    if (COUNT) {
                        n.test += act[k] ? 1u : 0u;
                        const bool anyl = wave_any(act[k]);
                        n.visits += (lane == 0 && anyl) ? 1u : 0u;
                        n.visits_full += (lane == 0 && anyp) ? 1u : 0u;
                    }
                    if (!anyp) continue;                  // wave-uniform
                    if (COUNT) n.full += pass ? 1u : 0u;
                    const FullRec fr = load_full(st, qi);
                    PairGeom g;
                    pair_geom(pr, fr, ct.dx, dy, g);
                    const float rq = fast_rsq(g.qw);
                    const float ex = profile<EPAN>(fr.se, g.num, rq * rq);
                    float y = (NEAR ? fabsf(fr.K) : fr.K) * un[k] * rq * ex;
                    if constexpr (NEAR) {
                        if (fr.K < 0.0f)
                            y *= norm_cdf(near_eta(fr.v0x, fr.v0y, fr.v0z, fr.mz, g.w0, g.w1, g.w2,
                                                   g.qw, rq, zn));
                    }
                    const bool bl = pass && !(y < tau2);
                    if constexpr (COLOR) {
                        if (!wave_any(bl)) continue;            // wave-uniform
                        const float om = fast_exp2(-(y > ymax ? ymax : y));
                        const float Tn = T[k] * om;
                        const bool stop = bl && Tn < Tmin;
                        const bool dob = bl && !stop;
                        const float wgt = dob ? (1.0f - om) * T[k] : 0.0f;
                        C0[k] = __fmaf_rn(fr.c0, wgt, C0[k]);
                        C1[k] = __fmaf_rn(fr.c1, wgt, C1[k]);
                        C2[k] = __fmaf_rn(fr.c2, wgt, C2[k]);
                        T[k] = dob ? Tn : T[k];
                        last[k] = dob ? (int)(bs + qi) : last[k];
                        act[k] = act[k] && !stop;
                        if (COUNT) n.blend += dob ? 1u : 0u;
                    } else {
                        C0[k] += bl ? y : 0.0f;
                        last[k] += bl ? 1 : 0;   // number of terms (starts at -1)
                        if (COUNT) n.blend += bl ? 1u : 0u;
                    }
                }
            }
        }
        __syncthreads();
        if (COLOR) {
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) any |= act[k];
            if (!wave_any(any)) break;                    // every pixel has stopped
        }
    }

    const int64_t HW = (int64_t)W * H;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        if (px < W && py < H) {
            const int64_t idx = (int64_t)py * W + px;
            const int64_t pidx = vi.pix_off + idx;
            if (COLOR) {
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
        atomicAdd(&b.counters[0], (unsigned long long)n.test);
        atomicAdd(&b.counters[1], (unsigned long long)n.full);
        atomicAdd(&b.counters[2], (unsigned long long)n.blend);
        atomicAdd(&b.counters[3], (unsigned long long)n.visits);
        atomicAdd(&b.counters[4], (unsigned long long)n.visits_full);
    }
    if (timed && lane == 0)
        b.wg_time[blockIdx.x] = make_uint2(cu_key(), (uint32_t)(wg_clock() - t_start));
}

// Sum v[0..15] over the 64 lanes (transpose-reduce).  Afterwards lane l with
// (l & 3) == 0 holds the total of index l / 4.
//   step 1: v_permlane32_swap pairs (v[k], v[k+8]); after the add, lanes 0-31
//           hold index k and lanes 32-63 index k + 8;
//   step 2: v_permlane16_swap pairs (v[k], v[k+4]); row r (16 lanes) now
//           holds indices 4 r + k, k = 0..3;
//   step 3: lanes l and l ^ 8 (DPP row rotate by 8) keep one pair of indices
//           each and send the other;
//   step 4: lanes l and 7 - l of each 8-lane half row (DPP half mirror) keep
//           one index each and send the other;
//   step 5: sums within each quad (DPP quad permutations).
__device__ __forceinline__ float swap_add32(float &a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_add16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// DPP lane moves (gfx9 encodings): row rotate right by 8, quad permutations
// [2,3,0,1] and [1,0,3,2].
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppQuadXor1 = 0xB1;

constexpr int kDppRowRor4 = 0x124;
constexpr int kDppRowRor2 = 0x122;
constexpr int kDppRowRor1 = 0x121;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_move_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// With N13 only v[0..12] are summed (v[13..15] are zero): step 1 pairs
// (v[k], v[k+8]) for k < 5, then (v[5], v[6]) and (v[7], 0), leaving seven
// slots.  Slot s and the lane bit h that picked the pair member give the
// index of the total a lane ends with, n13_index(s, h); -1: the lane holds
// no total.
__device__ __forceinline__ int n13_index(int s, int h)
{
    return s < 5 ? s + 8 * h : (s == 5 ? 5 + h : ((s == 6 && h == 0) ? 7 : -1));
}

template <bool N13, class SWAP>
__device__ __forceinline__ void pair_step1(float (&v)[16], SWAP swap_add)
{
    if constexpr (N13) {
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] = swap_add(v[k], v[k + 8]);
        v[5] = swap_add(v[5], v[6]);
        v[6] = swap_add(v[7], 0.0f);
        v[7] = 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = swap_add(v[k], v[k + 8]);
    }
}

// Index of the total lane l holds after wave_reduce16 (lanes l & 3 == 0).
template <bool N13>
__device__ __forceinline__ int wave_index(int lane)
{
    return N13 ? n13_index((lane >> 2) & 7, (lane >> 5) & 1) : lane >> 2;
}

// Steps 3 and 4 of wave_reduce16 as DPP adds with bank masks, each lane
// writing the sum of the slot it keeps: across l ^ 8 the lanes of banks 0-1 of
// each row keep slot 0 or 1 and those of banks 2-3 slot 2 or 3; across the
// half-row mirror (7 - i within each 8 lanes) banks 0 and 2 keep the first
// and banks 1 and 3 the second.  The compiler forms DPP adds only with every
// bank enabled and then routes the slots with selects.  The s_nops give the
// two wait states a DPP read needs after a VALU write of its source VGPR.
__device__ __forceinline__ float wave_steps34(float v0, float v1, float v2, float v3)
{
    float r0, r1, out;
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %1, %3, %3 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %1, %5, %5 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %2, %4, %4 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
        "v_add_f32_dpp %2, %6, %6 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
        "v_add_f32_dpp %0, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %2, %2 row_half_mirror row_mask:0xf bank_mask:0xa"
        : "=&v"(out), "=&v"(r0), "=&v"(r1)
        : "v"(v0), "v"(v1), "v"(v2), "v"(v3));
    return out;
}

template <bool N13>
__device__ __forceinline__ float wave_reduce16(float (&v)[16], int lane)
{
    (void)lane;
    pair_step1<N13>(v, [](float a, float b) { return swap_add32(a, b); });
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = swap_add16(v[k], v[k + 4]);
    v[0] = wave_steps34(v[0], v[1], v[2], v[3]);
    v[0] += dpp_move<kDppQuadXor2>(v[0]);
    v[0] += dpp_move<kDppQuadXor1>(v[0]);
    return v[0];
}

// 8x8 tiles, one pixel per lane (x = lane bits 0-2, y = lane bits 3-5): the
// 4x4 quarter of lane l is (l bit 2, l bit 5).  Sum v[0..15] over the 16
// lanes of each quarter at once.  Afterwards every lane holds one total of its
// quarter, of index quarter_index(l) (-1: none).
//   step 1: v_permlane16_swap pairs across lanes l, l ^ 16;
//   step 2: lanes l and l ^ 8 (DPP row rotate by 8) keep half of the slots
//           and send the other half;
//   steps 3, 4: the same within each quad, across l ^ 2 and then l ^ 1.
template <bool N13>
__device__ __forceinline__ int quarter_index(int lane)
{
    const int s = (lane & 3) | ((lane >> 1) & 4);
    return N13 ? n13_index(s, (lane >> 4) & 1) : s | ((lane >> 1) & 8);
}

// Slots k and k + D for k < n: lanes with hi keep slot k + D and send slot k,
// the others the reverse; slot k then holds the pair's sum across the lanes.
template <int CTRL, int D>
__device__ __forceinline__ void keep_send_add(float (&v)[16], int n, bool hi)
{
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < n) {
            const float send = hi ? v[k] : v[k + D];
            const float keep = hi ? v[k + D] : v[k];
            v[k] = keep + dpp_move<CTRL>(send);
        }
    }
}

// Step 2 for the pairs (v[k], v[k+4]), k < 3: lanes with bit 3 clear (banks
// 0-1 of each row) add slot k across l ^ 8, the others slot k + 4, each lane
// writing the sum of the slot it keeps with one bank-masked DPP add (the
// compiler forms DPP adds only with every bank enabled, and then needs two
// selects to route the slots).  The s_nop gives the two wait states a DPP read
// needs after a VALU write of its source VGPR.
#define VGR_PAIR_ADD8(D, A, C)                                                   \
    "v_add_f32_dpp " D ", " A ", " A " row_ror:8 row_mask:0xf bank_mask:0x3\n\t" \
    "v_add_f32_dpp " D ", " C ", " C " row_ror:8 row_mask:0xf bank_mask:0xc\n\t"

__device__ __forceinline__ void pair_add8x3(float (&v)[16])
{
    float r0, r1, r2;
    asm volatile("s_nop 1\n\t" VGR_PAIR_ADD8("%0", "%3", "%6") VGR_PAIR_ADD8("%1", "%4", "%7")
                     VGR_PAIR_ADD8("%2", "%5", "%8")
                 : "=&v"(r0), "=&v"(r1), "=&v"(r2)
                 : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[4]), "v"(v[5]), "v"(v[6]));
    v[0] = r0;
    v[1] = r1;
    v[2] = r2;
}

// The same for the four pairs k < 4.
__device__ __forceinline__ void pair_add8x4(float (&v)[16])
{
    float r0, r1, r2, r3;
    asm volatile("s_nop 1\n\t" VGR_PAIR_ADD8("%0", "%4", "%8") VGR_PAIR_ADD8("%1", "%5", "%9")
                     VGR_PAIR_ADD8("%2", "%6", "%10") VGR_PAIR_ADD8("%3", "%7", "%11")
                 : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
                 : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]),
                   "v"(v[6]), "v"(v[7]));
    v[0] = r0;
    v[1] = r1;
    v[2] = r2;
    v[3] = r3;
}
#undef VGR_PAIR_ADD8

template <bool N13>
__device__ __forceinline__ float quarter_reduce16(float (&v)[16], int lane)
{
    pair_step1<N13>(v, [](float a, float b) { return swap_add16(a, b); });
    if constexpr (N13) {
        // slot 7 is empty: slot 3 only needs its sum across l ^ 8
        pair_add8x3(v);
        v[3] += dpp_move<kDppRowRor8>(v[3]);
    } else {
        pair_add8x4(v);
    }
    keep_send_add<kDppQuadXor2, 2>(v, 2, lane & 2);
    // across l ^ 1 both slots are summed, then each lane takes its own: two
    // DPP adds (written out, so that the compiler neither sinks the adds into
    // the atomic's branch nor leaves the moves apart) and a select, instead of
    // two selects, a DPP move and an add.  The s_nop: two wait states before a
    // DPP read of a VGPR that a VALU instruction has just written.
    float s0, s1;
    asm volatile("s_nop 1\n\t"
                 "v_add_f32_dpp %0, %2, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
                 "v_add_f32_dpp %1, %3, %3 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
                 : "=&v"(s0), "=&v"(s1)
                 : "v"(v[0]), "v"(v[1]));
    return (lane & 1) ? s1 : s0;
}

// OR of a 64-bit lane mask over the lane's quarter (as in quarter_reduce16).
__device__ __forceinline__ uint64_t quarter_or(uint64_t m)
{
    uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    lo = a[0] | a[1];
    hi = c[0] | c[1];
    lo |= dpp_move_u<kDppRowRor8>(lo);
    hi |= dpp_move_u<kDppRowRor8>(hi);
    lo |= dpp_move_u<kDppQuadXor2>(lo);
    hi |= dpp_move_u<kDppQuadXor2>(hi);
    lo |= dpp_move_u<kDppQuadXor1>(lo);
    hi |= dpp_move_u<kDppQuadXor1>(hi);
    return ((uint64_t)hi << 32) | lo;
}

template <int TW, int TH, int MODE, bool COUNT, int B, bool WIN = false>
__global__ __launch_bounds__(64) void raster_bwd_kernel(RenderParams rp, Buffers b)
{
    static_assert(B == 32 || B == 64, "records per batch");
    constexpr int PPL = TileMap<TW, TH>::PPL;
    constexpr int RS = TileMap<TW, TH>::RS;
    constexpr bool COLOR = MODE != VGR_MODE_XRAY && MODE != kModeXrayNear && MODE != kModeXrayEpan;
    constexpr bool SPLAT = MODE == kModeSplat;   // colour with the 3DGS splatting alpha
    constexpr bool NEAR = MODE == kModeColorNear || MODE == kModeXrayNear;
    constexpr bool EPAN = MODE == kModeColorEpan || MODE == kModeXrayEpan;
    constexpr int NCH = COLOR ? 3 : 1;
    // the forward kept its pre-test masks for this shape and mode
    constexpr bool KEEP = COLOR || PPL == 1;
    // 8x8 tiles: each 4x4 quarter walks the records of its own pixels, so that
    // one step of the wave handles up to four records (quarter_reduce16).  Colour
    // modes with the volumetric opacity only: the splatting opacity's and the
    // X-ray backward's few operations per pair do not pay for the per-lane walk
    // (measured slower).
    constexpr bool QUAD = PPL == 1 && COLOR && !SPLAT;
    __shared__ Stage<B> st;

    const bool timed = b.wg_time != nullptr;   // uniform
    const uint64_t t_start = timed ? wg_clock() : 0;
    const int gt = (int)b.tile_order[blockIdx.x];
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

    // GB: dL/dC . (colour composited behind the current Gaussian); the replay
    // needs the colour behind only through this dot product
    float pyc[PPL], un[PPL], T[PPL], g[PPL][NCH], GB[PPL];
    int last[PPL];
    int maxlast = -1;
    Counts n;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int py = py0 + k * RS;
        pyc[k] = (float)py + 0.5f;
        const float uyn = (pyc[k] - vi.cy) / vi.fy;
        un[k] = sqrtf(ux * ux + uyn * uyn + 1.0f);
        const bool inside = px < W && py < H;
        const int64_t idx = (int64_t)py * W + px;
        last[k] = inside ? b.last_pos[vi.pix_off + idx] : -1;
        T[k] = inside ? b.T_final[vi.pix_off + idx] : 1.0f;
        float gbg = 0.0f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            g[k][c] = inside ? vi.dL[c * HW + idx] : 0.0f;
            gbg = __fmaf_rn(g[k][c], rp.bg[c], gbg);
        }
        GB[k] = T[k] * gbg;
        maxlast = max(maxlast, last[k]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) maxlast = max(maxlast, __shfl_xor(maxlast, off, 64));
    if (maxlast < (int)range.x) {   // uniform: no pixel of this tile blended anything
        if (timed && lane == 0)
            b.wg_time[rp.total_tiles + blockIdx.x] =
                make_uint2(cu_key(), (uint32_t)(wg_clock() - t_start));
        return;
    }
    const float tau2 = rp.tau2, ymax = rp.ymax;
    const float amin = rp.amin, amax = rp.amax;
    const float zn = vi.znear;
    float *rg = reinterpret_cast<float *>(b.rgrad);

    // One record of the batch (list position jpos) against the lane's pixels:
    // pass[k] marks the slots whose pixel the bound pre-test admits (dy is
    // recomputed here).
    auto record = [&](int qi, const PreRec &pr, float dx, const bool (&pass)[PPL], int jpos) {
        float acc[16];
        // -0 is the exact identity of addition, so the first term of each
        // sum needs no add
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = (e < 13 || NEAR) ? -0.0f : 0.0f;
        // lane masks (wave-uniform) of the slot's passing and blending
        // pixels; the branches test them directly
        uint64_t touched = 0;
        const FullRec fr = load_full(st, qi);
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const uint64_t pm = __builtin_amdgcn_ballot_w64(pass[k]);
            if (COUNT && !QUAD) n.visits_full += (lane == 0 && pm != 0) ? 1u : 0u;
            if (pm == 0) continue;                  // wave-uniform
            if (COUNT) n.full += pass[k] ? 1u : 0u;
            const float dy = (pyc[k] - pr.hy) - pr.ly;
            if constexpr (SPLAT) {
                // alpha = o exp2(-e); with tau = dL/dalpha alpha the record
                // gradient keeps sum tau (d d^T, d) and sum tau: dL/do =
                // sum tau / o, dL/dC = -1/2 sum tau d d^T, dL/dmu' = C sum tau d
                const float e = __fmaf_rn(dx, __fmaf_rn(fr.A01, dx, fr.A11 * dy),
                                          fr.A21 * (dy * dy));
                const float al = fr.K * fast_exp2(-e);
                const bool bl = pass[k] && !(al < amin);
                if (COUNT) n.blend += bl ? 1u : 0u;
                const uint64_t bm = __builtin_amdgcn_ballot_w64(!(al < amin)) & pm;
                if (bm == 0) continue;                      // wave-uniform
                const bool clamped = al > amax;
                const float a = clamped ? amax : al;
                const float om = 1.0f - a;
                const float inv = fast_rcp(om);
                const float Tb = T[k] * inv;
                const float gc = __fmaf_rn(g[k][0], fr.c0,
                                           __fmaf_rn(g[k][1], fr.c1, g[k][2] * fr.c2));
                const float da = __fmaf_rn(Tb, gc, -(inv * GB[k]));
                const float wgt = bl ? a * Tb : 0.0f;
                acc[10] = __fmaf_rn(g[k][0], wgt, acc[10]);
                acc[11] = __fmaf_rn(g[k][1], wgt, acc[11]);
                acc[12] = __fmaf_rn(g[k][2], wgt, acc[12]);
                GB[k] = __fmaf_rn(gc, wgt, GB[k]);
                T[k] = bl ? Tb : T[k];
                touched |= bm;
                const float tau = (bl && !clamped) ? da * al : 0.0f;
                const float tdx = tau * dx, tdy = tau * dy;
                acc[9] += tau;
                acc[3] += tdx;
                acc[4] += tdy;
                acc[0] += tdx * dx;
                acc[1] += tdx * dy;
                acc[2] += tdy * dy;
                continue;
            }
            PairGeom pg;
            pair_geom(pr, fr, dx, dy, pg);
            const float rq = fast_rsq(pg.qw);
            const float rq2 = rq * rq;
            const float ex = profile<EPAN>(fr.se, pg.num, rq2);
            float y = (NEAR ? fabsf(fr.K) : fr.K) * un[k] * rq * ex;
            // near-plane segment: y *= Phi(eta); hn = h (eta + 2 zn |w|) and
            // h = phi(eta) / Phi(eta) enter the moments below
            float hh = 0.0f, hn = 0.0f;
            if constexpr (NEAR) {
                if (fr.K < 0.0f) {
                    const float eta = near_eta(fr.v0x, fr.v0y, fr.v0z, fr.mz, pg.w0, pg.w1, pg.w2,
                                               pg.qw, rq, zn);
                    const float Phi = norm_cdf(eta);
                    y *= Phi;
                    // h stays finite on every lane (lanes whose pixel does not blend
                    // this record multiply it by t = 0): far out in the lower tail
                    // Phi underflows, and h tends to -eta there
                    hh = Phi > 1e-30f ? 0.39894228f * fast_exp2(-0.72134752f * eta * eta) / Phi
                                      : -eta;
                    hn = hh * __fmaf_rn(2.0f * zn, pg.qw * rq, eta);
                }
            }
            bool bl = pass[k] && !(y < tau2);
            if (COUNT) n.blend += bl ? 1u : 0u;
            const uint64_t bm = __builtin_amdgcn_ballot_w64(!(y < tau2)) & pm;
            if (bm == 0) continue;                      // wave-uniform
            float dy_;
            if constexpr (WIN) {
                // per-pixel window: the forward's masks name only composited
                // pairs, whose dL/dy and alpha T_before the replay left
                float2 wv = make_float2(0.0f, 0.0f);
                if (bl) wv = b.wpair[(size_t)jpos * 64 + lane];
                const float wgt = bl ? wv.y : 0.0f;
                acc[10] = __fmaf_rn(g[k][0], wgt, acc[10]);
                acc[11] = __fmaf_rn(g[k][1], wgt, acc[11]);
                acc[12] = __fmaf_rn(g[k][2], wgt, acc[12]);
                dy_ = bl ? wv.x : 0.0f;
            } else if constexpr (COLOR) {
                const bool clamped = y > ymax;
                const float om = fast_exp2(-(clamped ? ymax : y));
                const float inv = fast_rcp(om);
                const float alpha = 1.0f - om;
                const float Tb = T[k] * inv;
                // dL/dalpha = T_before (g.c) - (g.B) / (1 - alpha)
                const float gc = __fmaf_rn(g[k][0], fr.c0,
                                           __fmaf_rn(g[k][1], fr.c1, g[k][2] * fr.c2));
                const float da = __fmaf_rn(Tb, gc, -(inv * GB[k]));
                const float wgt = bl ? alpha * Tb : 0.0f;
                acc[10] = __fmaf_rn(g[k][0], wgt, acc[10]);
                acc[11] = __fmaf_rn(g[k][1], wgt, acc[11]);
                acc[12] = __fmaf_rn(g[k][2], wgt, acc[12]);
                GB[k] = __fmaf_rn(gc, wgt, GB[k]);
                T[k] = bl ? Tb : T[k];
                dy_ = (bl && !clamped) ? da * kLn2 * om : 0.0f;
            } else {
                dy_ = bl ? g[k][0] * kLn2 : 0.0f;
            }
            touched |= bm;
            // t = dL/d(ln x) = dL/dy * y (selected, not multiplied, to zero
            // for lanes that do not blend); since ln x is ln K' plus terms
            // free of K', the sum of t is K' dL/dK'
            const float t = bl ? dy_ * y : 0.0f;
            acc[9] += t;
            // z = mz (w x n) / |w|^2 = L (m - gamma u);  w' = w / |w|;
            // M += t (w' w'^T + z z^T) as (t w') w'^T + (t z) z^T (t is zero,
            // and z finite, on lanes that do not blend)
            const float cz = fr.mz * rq2;
            const float z0 = cz * (pg.w1 * pg.n2 - pg.w2 * pg.n1);
            const float z1 = cz * (pg.w2 * pg.n0 - pg.w0 * pg.n2);
            const float z2 = cz * (pg.w0 * pg.n1 - pg.w1 * pg.n0);
            const float p0 = pg.w0 * rq, p1 = pg.w1 * rq, p2 = pg.w2 * rq;
            // weight of the z terms: t, or t 3 / (1 - D^2) for the Epanechnikov
            // kernel (1 - D^2 > 0 wherever t is not zero)
            float tzw = t;
            if constexpr (EPAN)
                tzw = t != 0.0f ? t * (3.0f * fast_rcp(1.0f - fr.se * pg.num * rq2)) : 0.0f;
            const float tz0 = tzw * z0, tz1 = tzw * z1, tz2 = tzw * z2;
            float tw = t;   // weight of w' w'^T
            if constexpr (NEAR) {
                if (fr.K < 0.0f) {   // uniform over the lanes on this record
                    tw = __fmaf_rn(t, hn, t);
                    const float th = t * hh;
                    acc[13] += th * p0;
                    acc[14] += th * p1;
                    acc[15] += th * p2;
                }
            }
            const float tp0 = tw * p0, tp1 = tw * p1, tp2 = tw * p2;
            acc[6] += tz0;
            acc[7] += tz1;
            acc[8] += tz2;
            acc[0] += __fmaf_rn(tp0, p0, tz0 * z0);
            acc[1] += __fmaf_rn(tp0, p1, tz0 * z1);
            acc[2] += __fmaf_rn(tp0, p2, tz0 * z2);
            acc[3] += __fmaf_rn(tp1, p1, tz1 * z1);
            acc[4] += __fmaf_rn(tp1, p2, tz1 * z2);
            acc[5] += __fmaf_rn(tp2, p2, tz2 * z2);
        }
        if (touched != 0) {
            if constexpr (QUAD) {
                // lanes of the quarter that blended this step's record
                const uint64_t qm = ((lane & 4) ? 0xF0F0F0F0F0F0F0F0ull : 0x0F0F0F0F0F0F0F0Full) &
                                    ((lane & 32) ? ~0ull << 32 : ~0ull >> 32);
                const float tot = quarter_reduce16<!NEAR>(acc, lane);
                const int e = quarter_index<!NEAR>(lane);
                if ((touched & qm) != 0 && e >= 0)
                    atomicAdd(rg + (size_t)st.item[qi] * kGradFloats + e, tot);
            } else {
                const float tot = wave_reduce16<!NEAR>(acc, lane);
                const int e = wave_index<!NEAR>(lane);
                if ((lane & 3) == 0 && e >= 0)
                    atomicAdd(rg + (size_t)st.item[qi] * kGradFloats + e, tot);
            }
        }
    };

    if constexpr (KEEP) {
        // Batches aligned as in the forward, whose pre-test masks are reused:
        // the walk visits only records some pixel of the tile admits.
        for (int bs = (int)range.x + ((maxlast - (int)range.x) / B) * B; bs >= (int)range.x;
             bs -= B) {
            const int j = bs + lane;
            if (lane < B && j <= maxlast) stage_record(st, b, lane, b.inst_val[j]);
            uint64_t mask[PPL];
            uint64_t any = 0;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                // records of the batch up to the pixel's last blended one
                const int d = last[k] - bs;
                const uint64_t lim = d < 0 ? 0ull : (d >= 63 ? ~0ull : (2ull << d) - 1ull);
                mask[k] = b.pmask[mask_word<B>((uint32_t)bs, gt, lane) * PPL + k] & lim;
                any |= mask[k];
            }
            if constexpr (QUAD) {
                // the records some pixel of the lane's quarter admits, walked
                // from the back; a quarter with none left idles on record 0
                // (staged, so its arithmetic stays finite) with no pixel passing
                // (bit-reversed masks: the next record is the lowest set bit)
                uint64_t ur = __builtin_bitreverse64(quarter_or(any));
                const uint64_t mr = __builtin_bitreverse64(mask[0]);
                __syncthreads();
                bool act = ur != 0;
                if (wave_any(act)) do {
                    const int jr = act ? __builtin_ctzll(ur) : 63;
                    const int qi = 63 - jr;
                    ur &= ur - 1ull;
                    if (COUNT) {
                        n.visits += lane == 0 ? 1u : 0u;
                        n.visits_full += (act && (lane & 0x1B) == 0) ? 1u : 0u;
                    }
                    const RecRegs rr = load_regs(st, qi);
                    const PreRec pr = pre_of(rr);
                    const float dx = (pxc - pr.hx) - pr.lx;
                    bool pass[PPL];
                    pass[0] = act && ((mr >> jr) & 1u);
                    record(qi, pr, dx, pass, bs + qi);
                    act = ur != 0;
                } while (wave_any(act));
                __syncthreads();
                continue;
            }
            // union over the wave: OR within each row of 16 lanes, then of the rows
            uint32_t lo = (uint32_t)any, hi = (uint32_t)(any >> 32);
            lo |= dpp_move_u<kDppRowRor8>(lo);
            hi |= dpp_move_u<kDppRowRor8>(hi);
            lo |= dpp_move_u<kDppRowRor4>(lo);
            hi |= dpp_move_u<kDppRowRor4>(hi);
            lo |= dpp_move_u<kDppRowRor2>(lo);
            hi |= dpp_move_u<kDppRowRor2>(hi);
            lo |= dpp_move_u<kDppRowRor1>(lo);
            hi |= dpp_move_u<kDppRowRor1>(hi);
            const uint32_t ulo = __builtin_amdgcn_readlane(lo, 0) | __builtin_amdgcn_readlane(lo, 16) |
                                 __builtin_amdgcn_readlane(lo, 32) | __builtin_amdgcn_readlane(lo, 48);
            const uint32_t uhi = __builtin_amdgcn_readlane(hi, 0) | __builtin_amdgcn_readlane(hi, 16) |
                                 __builtin_amdgcn_readlane(hi, 32) | __builtin_amdgcn_readlane(hi, 48);
            uint64_t u = ((uint64_t)uhi << 32) | ulo;   // wave-uniform
            __syncthreads();
            while (u != 0) {
                const int qi = 63 - __builtin_clzll(u);
                u &= ~(1ull << qi);
                if (COUNT) n.visits += lane == 0 ? 1u : 0u;
                const RecRegs rr = load_regs(st, qi);
                const PreRec pr = pre_of(rr);
                const float dx = (pxc - pr.hx) - pr.lx;
                bool pass[PPL];
#pragma unroll
                for (int k = 0; k < PPL; ++k) pass[k] = (mask[k] >> qi) & 1u;
                record(qi, pr, dx, pass, bs + qi);
            }
            __syncthreads();
        }
    } else {
        for (int be = maxlast + 1; be > (int)range.x; be -= B) {
            const int bs = max((int)range.x, be - B);
            const int j = bs + lane;
            if (lane < B && j < be) stage_record(st, b, lane, b.inst_val[j]);
            __syncthreads();
            for (int qi = be - 1 - bs; qi >= 0; --qi) {
                const int jpos = bs + qi;
                const PreRec pr = load_pre(st, qi);
                const ColTerms ct = col_terms(pr, pxc);
                bool pass[PPL];
                bool anyp = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    float dy;
                    const bool inl = jpos <= last[k];
                    pass[k] = inl && pre_test(pr, ct, pyc[k], dy);
                    anyp |= pass[k];
                    if (COUNT) {
                        n.test += inl ? 1u : 0u;
                        const bool anyl = wave_any(inl);
                        n.visits += (lane == 0 && anyl) ? 1u : 0u;
                    }
                }
                if (!wave_any(anyp)) continue;             // wave-uniform
                record(qi, pr, ct.dx, pass, jpos);
            }
            __syncthreads();
        }
    }
    if (COUNT) {
        atomicAdd(&b.counters[8], (unsigned long long)n.test);
        atomicAdd(&b.counters[9], (unsigned long long)n.full);
        atomicAdd(&b.counters[10], (unsigned long long)n.blend);
        atomicAdd(&b.counters[11], (unsigned long long)n.visits);
        atomicAdd(&b.counters[12], (unsigned long long)n.visits_full);
    }
    if (timed && lane == 0)
        b.wg_time[rp.total_tiles + blockIdx.x] =
            make_uint2(cu_key(), (uint32_t)(wg_clock() - t_start));
}

// ---------------------------------------------------------------------------
// Per-pixel re-sorting window (rp.pixel_window = W > 0, on top of the
// per-tile order; 8x8 tiles, one pixel per lane, 64-record batches).
//
// Forward: each lane walks its pixel's passing pairs in list order as the
// colour forward does.  A pair that reaches alpha_min meets a window of W - 1
// slots: whichever of the pair and the slots has the smallest key (the view
// depth of the Gaussian's maximum on the pixel's own ray, mz (v0 . w) / |w|^2;
// ties by list position) is composited, and the pair takes the freed slot.
// Empty slots count as smaller than every key, so the first W - 1 pairs only
// fill the window; at the end of the list it drains in key order.  Each
// composited pair is appended to the pixel's compositing sequence (wseq:
// 1 - alpha and list position, entry k of the tile's lanes side by side), and
// its bit is set in the mask word of its batch (where the colour forward
// keeps its pre-test masks).
//
// Backward: raster_bwd_window_replay_kernel walks each pixel's sequence from
// its end with the colour backward's replay arithmetic and writes every
// composited pair's dL/dy and alpha T_before at its list position; the
// rasteriser backward (WIN) then visits the composited pairs the masks name
// and reads those values instead of replaying in list order.
// One lane's window: keys and list positions in registers (the argmin runs
// over them), each slot's payload (1 - alpha, negated if clamped; colour) in
// LDS at pay[slot][lane], read and written at the slot index.
template <int WS>
struct Window {
    float k[WS];          // key (-inf: empty, taken first; +inf: unused)
    int p[WS];            // list position (-1: empty)
    float mink;           // smallest (key, position) ...
    int mins, minp;       // ... its slot and position
    float4 (*pay)[64];
    int lane;

    __device__ __forceinline__ void rescan()
    {
        mink = k[0];
        mins = 0;
        minp = p[0];
#pragma unroll
        for (int s = 1; s < WS; ++s) {
            const bool lt = k[s] < mink || (k[s] == mink && p[s] < minp);
            mink = lt ? k[s] : mink;
            mins = lt ? s : mins;
            minp = lt ? p[s] : minp;
        }
    }
    // the payload of the smallest slot (meaningless where that slot is empty)
    __device__ __forceinline__ float4 take() const { return pay[mins][lane]; }
    __device__ __forceinline__ void put(bool on, float key, int pos, const float4 &v)
    {
        if (on) pay[mins][lane] = v;
#pragma unroll
        for (int s = 0; s < WS; ++s) {
            const bool w = on && s == mins;
            k[s] = w ? key : k[s];
            p[s] = w ? pos : p[s];
        }
    }
};

template <int MODE, int WS>
__global__ __launch_bounds__(64) void raster_fwd_window_kernel(RenderParams rp, Buffers b)
{
    constexpr int B = 64;
    constexpr bool NEAR = MODE == kModeColorNear;
    constexpr bool EPAN = MODE == kModeColorEpan;
    __shared__ Stage<B> st;
    __shared__ float4 wpay[WS][64];

    const bool timed = b.wg_time != nullptr;   // uniform
    const uint64_t t_start = timed ? wg_clock() : 0;
    const int gt = (int)b.tile_order[blockIdx.x];
    const int v = find_view(b.views, rp.n_views, gt);
    const ViewInfo &vi = b.views[v];
    const int lt = gt - vi.tile_off;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * 8 + (lane & 7), py = ty * 8 + (lane >> 3);
    const int W = vi.width, H = vi.height;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    const float ux = (pxc - vi.cx) / vi.fx;
    const float uyn = (pyc - vi.cy) / vi.fy;
    const float un = sqrtf(ux * ux + uyn * uyn + 1.0f);
    bool act = px < W && py < H;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int nseq = 0, lastp = -1, visited = -1;
    const uint2 range = b.ranges[gt];
    const float tau2 = rp.tau2, ymax = rp.ymax, Tmin = rp.T_min;
    const float zn = vi.znear;
    const int nslot = rp.pixel_window - 1;
    Window<WS> win;
    win.pay = wpay;
    win.lane = lane;
#pragma unroll
    for (int s = 0; s < WS; ++s) {
        win.k[s] = s < nslot ? -INFINITY : INFINITY;   // empty: taken first; unused: never
        win.p[s] = -1;
        // a slot never filled is still read (and multiplied by a zero weight)
        wpay[s][lane] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
    }
    win.rescan();
    // Composite one pair (oms: 1 - alpha, negated where alpha was clamped) if
    // `on`, or stop the pixel where T (1 - alpha) < T_min (Sec. 4.1).
    // composited pairs of the current batch (bit q: list position cur + q);
    // pairs of earlier batches are marked in their batch's word, which this
    // lane alone owns and has written at the end of that batch
    uint64_t cm = 0;
    uint32_t cur = range.x;
    auto composite = [&](bool on, float oms, float c0, float c1, float c2, int pos) {
        const float om = fabsf(oms);
        const float Tn = T * om;
        const bool stop = on && Tn < Tmin;
        const bool dob = on && !stop;
        const float wgt = dob ? (1.0f - om) * T : 0.0f;
        C0 = __fmaf_rn(c0, wgt, C0);
        C1 = __fmaf_rn(c1, wgt, C1);
        C2 = __fmaf_rn(c2, wgt, C2);
        if (dob) {
            b.wseq[window_seq(range.x, nseq, lane)] = make_int2(__float_as_int(oms), pos);
            if ((uint32_t)pos >= cur) {
                cm |= 1ull << ((uint32_t)pos - cur);
            } else {
                const uint32_t ob = range.x + (((uint32_t)pos - range.x) / B) * B;
                uint64_t &wd = b.pmask[mask_word<B>(ob, gt, lane)];
                wd |= 1ull << ((uint32_t)pos - ob);
            }
        }
        T = dob ? Tn : T;
        lastp = dob ? pos : lastp;
        nseq += dob ? 1 : 0;
        act = act && !stop;
    };

    for (uint32_t bs = range.x; bs < range.y; bs += B) {
        const uint32_t j = bs + lane;
        if (j < range.y) stage_record(st, b, lane, b.inst_val[j]);
        __syncthreads();
        const int nb = (int)min((uint32_t)B, range.y - bs);
        // bound pre-test of the batch (broadcast records), kept for the backward
        uint32_t mh[2] = { 0u, 0u };
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int qend = min(nb, 32 * h + 32);
            for (int qi = 32 * h; qi < qend; ++qi) {
                const PreRec pr = load_pre(st, qi);
                const ColTerms ct = col_terms(pr, pxc);
                float dy;
                const bool pass = act && pre_test(pr, ct, pyc, dy);
                mh[h] |= pass ? 1u << (qi & 31) : 0u;
            }
        }
        uint64_t mk = ((uint64_t)mh[1] << 32) | mh[0];
        cur = bs;
        cm = 0;
        while (wave_any(mk != 0 && act)) {                 // wave-uniform loop
            const bool has = mk != 0 && act;
            const int qi = has ? (int)__builtin_ctzll(mk) : 0;
            mk &= mk - 1;
            const RecRegs rr = load_regs(st, qi);
            const PreRec pr = pre_of(rr);
            const FullRec fr = full_of(rr);
            const float dx = (pxc - pr.hx) - pr.lx;
            const float dy = (pyc - pr.hy) - pr.ly;
            PairGeom g;
            pair_geom(pr, fr, dx, dy, g);
            const float rq = fast_rsq(g.qw);
            const float ex = profile<EPAN>(fr.se, g.num, rq * rq);
            float y = (NEAR ? fabsf(fr.K) : fr.K) * un * rq * ex;
            if constexpr (NEAR) {
                if (fr.K < 0.0f)
                    y *= norm_cdf(near_eta(fr.v0x, fr.v0y, fr.v0z, fr.mz, g.w0, g.w1, g.w2, g.qw, rq,
                                           zn));
            }
            const bool cand = has && !(y < tau2);
            const float om = fast_exp2(-(y > ymax ? ymax : y));
            const float oms = y > ymax ? -om : om;
            const float vw = __fmaf_rn(fr.v0x, g.w0, __fmaf_rn(fr.v0y, g.w1, fr.v0z * g.w2));
            const float key = fr.mz * vw * (rq * rq);
            const int pos = (int)bs + qi;
            visited = has ? pos : visited;
            // the pair goes first if it precedes every entry; otherwise the
            // smallest entry leaves (none while its slot is empty) and the
            // pair takes the slot
            const bool direct = cand && key < win.mink;
            const bool swap = cand && !direct;
            const float4 w = win.take();
            const int sp = win.minp;
            composite(direct || (swap && sp >= 0), direct ? oms : w.x, direct ? fr.c0 : w.y,
                      direct ? fr.c1 : w.z, direct ? fr.c2 : w.w, direct ? pos : sp);
            win.put(swap, key, pos, make_float4(oms, fr.c0, fr.c1, fr.c2));
            win.rescan();
        }
        // the batch's composited pairs, for the backward (every later mark
        // of this batch is a read-modify-write of this word)
        b.pmask[mask_word<B>(bs, gt, lane)] = cm;
        cur = range.y;
        __syncthreads();
        if (!wave_any(act)) break;                          // every pixel has stopped
    }
    // end of the list: the window drains in key order (slots never filled
    // take no part)
#pragma unroll
    for (int s = 0; s < WS; ++s) win.k[s] = win.k[s] == -INFINITY ? INFINITY : win.k[s];
    win.rescan();
    while (wave_any(act && win.mink < INFINITY)) {
        const bool on = act && win.mink < INFINITY;
        const float4 w = win.take();
        composite(on, w.x, w.y, w.z, w.w, win.minp);
#pragma unroll
        for (int s = 0; s < WS; ++s) win.k[s] = (on && s == win.mins) ? INFINITY : win.k[s];
        win.rescan();
    }

    if (px < W && py < H) {
        const int64_t HW = (int64_t)W * H;
        const int64_t idx = (int64_t)py * W + px;
        const int64_t pidx = vi.pix_off + idx;
        vi.out[idx] = __fmaf_rn(T, rp.bg[0], C0);
        vi.out[HW + idx] = __fmaf_rn(T, rp.bg[1], C1);
        vi.out[2 * HW + idx] = __fmaf_rn(T, rp.bg[2], C2);
        b.T_final[pidx] = T;
        b.last_pos[pidx] = visited;
        b.wcount[pidx] = nseq;
        b.last_id[pidx] = lastp >= 0 ? (int32_t)((int64_t)b.inst_val[lastp] - (int64_t)v * rp.n) : -1;
    }
    if (timed && lane == 0)
        b.wg_time[blockIdx.x] = make_uint2(cu_key(), (uint32_t)(wg_clock() - t_start));
}

// Reverse replay of each pixel's compositing sequence (per-pixel window):
// T before a pair is T after it over its 1 - alpha, and GB = dL/dC . (colour
// behind it) accumulates from T_final bg, as in the colour backward, with the
// colour read from the pair's record; writes (dL/dy, alpha T_before) at the
// pair's list position.
__global__ __launch_bounds__(64) void raster_bwd_window_replay_kernel(RenderParams rp, Buffers b)
{
    const int gt = (int)b.tile_order[blockIdx.x];
    const int v = find_view(b.views, rp.n_views, gt);
    const ViewInfo &vi = b.views[v];
    const int lt = gt - vi.tile_off;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x;
    const int px = tx * 8 + (lane & 7), py = ty * 8 + (lane >> 3);
    if (px >= vi.width || py >= vi.height) return;
    const int64_t HW = (int64_t)vi.width * vi.height;
    const int64_t idx = (int64_t)py * vi.width + px;
    const int64_t pidx = vi.pix_off + idx;
    const int n = b.wcount[pidx];
    float T = b.T_final[pidx];
    float g[3], gbg = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        g[c] = vi.dL[c * HW + idx];
        gbg = __fmaf_rn(g[c], rp.bg[c], gbg);
    }
    float GB = T * gbg;
    const uint2 range = b.ranges[gt];
    // eight steps at a time: their sequence entries, then their records'
    // item ids, then their colours are loaded together (three round trips
    // per eight steps instead of one per load), then the eight steps run in
    // order
    constexpr int U = 8;
    for (int k = n - 1; k >= 0; k -= U) {
        int2 e[U];
        uint32_t item[U];
        float4 cc[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            e[u] = k - u >= 0 ? b.wseq[window_seq(range.x, k - u, lane)] : make_int2(0, 0);
#pragma unroll
        for (int u = 0; u < U; ++u) item[u] = k - u >= 0 ? b.inst_val[e[u].y] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u)
            cc[u] = k - u >= 0 ? b.geom[(size_t)item[u] * kRecVec + 5] : make_float4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k - u < 0) break;
            const float oms = __int_as_float(e[u].x);
            const int pos = e[u].y;
            const float om = fabsf(oms);
            const float inv = fast_rcp(om);
            const float alpha = 1.0f - om;
            const float Tb = T * inv;
            // dL/dalpha = T_before (g.c) - (g.B) / (1 - alpha)
            const float gc = __fmaf_rn(g[0], cc[u].x, __fmaf_rn(g[1], cc[u].y, g[2] * cc[u].z));
            const float da = __fmaf_rn(Tb, gc, -(inv * GB));
            const float wgt = alpha * Tb;
            GB = __fmaf_rn(gc, wgt, GB);
            T = Tb;
            b.wpair[(size_t)pos * 64 + lane] =
                make_float2(oms < 0.0f ? 0.0f : da * kLn2 * om, wgt);
        }
    }
}

template <int MODE>
hipError_t window_fwd_mode(const RenderParams &rp, const Buffers &b, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    const int ns = rp.pixel_window - 1;
    if (ns <= 1) raster_fwd_window_kernel<MODE, 1><<<grid, block, 0, s>>>(rp, b);
    else if (ns <= 3) raster_fwd_window_kernel<MODE, 3><<<grid, block, 0, s>>>(rp, b);
    else if (ns <= 7) raster_fwd_window_kernel<MODE, 7><<<grid, block, 0, s>>>(rp, b);
    else if (ns <= 15) raster_fwd_window_kernel<MODE, 15><<<grid, block, 0, s>>>(rp, b);
    else raster_fwd_window_kernel<MODE, 31><<<grid, block, 0, s>>>(rp, b);
    return hipGetLastError();
}

hipError_t window_fwd(const RenderParams &rp, const Buffers &b, hipStream_t s)
{
    if (rp.kernel == VGR_KERNEL_EPANECHNIKOV) return window_fwd_mode<kModeColorEpan>(rp, b, s);
    if (rp.near_segment) return window_fwd_mode<kModeColorNear>(rp, b, s);
    return window_fwd_mode<VGR_MODE_COLOR>(rp, b, s);
}

hipError_t window_bwd(const RenderParams &rp, const Buffers &b, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    raster_bwd_window_replay_kernel<<<grid, block, 0, s>>>(rp, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (rp.kernel == VGR_KERNEL_EPANECHNIKOV)
        raster_bwd_kernel<8, 8, kModeColorEpan, false, 64, true><<<grid, block, 0, s>>>(rp, b);
    else if (rp.near_segment)
        raster_bwd_kernel<8, 8, kModeColorNear, false, 64, true><<<grid, block, 0, s>>>(rp, b);
    else
        raster_bwd_kernel<8, 8, VGR_MODE_COLOR, false, 64, true><<<grid, block, 0, s>>>(rp, b);
    return hipGetLastError();
}

template <int TW, int TH, int B>
hipError_t fwd_shape(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    if (rp.alpha_model == VGR_ALPHA_SPLAT) {
        if (count) raster_fwd_kernel<TW, TH, kModeSplat, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_fwd_kernel<TW, TH, kModeSplat, false, B><<<grid, block, 0, s>>>(rp, b);
    } else if (rp.kernel == VGR_KERNEL_EPANECHNIKOV) {
        if (rp.mode == VGR_MODE_COLOR) {
            if (count) raster_fwd_kernel<TW, TH, kModeColorEpan, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_fwd_kernel<TW, TH, kModeColorEpan, false, B><<<grid, block, 0, s>>>(rp, b);
        } else {
            if (count) raster_fwd_kernel<TW, TH, kModeXrayEpan, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_fwd_kernel<TW, TH, kModeXrayEpan, false, B><<<grid, block, 0, s>>>(rp, b);
        }
    } else if (rp.near_segment) {
        if (rp.mode == VGR_MODE_COLOR) {
            if (count) raster_fwd_kernel<TW, TH, kModeColorNear, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_fwd_kernel<TW, TH, kModeColorNear, false, B><<<grid, block, 0, s>>>(rp, b);
        } else {
            if (count) raster_fwd_kernel<TW, TH, kModeXrayNear, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_fwd_kernel<TW, TH, kModeXrayNear, false, B><<<grid, block, 0, s>>>(rp, b);
        }
    } else if (rp.mode == VGR_MODE_COLOR) {
        if (count) raster_fwd_kernel<TW, TH, VGR_MODE_COLOR, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_fwd_kernel<TW, TH, VGR_MODE_COLOR, false, B><<<grid, block, 0, s>>>(rp, b);
    } else {
        if (count) raster_fwd_kernel<TW, TH, VGR_MODE_XRAY, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_fwd_kernel<TW, TH, VGR_MODE_XRAY, false, B><<<grid, block, 0, s>>>(rp, b);
    }
    return hipGetLastError();
}

template <int TW, int TH, int B>
hipError_t bwd_shape(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    const dim3 grid(rp.total_tiles), block(64);
    if (rp.alpha_model == VGR_ALPHA_SPLAT) {
        if (count) raster_bwd_kernel<TW, TH, kModeSplat, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_bwd_kernel<TW, TH, kModeSplat, false, B><<<grid, block, 0, s>>>(rp, b);
    } else if (rp.kernel == VGR_KERNEL_EPANECHNIKOV) {
        if (rp.mode == VGR_MODE_COLOR) {
            if (count) raster_bwd_kernel<TW, TH, kModeColorEpan, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_bwd_kernel<TW, TH, kModeColorEpan, false, B><<<grid, block, 0, s>>>(rp, b);
        } else {
            if (count) raster_bwd_kernel<TW, TH, kModeXrayEpan, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_bwd_kernel<TW, TH, kModeXrayEpan, false, B><<<grid, block, 0, s>>>(rp, b);
        }
    } else if (rp.near_segment) {
        if (rp.mode == VGR_MODE_COLOR) {
            if (count) raster_bwd_kernel<TW, TH, kModeColorNear, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_bwd_kernel<TW, TH, kModeColorNear, false, B><<<grid, block, 0, s>>>(rp, b);
        } else {
            if (count) raster_bwd_kernel<TW, TH, kModeXrayNear, true, B><<<grid, block, 0, s>>>(rp, b);
            else raster_bwd_kernel<TW, TH, kModeXrayNear, false, B><<<grid, block, 0, s>>>(rp, b);
        }
    } else if (rp.mode == VGR_MODE_COLOR) {
        if (count) raster_bwd_kernel<TW, TH, VGR_MODE_COLOR, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_bwd_kernel<TW, TH, VGR_MODE_COLOR, false, B><<<grid, block, 0, s>>>(rp, b);
    } else {
        if (count) raster_bwd_kernel<TW, TH, VGR_MODE_XRAY, true, B><<<grid, block, 0, s>>>(rp, b);
        else raster_bwd_kernel<TW, TH, VGR_MODE_XRAY, false, B><<<grid, block, 0, s>>>(rp, b);
    }
    return hipGetLastError();
}

}  // namespace

namespace {

template <int B>
hipError_t fwd_batch(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.tile_w == 8 && rp.tile_h == 8) return fwd_shape<8, 8, B>(rp, b, count, s);
    if (rp.tile_w == 16 && rp.tile_h == 8) return fwd_shape<16, 8, B>(rp, b, count, s);
    if (rp.tile_w == 32 && rp.tile_h == 8) return fwd_shape<32, 8, B>(rp, b, count, s);
    return fwd_shape<16, 16, B>(rp, b, count, s);
}

template <int B>
hipError_t bwd_batch(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.tile_w == 8 && rp.tile_h == 8) return bwd_shape<8, 8, B>(rp, b, count, s);
    if (rp.tile_w == 16 && rp.tile_h == 8) return bwd_shape<16, 8, B>(rp, b, count, s);
    if (rp.tile_w == 32 && rp.tile_h == 8) return bwd_shape<32, 8, B>(rp, b, count, s);
    return bwd_shape<16, 16, B>(rp, b, count, s);
}

}  // namespace

hipError_t launch_raster_fwd(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.total_tiles <= 0) return hipSuccess;
    if (rp.pixel_window > 0) return window_fwd(rp, b, s);
    return rp.batch == 32 ? fwd_batch<32>(rp, b, count, s) : fwd_batch<64>(rp, b, count, s);
}

hipError_t launch_raster_bwd(const RenderParams &rp, const Buffers &b, bool count, hipStream_t s)
{
    if (rp.total_tiles <= 0) return hipSuccess;
    if (rp.pixel_window > 0) return window_bwd(rp, b, s);
    return rp.batch == 32 ? bwd_batch<32>(rp, b, count, s) : bwd_batch<64>(rp, b, count, s);
}

}  // namespace vgr
