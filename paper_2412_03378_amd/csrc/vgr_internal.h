// Internal declarations shared by the HIP translation units of libvgr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vgr.h"

namespace vgr {

// log2(e), ln(2), sqrt(2 pi) and sqrt(log2(e)/2), the scale folded into the
// record so that the rasteriser's exponent is exp2(-(log2 e / 2) D^2).
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kSqrt2Pi = 2.5066282746310002f;
constexpr float kHalfLog2eSqrt = 0.8493218002880191f;

constexpr int kMaxViews = 64;
constexpr int kRecVec = 8;        // float4 per rasteriser record (128 bytes), see layout below
constexpr float kConicMargin = 0.05f;
constexpr float kCullLevel = 0.1f;   // tile culling level of the bound form (> kConicMargin)
constexpr float kCullPad = 0.02f;    // pixels added on both ends of a culled row span
constexpr int kGradFloats = 16;   // record gradient per (Gaussian, view)
// rasteriser template modes beyond VGR_MODE_COLOR / VGR_MODE_XRAY: colour with
// the splatting alpha; colour and X-ray with the near-plane segment; colour
// and X-ray with the Epanechnikov kernel
constexpr int kModeSplat = 2, kModeColorNear = 3, kModeXrayNear = 4;
constexpr int kModeColorEpan = 5, kModeXrayEpan = 6;

// Rasteriser record of one (Gaussian, view), 128 bytes (8 float4, one cache
// line), in the Gaussian's view space with L = diag(1/s) Rc^T (Rc = R_view
// R(q)), so that Sigma_v^-1 = L^T L, and m the view-space mean (computed in
// FP64).  The fields of the bound pre-test come first, so that a rasteriser
// step that rejects every pixel reads three float4:
//   g0 = (hx, hy, lx, ly)       projected mean (fx mx/mz + cx, fy my/mz + cy) in
//                               pixels, split into an integer hi part h and an
//                               FP32 residual l (|l| <= 0.5), so that the pixel
//                               offset (p + 0.5 - h) - l keeps full precision
//   g1 = (Q00, 2 Q01, 2 l0, 2 l1)
//   g2 = (Q11, A00, A10, A20)   A = L[:, 0:2] diag(1/fx, 1/fy)
//   g3 = (A01, A11, A21, v0x)   v0 = L m / mz: L applied to the ray through the mean
//   g4 = (v0y, v0z, K', se)     K' = kappa sqrt(2 pi) log2 e,  se = (log2 e / 2) mz^2;
//                               K' < 0 (|K'| the value) flags a record that needs
//                               the near-plane segment factor.  Epanechnikov
//                               kernel: K' = (4/3) kappa log2 e, se = mz^2
//   g5 = (r, g, b, mz)          colour after the activation (0 in X-ray mode)
//   g6 = (cx, cy, a, P)         tile-culling ellipse (see cull_row in the
//   g7 = (R, ymax, yl, on)        preprocess source); on = 0: no culling
// With the splatting model (VGR_ALPHA_SPLAT) g0, g1, g5, g6, g7 keep their
// meaning (l = 0) and g2 = (Q11, 0, 0, 0), g3 = (c00, c01, c11, 0),
// g4 = (0, 0, o, 0) with c = log2(e) (C00/2, C01, C11/2), C = Sigma'^-1:
// alpha = o exp2(-(c00 dx^2 + c01 dx dy + c11 dy^2)).  Its record gradient,
// with tau = dL/dalpha alpha summed over the pixels that blend it: [0..2]
// sum tau (dx^2, dx dy, dy^2), [3..4] sum tau (dx, dy), [9] sum tau,
// [10..12] dL/dc.
// For the pixel with centre (px + 0.5, py + 0.5), ray u = (ux, uy, 1), and
// pixel offset d = (px + 0.5, py + 0.5) - h - l:
//   a = A d,  w = L u = v0 + a,  L m x L u = mz (v0 x a)
//   D^2 = mz^2 |v0 x a|^2 / |w|^2   (minimum Mahalanobis distance of the ray;
//                                    free of cancellation near the centre)
//   beta = |u| / |w|,  log2(e) x = K' |u| exp2(-(log2 e / 2) D^2) / |w|
//   (Epanechnikov: log2(e) x = K' |u| (1 - D^2)^(3/2) / |w| for D^2 < 1, else 0).
// Bound pre-test: f(d) = d^T Q d + 2 l^T d - 1 has the sign of D^2 - D2max
// (it is |w|^2 (D^2 - D2max) / (D2max |v0|^2)), so f > 0.05 proves
// alpha < alpha_min for that pixel at a cost of three FP32 operations.  The
// margin covers the FP32 evaluation error when the 2x2 form Q is positive
// definite with condition number <= 1e4; otherwise Q = l = 0 (f = -1, no
// pixel is rejected early).
//
// Record gradient, 16 floats, as moments in the Gaussian's L-frame.  Per pixel,
// with t = dL/d(ln x), v = m - gamma u (mean minus closest ray point) and
// z = L v = mz (w x n) / |w|^2 (no cancellation), Sec. 4.2 gives
//   d ln x / dm = -Sigma^-1 v = -L^T z,
//   d ln x / dSigma^-1 = -1/2 (u u^T / u^T Sigma^-1 u + v v^T)
//                      = -1/2 L^-1 (w w^T / |w|^2 + z z^T) L^-T,
// so the sums  M = sum t (w w^T/|w|^2 + z z^T)  (symmetric) and  Z = sum t z
// carry the whole geometric gradient (Epanechnikov kernel: ln x has
// (3/2) ln(1 - D^2) in place of -D^2/2, so the z terms carry t 3/(1 - D^2)
// in place of t):
//   [0..5] M00 M01 M02 M11 M12 M22, [6..8] Z, [9] sum t (= K' dL/dK'), [10..12] dL/dc,
//   [13..15] U = sum t h w/|w| (near-plane segment, else 0).
// With the segment factor Phi(eta), eta = (gamma - t_n)/beta = mz (v0.w')
// - zn |w| (w' = w/|w|) and h = phi(eta)/Phi(eta), the w' w'^T weight in M
// becomes t (1 + h (eta + 2 zn |w|)), and the preprocess backward subtracts
// (Lm) U^T + U (Lm)^T from M and adds L^T U to dL/dm.

struct ViewInfo {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float znear;
    float o[3];          // world camera centre -R^-1 t (for the SH direction)
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tile_off;    // first global tile id of this view
    int32_t pad0;
    int64_t pix_off;     // offset of this view in per-pixel workspace arrays
    float *out;          // caller image
    const float *dL;     // caller upstream gradient (backward)
};

struct RenderParams {
    int32_t mode;
    int32_t sh_degree;
    int32_t act;
    int32_t n_views;
    int64_t n;           // Gaussians
    float tau;           // skip threshold on x (colour: -ln(1-alpha_min); xray: x_min)
    float tau2;          // tau * log2(e)
    float ymax;          // -log2(1 - alpha_max)
    float T_min;
    float bg[3];
    int32_t tile_w, tile_h;
    int32_t total_tiles;
    int32_t density;     // VGR_DENSITY_KAPPA or VGR_DENSITY_THETA
    int32_t alpha_model; // VGR_ALPHA_VOLUMETRIC or VGR_ALPHA_SPLAT
    float amin, amax;    // alpha_min, alpha_max (splatting model)
    int32_t near_segment;// integrate from the near plane (records flagged by K' < 0)
    int32_t tile_resort; // per-tile order by the depth of the maximum on the tile-centre ray
    int32_t kernel;      // VGR_KERNEL_GAUSSIAN or VGR_KERNEL_EPANECHNIKOV
    int32_t batch;       // records staged per rasteriser batch: 32 or 64
    int32_t pixel_window;// per-pixel re-sorting window W (0: off; 8x8 tiles, batch 64)
};

// Device workspace views handed to kernels.
struct Buffers {
    float4 *geom;        // n_views * n records (kRecVec float4 each)
    uint32_t *depth_key; // n_views * n
    uint32_t *item_ids;  // n_views * n (item = view * n + Gaussian; the items with
                         // instances, sorted by depth)
    uint32_t *key2;      // n_views * n: depth keys in item order, then sort ping-pong
    uint32_t *item2;     // n_views * n, sort ping-pong
    uint32_t *counts;    // n_views * n, tiles per item (item order)
    uint32_t *cnt_sorted;// n_views * n, tiles per item in depth order
    uint32_t *offsets;   // n_views * n + 1, exclusive scan of cnt_sorted
    ushort4 *rect;       // n_views * n, tile rectangle [x0, y0, x1, y1]
    uint32_t *inst_key;  // capacity: global tile id
    uint32_t *inst_val;  // capacity: item
    uint32_t *inst_key2; // capacity, sort ping-pong
    uint32_t *inst_val2; // capacity, sort ping-pong
    uint2 *ranges;       // total tiles
    uint32_t *tile_key;  // total tiles: cost key, then sorted
    uint32_t *tile_order;// total tiles: tiles by decreasing list length
    uint32_t *tile_key2; // total tiles, sort ping-pong
    uint32_t *tile_order2;
    float *T_final;      // total pixels
    int32_t *last_pos;   // total pixels: list position of last blended (-1); with the
                         // per-pixel window, of the last pair the pixel visited
    int32_t *last_id;    // total pixels: Gaussian index of last blended (-1)
    float4 *rgrad;       // n_views * n * 4 float4 (record gradients)
    uint64_t *pmask;     // pmask_words(): bound pre-test lane masks of each B-record
                         // batch of a tile list, written by the forward where
                         // raster_keeps_masks() and read by the backward (with
                         // the per-pixel window: the pairs composited)
    // per-pixel window (pixel_window > 0), capacity * 64 slots each:
    int2 *wseq;          // the k-th composited pair of tile lane l (tile list
                         // starting at s) at window_seq(s, k, l) = (s + k) 64 + l:
                         // (bits of 1 - alpha, negated where alpha was clamped;
                         // list position)
    float2 *wpair;       // at (list position) * 64 + lane, written by the backward
                         // replay for composited pairs: (dL/dy, 0 where alpha was
                         // clamped; alpha T_before)
    int32_t *wcount;     // total pixels: pairs composited
    uint32_t *blk_counts;// preprocess blocks: instances per block
    uint32_t *d_total;   // [0] = instance count K, [1] overflow flag, [4] K from the
                         // preprocess, [6] items with instances (the first of the
                         // depth order)
    uint32_t *h_total;   // or null: pinned host words (device address) that the totals
                         // kernel fills with d_total[4] at [0] and d_total[6] at [2]
    unsigned long long *counters;  // pair and visit counters: forward [0..4], backward [8..12]
    uint2 *wg_time;      // timed runs (else null): per rasteriser workgroup (launch slot) the
                         // compute unit key and its duration in clock ticks, forward
                         // at [0, total tiles), backward at [total tiles, 2 total tiles)
    const ViewInfo *views;
};

// The forward keeps, for each B-record batch of a tile's list, every lane's
// bound pre-test mask per pixel slot (bit q: record q of the batch may reach
// the pixel), where it computes them for the whole batch: colour mode, and
// X-ray mode with one pixel per lane.  Batch k of tile t (records
// start_t + B k ...) keeps its masks at words
// (((start_t + B k) 64/B + 64 t + lane) * ppl + slot): tile t's batches span
// fewer than len_t 64/B + 64 slots, so the tiles' spans do not overlap.
inline bool raster_keeps_masks(int mode, int tile_w, int tile_h)
{
    return mode == VGR_MODE_COLOR || tile_w * tile_h == 64;
}
inline int64_t pmask_words(int64_t instances, int32_t total_tiles, int tile_w, int tile_h,
                           int batch)
{
    return (instances * (64 / batch) + 64 * (int64_t)total_tiles) * (int64_t)(tile_w * tile_h / 64);
}

// ---- launches (each returns hipSuccess or the first error) ----
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);

hipError_t launch_preprocess(const RenderParams &rp, const Buffers &b, const float *means,
                             const float *quats, const float *scales, const float *dens,
                             const float *sh, hipStream_t s);
// Size of Buffers::blk_counts: the instance partial sums per preprocess block,
// then the counts of items with instances per (view, block).
int64_t preprocess_blocks(int64_t n, int32_t n_views);
// The items with instances (depth key != 0xFFFFFFFF in key2, item order) to
// the front of (depth_key, item_ids), in item order, for the depth sort of
// d_total[6] items (after the preprocess's count scan).
hipError_t launch_compact_items(const RenderParams &rp, const Buffers &b, hipStream_t s);
// Tile counts of the m items in depth order into cnt_sorted, with their sums
// per kScanGrain items into partial (for launch_count_scan).  Also clears the
// per-tile ranges and the tile-order counters.
hipError_t launch_gather_counts(const Buffers &b, int64_t m, int32_t total_tiles,
                                uint32_t *partial, hipStream_t s);
hipError_t launch_emit(const RenderParams &rp, const Buffers &b, int64_t m, int64_t capacity,
                       hipStream_t s);
// clear: zero the ranges first (done by launch_gather_counts when it ran).
hipError_t launch_ranges(const Buffers &b, int64_t capacity_bound, int32_t total_tiles,
                         bool clear, hipStream_t s);
// Per-tile re-sorting: key[j] = order-preserving bits of the view depth of
// the maximum of instance j's Gaussian on its tile-centre ray, idx[j] = j
// (j < the device instance count, at most bound).
hipError_t launch_resort_keys(const RenderParams &rp, const Buffers &b, uint32_t *key,
                              uint32_t *idx, int64_t bound, hipStream_t s);
// Permute the instance lists: (inst_key, inst_val)[j] = old[idx[j]], through
// the scratch arrays tmp_key / tmp_val.
hipError_t launch_resort_permute(const Buffers &b, const uint32_t *idx, uint32_t *tmp_key,
                                 uint32_t *tmp_val, int64_t bound, hipStream_t s);
// Order tiles by decreasing list length (heaviest first) into b.tile_order.
// clear: zero its counters first (done by launch_gather_counts when it ran).
hipError_t launch_tile_order(const Buffers &b, int32_t total_tiles, bool clear, hipStream_t s);
hipError_t launch_raster_fwd(const RenderParams &rp, const Buffers &b, bool count,
                             hipStream_t s);
hipError_t launch_raster_bwd(const RenderParams &rp, const Buffers &b, bool count,
                             hipStream_t s);
// Per-pixel window: bytes of the pair buffers per instance of capacity.
constexpr int64_t kWindowBytesPerInstance = 64 * (8 + 8);
// Entry k of tile lane `lane`'s compositing sequence (tile list starting at
// `start`; k below the list length): entry k of the tile's 64 lanes side by
// side, so that lanes at the same length store to one line.
__host__ __device__ inline size_t window_seq(uint32_t start, int k, int lane)
{
    return ((size_t)start + (size_t)k) * 64 + (size_t)lane;
}
// accumulate: add to the gradient arrays; otherwise overwrite every element.
// gnorm / vcount (may be null): densification statistics, always added to.
hipError_t launch_preprocess_bwd(const RenderParams &rp, const Buffers &b, const float *means,
                                 const float *quats, const float *scales, const float *dens,
                                 const float *sh, float *d_means, float *d_quats,
                                 float *d_scales, float *d_dens, float *d_sh, bool accumulate,
                                 float *gnorm, int32_t *vcount, hipStream_t s);

// Exclusive scan of the per-item instance counts in (n host-known, out may
// alias nothing), whose sums per kScanGrain values, tmp[0..ceil(n /
// kScanGrain)), the count gather already wrote: out = exclusive scan, out[n] =
// total K, and K (clamped to capacity, with the overflow flags) into
// d_total[0], [1], [5]; d_total[7] = 0.  tmp: scan_tmp_words(n) u32.
constexpr int64_t kScanGrain = 256;
int64_t scan_tmp_words(int64_t n);
hipError_t launch_count_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                             uint32_t *d_total, int64_t capacity, hipStream_t s);

// Radix sort of (key, val) u32 pairs; element count read from *d_n on the
// device, grids sized for n_bound.  Ping-pong buffers keys/vals <-> keys2/vals2;
// the sorted result ends in (keys, vals).  tmp: radix_tmp_words(n_bound).
int64_t radix_tmp_words(int64_t n_bound);
hipError_t launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                             const uint32_t *d_n, int64_t n_bound, int bits, uint32_t *tmp,
                             hipStream_t s);

}  // namespace vgr
