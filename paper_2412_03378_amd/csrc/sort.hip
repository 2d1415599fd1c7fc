// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs, written for wave64 gfx950.  The rasteriser uses them to order the
// (tile, depth) instance lists: the compositing assumes the Gaussians sorted
// front to back (Sec. 3.2), and the tile rasteriser sorts them per tile rather
// than per pixel (Sec. 7, Limitations).
//
// Radix pass = histogram kernel + per-digit exclusive scan of the digit-major
// table of per-block counts (one block per digit) + scatter kernel, which adds
// the digit starts (a scan of the 256 digit totals) itself.  The scatter ranks
// keys stably inside a 4096-key tile: each wave owns 1024 consecutive keys,
// ranks 64 keys at a time by matching digits with one ballot per digit bit,
// and keeps running per-digit counters in LDS.  The tile is then reordered by
// digit in LDS and written out run by run, so that neighbouring threads write
// neighbouring addresses.
#include "vgr_internal.h"

namespace vgr {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;   // 4096
static_assert(kTile % kScanGrain == 0, "scan grain");
constexpr int kWaves = kThreads / 64;

__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan across the 256 threads of a block; *total gets the sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        uint32_t s = wsum[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Single block: exclusive scan of the nb block sums in place, chunk by chunk.
// With d_total, the total is also the instance count K: d_total[0] = K
// clamped to capacity, d_total[1] = overflow, d_total[5] set (sticky) on
// overflow, d_total[7] = 0 (the emission's mismatch counter).
__global__ __launch_bounds__(kThreads) void scan_partials_kernel(uint32_t *__restrict__ partial,
                                                                 int64_t nb,
                                                                 uint32_t *__restrict__ total_out,
                                                                 uint32_t *__restrict__ d_total,
                                                                 int64_t capacity)
{
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kTile) {
        uint32_t v[kItems];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
            v[i] = idx < nb ? partial[idx] : 0u;
            s += v[i];
        }
        uint32_t chunk_total;
        uint32_t off = block_exclusive_scan(s, &chunk_total) + carry;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            int64_t idx = base + (int64_t)threadIdx.x * kItems + i;
            if (idx < nb) partial[idx] = off;
            off += v[i];
        }
        carry += chunk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
    if (threadIdx.x == 0 && d_total) {
        const bool over = (int64_t)carry > capacity;
        d_total[0] = over ? (uint32_t)capacity : carry;
        d_total[1] = over ? 1u : 0u;
        if (over) d_total[5] = 1u;   // sticky until the host clears it
        d_total[7] = 0u;
    }
}

__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t *__restrict__ in,
                                                             uint32_t *__restrict__ out,
                                                             int64_t n,
                                                             const uint32_t *__restrict__ partial)
{
    __shared__ uint32_t tile[kTile];
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
        tile[i * kThreads + threadIdx.x] = idx < n ? in[idx] : 0u;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        v[i] = tile[threadIdx.x * kItems + i];
        s += v[i];
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan(s, &total) + partial[blockIdx.x * (kTile / kScanGrain)];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        tile[threadIdx.x * kItems + i] = off;
        off += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
        if (idx < n) out[idx] = tile[i * kThreads + threadIdx.x];
    }
}

// ---------------------------------------------------------------- radix ---

template <int IPT>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                              const uint32_t *__restrict__ d_n,
                                                              int shift, uint32_t mask,
                                                              uint32_t *__restrict__ hist, int nb)
{
    __shared__ uint32_t h[kWaves][256];
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) h[k][threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = *d_n;
    const int64_t base = (int64_t)blockIdx.x * (kThreads * IPT);
    if (base < n) {
#pragma unroll 4
        for (int i = 0; i < IPT; ++i) {
            int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
            if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) s += h[k][threadIdx.x];
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = s;
}

// One block per digit: exclusive scan, in place, of that digit's row of the
// digit-major table (the per-block counts), and the row total into tot[d].
__global__ __launch_bounds__(kThreads) void radix_rowscan_kernel(uint32_t *__restrict__ table,
                                                                 int nb,
                                                                 uint32_t *__restrict__ tot)
{
    uint32_t *row = table + (int64_t)blockIdx.x * nb;
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kTile) {
        uint32_t v[kItems];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int idx = base + threadIdx.x * kItems + i;
            v[i] = idx < nb ? row[idx] : 0u;
            s += v[i];
        }
        uint32_t chunk;
        uint32_t off = block_exclusive_scan(s, &chunk) + carry;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int idx = base + threadIdx.x * kItems + i;
            if (idx < nb) row[idx] = off;
            off += v[i];
        }
        carry += chunk;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

template <int IPT>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const uint32_t *__restrict__ d_n, int shift, int dbits, const uint32_t *__restrict__ offs,
    const uint32_t *__restrict__ tot, int nb)
{
    __shared__ uint32_t cnt[kWaves][256];
    __shared__ uint32_t gdelta[256];   // global start minus block-local start
    constexpr int TILE = kThreads * IPT;
    __shared__ uint32_t sk[TILE], sv[TILE];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t mask = (1u << dbits) - 1u;
    const int64_t n = *d_n;
    const int64_t blk_base = (int64_t)blockIdx.x * TILE;
    if (blk_base >= n) return;   // uniform across the block
    // start of each digit = exclusive scan of the digit totals
    uint32_t tot_all;
    const uint32_t digit_start = block_exclusive_scan(tot[threadIdx.x], &tot_all);
#pragma unroll
    for (int k = 0; k < kWaves; ++k) cnt[k][threadIdx.x] = 0;
    __syncthreads();

    const int64_t wbase = blk_base + (int64_t)w * (TILE / kWaves);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t k[IPT], v[IPT], r[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t idx = wbase + i * 64 + lane;
        bool valid = idx < n;
        k[i] = valid ? keys[idx] : 0u;
        v[i] = valid ? vals[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t idx = wbase + i * 64 + lane;
        bool valid = idx < n;
        uint32_t d = (k[i] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t below = (uint32_t)__popcll(peers & lt_mask);
        uint32_t prev = valid ? cnt[w][d] : 0u;
        r[i] = prev + below;
        if (valid && below == 0) cnt[w][d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // per digit: block-local start (scan over digits of the block's counts),
        // then each wave's start inside it; global start from the digit-major
        // table of block offsets
        const int d = threadIdx.x;
        uint32_t c_d = 0;
#pragma unroll
        for (int k2 = 0; k2 < kWaves; ++k2) c_d += cnt[k2][d];
        uint32_t blk_count;
        const uint32_t ls = block_exclusive_scan(c_d, &blk_count);
        gdelta[d] = digit_start + offs[(int64_t)d * nb + blockIdx.x] - ls;
        uint32_t run = ls;
#pragma unroll
        for (int k2 = 0; k2 < kWaves; ++k2) {
            uint32_t c = cnt[k2][d];
            cnt[k2][d] = run;
            run += c;
        }
    }
    __syncthreads();
    // reorder the tile by digit in LDS ...
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t idx = wbase + i * 64 + lane;
        if (idx < n) {
            uint32_t d = (k[i] >> shift) & mask;
            uint32_t lp = cnt[w][d] + r[i];
            sk[lp] = k[i];
            sv[lp] = v[i];
        }
    }
    __syncthreads();
    // ... and write it out in order: consecutive threads write consecutive
    // positions of the same digit run
    const int64_t cnt_blk = min((int64_t)TILE, n - blk_base);
    for (int e = threadIdx.x; e < cnt_blk; e += kThreads) {
        const uint32_t key = sk[e];
        const uint32_t d = (key >> shift) & mask;
        const uint32_t pos = gdelta[d] + (uint32_t)e;
        keys_out[pos] = key;
        vals_out[pos] = sv[e];
    }
}

__global__ void copy_pairs_kernel(const uint32_t *__restrict__ k, const uint32_t *__restrict__ v,
                                  uint32_t *__restrict__ ko, uint32_t *__restrict__ vo,
                                  const uint32_t *__restrict__ d_n, int64_t bound)
{
    const int64_t n = *d_n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n && i < bound;
         i += (int64_t)gridDim.x * blockDim.x) {
        ko[i] = k[i];
        vo[i] = v[i];
    }
}

inline int64_t blocks_for(int64_t n) { return (n + kTile - 1) / kTile; }

}  // namespace

int64_t scan_tmp_words(int64_t n)
{
    return (n + kScanGrain - 1) / kScanGrain + 1;
}

hipError_t launch_count_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                             uint32_t *d_total, int64_t capacity, hipStream_t s)
{
    const int64_t ng = n > 0 ? (n + kScanGrain - 1) / kScanGrain : 0;
    scan_partials_kernel<<<1, kThreads, 0, s>>>(tmp, ng, out + (n > 0 ? n : 0), d_total,
                                                capacity);
    if (n > 0)
        scan_down_kernel<<<dim3((unsigned)blocks_for(n)), dim3(kThreads), 0, s>>>(in, out, n, tmp);
    return hipGetLastError();
}

// Keys per thread of a radix pass: 4 (1024-key tiles) below 4M keys, so that
// smaller sorts still spread over all CUs, else 16 (4096-key tiles).
constexpr int64_t kSmallSort = 1 << 22;

inline int64_t radix_blocks(int64_t n, int ipt) { return (n + kThreads * ipt - 1) / (kThreads * ipt); }

// Enough for a sort of any n <= n_bound (a smaller sort may use the smaller
// tiles and so more blocks).
int64_t radix_tmp_words(int64_t n_bound)
{
    const int64_t n = n_bound > 0 ? n_bound : 1;
    const int64_t nb_own = radix_blocks(n, n <= kSmallSort ? 4 : kItems);
    const int64_t nb_small = radix_blocks(n < kSmallSort ? n : kSmallSort, 4);
    return 256 * (nb_own > nb_small ? nb_own : nb_small) + 256;
}

hipError_t launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2,
                             const uint32_t *d_n, int64_t n_bound, int bits, uint32_t *tmp,
                             hipStream_t s)
{
    if (n_bound <= 0 || bits <= 0) return hipSuccess;
    const bool small = n_bound <= kSmallSort;
    const int64_t nb = radix_blocks(n_bound, small ? 4 : kItems);
    const int64_t table = 256 * nb;
    uint32_t *hist = tmp;            // digit-major per-block counts, then their row scans
    uint32_t *tot = tmp + table;     // per-digit totals
    const int passes = (bits + 7) / 8;
    // spread the bits evenly over the passes (each at most 8)
    int shift = 0;
    uint32_t *ki = keys, *vi = vals, *ko = keys2, *vo = vals2;
    for (int p = 0; p < passes; ++p) {
        const int dbits = (bits - shift + (passes - p) - 1) / (passes - p);
        const uint32_t mask = (1u << dbits) - 1u;
        const dim3 g((unsigned)nb), t(kThreads);
        if (small) radix_hist_kernel<4><<<g, t, 0, s>>>(ki, d_n, shift, mask, hist, (int)nb);
        else radix_hist_kernel<kItems><<<g, t, 0, s>>>(ki, d_n, shift, mask, hist, (int)nb);
        radix_rowscan_kernel<<<256, kThreads, 0, s>>>(hist, (int)nb, tot);
        if (small)
            radix_scatter_kernel<4><<<g, t, 0, s>>>(ki, vi, ko, vo, d_n, shift, dbits, hist, tot,
                                                     (int)nb);
        else
            radix_scatter_kernel<kItems><<<g, t, 0, s>>>(ki, vi, ko, vo, d_n, shift, dbits, hist,
                                                          tot, (int)nb);
        shift += dbits;
        uint32_t *tt;
        tt = ki; ki = ko; ko = tt;
        tt = vi; vi = vo; vo = tt;
    }
    if (ki != keys) {
        const int64_t grid = (n_bound + 255) / 256 < 65536 ? (n_bound + 255) / 256 : 65536;
        copy_pairs_kernel<<<dim3((unsigned)grid), 256, 0, s>>>(ki, vi, keys, vals, d_n, n_bound);
    }
    return hipGetLastError();
}

}  // namespace vgr
