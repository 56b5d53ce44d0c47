// sort.hip - the discrete stage of tile-based splatting: per-record tile counts
// scanned in depth order, one (tile, record) key per touched tile, a stable
// radix sort of those keys by tile, and per-tile [start, end) ranges.
//
// The order that compositing needs is (global tile, depth, record).  It is
// reached with two stable sorts: records are first sorted by their float32
// depth bits (stable, so ties keep the record order), the duplication then
// emits keys in that order, and a stable sort by tile id alone finishes the job.
// The tile sort thus needs only ceil(log2(tiles)) key bits instead of tile bits
// plus 32 depth bits.
//
// Radix sort: least-significant-digit first, 8-bit digits, reduce-then-scan
// with a fixed grid of G workgroups, each owning one contiguous chunk of the
// input whose size is derived from the key count read on the device, so the
// launches do not depend on a host-side count (graph capture).  Per pass:
//   hist    per-workgroup digit histogram (per-wave LDS sub-histograms)
//   colscan one workgroup per digit scans that digit's G counts
//   scatter each workgroup re-reads its chunk in 2048-key tiles; a wave ranks
//           its 64 keys per round by matching digits with 8 ballots (peer
//           masks), keeps per-wave running digit counts in LDS, and the tile's
//           waves are combined in digit order, which keeps the sort stable.
#include "gs_internal.h"

namespace gsf {
namespace {

__device__ __forceinline__ uint32_t chunk_size(uint32_t n, int G) {
    const uint32_t per = (n + (uint32_t)G - 1u) / (uint32_t)G;
    return (per + 255u) & ~255u;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t x, uint32_t *s_wave, uint32_t &total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (k < w) base += s_wave[k];
    total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    return base + inc - x;
}

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ n_dev,
                                                           uint32_t n_host, int shift, int bits,
                                                           uint32_t *__restrict__ hist, int G) {
    __shared__ uint32_t h[4][256];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t chunk = chunk_size(n, G);
    const uint32_t start = min(n, (uint32_t)blockIdx.x * chunk);
    const uint32_t end = min(n, start + chunk);
    const int w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < 4 * 256; d += kSortBlock) (&h[0][0])[d] = 0u;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    for (uint32_t idx = start + threadIdx.x; idx < end; idx += kSortBlock)
        atomicAdd(&h[w][(keys[idx] >> shift) & mask], 1u);
    __syncthreads();
    const int nd = 1 << bits;
    for (int d = threadIdx.x; d < nd; d += kSortBlock)
        hist[(size_t)d * G + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// One workgroup per digit: exclusive scan of that digit's per-workgroup counts.
__global__ __launch_bounds__(256) void k_radix_colscan(uint32_t *__restrict__ hist, int G,
                                                       uint32_t *__restrict__ digit_tot) {
    __shared__ uint32_t s_wave[4];
    uint32_t *row = hist + (size_t)blockIdx.x * G;
    const int per = (G + 255) / 256;
    const int base = threadIdx.x * per;
    uint32_t local[4];
    uint32_t sum = 0;
    for (int k = 0; k < per; k++) {
        const uint32_t c = base + k < G ? row[base + k] : 0u;
        local[k] = c;
        sum += c;
    }
    uint32_t total;
    uint32_t run = block_excl_scan_256(sum, s_wave, total);
    for (int k = 0; k < per; k++)
        if (base + k < G) {
            row[base + k] = run;
            run += local[k];
        }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
    int bits, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ digit_tot, int G) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_cnt[4][256];
    __shared__ uint32_t s_tot[256];
    __shared__ uint32_t s_wave[4];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t chunk = chunk_size(n, G);
    const uint32_t start = min(n, (uint32_t)blockIdx.x * chunk);
    const uint32_t end = min(n, start + chunk);
    const int nd = 1 << bits;
    const uint32_t mask = (uint32_t)nd - 1u;
    const int t = threadIdx.x, w = t >> 6, lane = __lane_id();
    {   // global base of each digit for this workgroup
        const uint32_t tot = t < nd ? digit_tot[t] : 0u;
        uint32_t all;
        const uint32_t dp = block_excl_scan_256(tot, s_wave, all);
        if (t < nd) s_base[t] = dp + hist[(size_t)t * G + blockIdx.x];
    }
    for (uint32_t tile0 = start; tile0 < end; tile0 += kSortTile) {
        for (int k = t; k < 4 * 256; k += kSortBlock) (&s_cnt[0][0])[k] = 0u;
        __syncthreads();
        uint32_t key[kSortIpt], val[kSortIpt], rank[kSortIpt];
        const uint32_t wbase = tile0 + (uint32_t)w * 64u * kSortIpt;
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {
            const uint32_t idx = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            const bool valid = idx < end;
            key[r] = valid ? kin[idx] : 0u;
            val[r] = valid ? vin[idx] : 0u;
            const uint32_t d = (key[r] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < bits; b++) {
                const uint64_t bal = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bal : ~bal;
            }
            const uint32_t below = lanes_below(peers);
            uint32_t base = 0;
            if (valid) base = s_cnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (valid && below == 0u) s_cnt[w][d] = base + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
            rank[r] = base + below;
        }
        __syncthreads();
        if (t < nd) {   // combine the waves of this tile in order, per digit
            uint32_t run = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t c = s_cnt[k][t];
                s_cnt[k][t] = run;
                run += c;
            }
            s_tot[t] = run;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {
            const uint32_t idx = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            if (idx < end) {
                const uint32_t d = (key[r] >> shift) & mask;
                const uint32_t pos = s_base[d] + s_cnt[w][d] + rank[r];
                kout[pos] = key[r];
                vout[pos] = val[r];
            }
        }
        __syncthreads();
        if (t < nd) s_base[t] += s_tot[t];
        __syncthreads();
    }
}

// ---- scan of tile counts in depth order + key duplication -------------------------

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t *__restrict__ order,
                                                            const uint32_t *__restrict__ count,
                                                            int nrec, uint32_t *__restrict__ block_sums) {
    __shared__ uint32_t s_wave[4];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanIpt;
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; k++)
        if (base + k < nrec) sum += count[order[base + k]];
    uint32_t total;
    block_excl_scan_256(sum, s_wave, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t *__restrict__ block_sums, int nblocks,
                                                   uint32_t *__restrict__ m_dev,
                                                   unsigned long long *__restrict__ m_total,
                                                   uint32_t *__restrict__ flags, int64_t capacity) {
    __shared__ unsigned long long s_part[1024];
    const int per = (nblocks + 1023) / 1024;
    const int base = threadIdx.x * per;
    unsigned long long sum = 0;
    for (int k = 0; k < per; k++)
        if (base + k < nblocks) sum += block_sums[base + k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int o = 1; o < 1024; o <<= 1) {
        const unsigned long long y = threadIdx.x >= o ? s_part[threadIdx.x - o] : 0ull;
        __syncthreads();
        s_part[threadIdx.x] += y;
        __syncthreads();
    }
    unsigned long long run = s_part[threadIdx.x] - sum;
    for (int k = 0; k < per; k++)
        if (base + k < nblocks) {
            const uint32_t c = block_sums[base + k];
            block_sums[base + k] = (uint32_t)min(run, 0xFFFFFFFFull);
            run += c;
        }
    if (threadIdx.x == 1023) {
        const unsigned long long total = s_part[1023];
        *m_total = total;
        if (total > (unsigned long long)capacity) {
            *m_dev = 0u;
            atomicOr(flags, GSF_FLAG_CAPACITY);
        } else {
            *m_dev = (uint32_t)total;
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_dup(
    const uint32_t *__restrict__ order, const uint32_t *__restrict__ count,
    const uint2 *__restrict__ rect, int nrec, int n, const ViewDesc *__restrict__ views,
    const uint32_t *__restrict__ block_prefix, const unsigned long long *__restrict__ m_total,
    int64_t capacity, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    __shared__ uint32_t s_wave[4];
    if (*m_total > (unsigned long long)capacity) return;    // overflow: emit nothing
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanIpt;
    uint32_t rec[kScanIpt], cnt[kScanIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; k++) {
        rec[k] = base + k < nrec ? order[base + k] : 0u;
        cnt[k] = base + k < nrec ? count[rec[k]] : 0u;
        sum += cnt[k];
    }
    uint32_t total;
    uint32_t off = block_prefix[blockIdx.x] + block_excl_scan_256(sum, s_wave, total);
#pragma unroll
    for (int k = 0; k < kScanIpt; k++) {
        if (cnt[k] == 0u) continue;
        const uint32_t r = rec[k];
        const int v = (int)(r / (uint32_t)n);
        const ViewDesc vd = views[v];
        const uint2 rc = rect[r];
        const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu, y1 = rc.y >> 16;
        uint32_t o = off;
        for (uint32_t ty = y0; ty <= y1; ty++) {
            const uint32_t row = (uint32_t)vd.tile_off + ty * (uint32_t)vd.tiles_x;
            for (uint32_t tx = x0; tx <= x1; tx++) {
                keys[o] = row + tx;
                vals[o] = r;
                o++;
            }
        }
        off += cnt[k];
    }
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ m_dev,
                                                     uint32_t m_host, int total_tiles,
                                                     uint2 *__restrict__ ranges) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total_tiles) return;
    const uint32_t m = m_dev ? *m_dev : m_host;
    // lower bounds of t and t + 1
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < (uint32_t)t) lo = mid + 1; else hi = mid;
    }
    const uint32_t a = lo;
    hi = m;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < (uint32_t)t + 1u) lo = mid + 1; else hi = mid;
    }
    ranges[t] = make_uint2(a, lo);
}

}  // namespace

int radix_grid_for(int64_t capacity) {
    int64_t g = (capacity + kSortTile - 1) / kSortTile;
    if (g < 1) g = 1;
    if (g > kSortMaxGrid) g = kSortMaxGrid;
    return (int)g;
}

int launch_radix_sort(hipStream_t s, const uint32_t *kin, const uint32_t *vin, uint32_t *ka,
                      uint32_t *va, uint32_t *kb, uint32_t *vb, const uint32_t *n_dev,
                      uint32_t n_host, int bits, int grid, uint32_t *hist, uint32_t *digit_tot) {
    int where = 0;
    const uint32_t *ks = kin, *vs = vin;
    for (int shift = 0; shift < bits; shift += 8) {
        const int b = bits - shift < 8 ? bits - shift : 8;
        uint32_t *kd = where == 1 ? kb : ka, *vd = where == 1 ? vb : va;
        k_radix_hist<<<grid, kSortBlock, 0, s>>>(ks, n_dev, n_host, shift, b, hist, grid);
        k_radix_colscan<<<1 << b, 256, 0, s>>>(hist, grid, digit_tot);
        k_radix_scatter<<<grid, kSortBlock, 0, s>>>(ks, vs, kd, vd, n_dev, n_host, shift, b, hist,
                                                    digit_tot, grid);
        where = where == 1 ? 2 : 1;
        ks = kd;
        vs = vd;
    }
    return where;
}

void launch_scan_duplicate(hipStream_t s, const uint32_t *order, const uint32_t *count,
                           const uint2 *rect, int nrec, int n, const ViewDesc *views, int nviews,
                           uint32_t *block_sums, uint32_t *keys, uint32_t *vals, uint32_t *m_dev,
                           unsigned long long *m_total, uint32_t *flags, int64_t capacity) {
    (void)nviews;
    const int nb = (nrec + kScanTile - 1) / kScanTile;
    k_scan_reduce<<<nb, kScanBlock, 0, s>>>(order, count, nrec, block_sums);
    k_scan_top<<<1, 1024, 0, s>>>(block_sums, nb, m_dev, m_total, flags, capacity);
    k_scan_dup<<<nb, kScanBlock, 0, s>>>(order, count, rect, nrec, n, views, block_sums, m_total,
                                         capacity, keys, vals);
}

void launch_tile_ranges(hipStream_t s, const uint32_t *keys, const uint32_t *m_dev, uint32_t m_host,
                        int total_tiles, uint2 *ranges) {
    k_tile_ranges<<<(total_tiles + 255) / 256, 256, 0, s>>>(keys, m_dev, m_host, total_tiles, ranges);
}

}  // namespace gsf
