// sort.hip - the discrete stage of tile-based splatting: one key per
// (tile, record) pair whose support box touches the tile, ordered by
// (global tile, camera depth, record), and per-tile [start, end) ranges.
//
//   1. scan + duplicate: an exclusive scan of the records' touched-tile counts
//      (record order; the projection writes each 256-record block's total)
//      places every record's keys; key = global tile id,
//      value = record id.  The total is checked against the key capacity on the
//      device.  No global atomics: counters with thousands of writers serialise
//      badly across the XCDs of this chip.
//   2. a stable least-significant-digit radix sort of the keys by tile id
//      (8-bit digits, ceil(log2(tiles)) bits): a fixed grid of G workgroups,
//      each owning one contiguous chunk whose size follows from the key count
//      read on the device (graph capture).  Per pass: per-workgroup digit
//      histograms (per-wave LDS sub-histograms), a column scan per digit, and a
//      scatter that ranks each wave's 64 keys with 8 ballots (peer masks) and
//      combines the waves in order (stable);
//   3. tile ranges from the boundaries of the sorted keys;
//   4. one workgroup per tile sorts its list by the float32 depth bits, equal
//      depths keeping the record order the list has on entry: lists of at most
//      256 keys are ranked (each entry counts the entries before it), longer
//      ones run the same stable LDS ranking as the tile sort (4 passes, skipped
//      when a digit is uniform), on global scratch beyond the LDS capacity.
// Depth bits of positive floats order like the floats, so the result is the
// (tile, depth, record) order.
#include "gs_internal.h"

namespace gsf {
namespace {

constexpr int kSortBlock = 256;              // threads per radix-sort workgroup (4 waves)
constexpr int kSortIpt = 8;                  // keys per thread per chunk tile
constexpr int kSortTile = kSortBlock * kSortIpt;
constexpr int kSortMaxGrid = 1024;
constexpr int kScanBlock = 256;
constexpr int kScanIpt = 1;                  // 256 records per block: 50k records fill 196 blocks
constexpr int kScanTile = kScanBlock * kScanIpt;
static_assert(kScanTile == 256, "the projection writes the count totals of 256-record blocks");
constexpr int kOwnPrefixBlocks = 1024;       // up to this many scan blocks, each sums its own prefix (no k_scan_top)
constexpr int kTileSortBlock = 256;
constexpr int kTileSortLds = 1024;           // list length sorted in LDS (22 KB: 7 workgroups per CU); longer lists use global scratch

__device__ __forceinline__ uint32_t chunk_size(uint32_t n, int G) {
    const uint32_t per = (n + (uint32_t)G - 1u) / (uint32_t)G;
    return (per + 255u) & ~255u;
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

// ---- 2. stable radix sort by tile id ------------------------------------------

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
    // Each pass over the chunk takes up to kSortTile keys; wave w ranks the
    // contiguous run [wbase, wbase + span) of them, span being the fewest whole
    // rounds of 64 that cover the keys left, so a short chunk still spreads over
    // the four waves (earlier waves hold earlier keys, as the in-order
    // combination needs).
    for (uint32_t tile0 = start, span; tile0 < end; tile0 += 4u * span) {
        const uint32_t left = end - tile0;
        span = min(64u * kSortIpt, (left + 255u) / 256u * 64u);
        const int rounds = (int)(span / 64u);   // workgroup-uniform
        for (int k = t; k < 4 * 256; k += kSortBlock) (&s_cnt[0][0])[k] = 0u;
        __syncthreads();
        uint32_t key[kSortIpt], val[kSortIpt], rank[kSortIpt];
        const uint32_t wbase = tile0 + (uint32_t)w * span;
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {
            if (r >= rounds) break;
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
            if (r >= rounds) break;
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

// ---- 1. scan of the touched-tile counts + key duplication (record order) -------

// The per-block totals of the counts (256 records a block) come from the
// projection kernel, which computes the counts.

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
        const unsigned long long y = threadIdx.x >= (unsigned)o ? s_part[threadIdx.x - o] : 0ull;
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

// Keys of each record (one per listed tile) at its scanned offset; also
// clears the tile ranges (grid-stride) before the boundary pass fills them.
// The block's keys are written by all its threads together, key q of the block
// by thread q mod 256: the record owning q is found by binary search over the
// block's offsets in LDS, so one record's many keys are spread over the block
// and consecutive threads write consecutive addresses.  Within a record the
// keys run over the box rows, each row's tiles being those its support
// ellipse reaches (row_span, the rule the projection counted with): from the
// packed spans, or from the record's row table, which the thread owning the
// record writes first (at the record's own key positions) and the key's
// thread then searches for the key's row.
__global__ __launch_bounds__(kScanBlock) void k_scan_dup(
    const uint32_t *__restrict__ count, const uint2 *__restrict__ rect,
    const float4 *__restrict__ ell, const uint2 *__restrict__ rspan, SplatPtrs sp,
    uint32_t *__restrict__ koff, uint2 *rowtab, int nrec, int n, int tile,
    const ViewDesc *__restrict__ views, const uint32_t *__restrict__ block_prefix, int nblocks,
    bool own_prefix, uint32_t *__restrict__ m_dev, unsigned long long *__restrict__ m_total,
    uint32_t *__restrict__ flags, int64_t capacity, uint32_t *__restrict__ keys,
    uint32_t *__restrict__ vals, uint2 *__restrict__ ranges, int total_tiles) {
    __shared__ uint32_t s_wave[4];
    __shared__ unsigned long long s_tot[4];
    __shared__ uint32_t s_off[kScanTile];   // block-local exclusive key offset per record
    __shared__ uint2 s_rect[kScanTile];
    __shared__ int s_view[kScanTile];
    __shared__ uint2 s_pack[kScanTile];       // packed row spans, or (row-table entries, -)
    __shared__ ViewDesc s_views[kMaxViews];   // read per key: kept in LDS, not reloaded from memory
    for (int t = blockIdx.x * kScanBlock + threadIdx.x; t < total_tiles; t += gridDim.x * kScanBlock)
        ranges[t] = make_uint2(0u, 0u);
    if ((int)threadIdx.x < min(nrec / n, kMaxViews)) s_views[threadIdx.x] = views[threadIdx.x];
    // The block's first key and the key total.  With own_prefix (at most
    // kOwnPrefixBlocks blocks) block_prefix holds the per-block totals and each
    // block sums those before it itself, block 0 publishing the total; else
    // k_scan_top has scanned them in place and published it.
    uint32_t gbase;
    unsigned long long total_keys;
    if (own_prefix) {
        unsigned long long pre = 0ull, all = 0ull;
        for (int b = threadIdx.x; b < nblocks; b += kScanBlock) {
            const unsigned long long c = block_prefix[b];
            all += c;
            if (b < (int)blockIdx.x) pre += c;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            pre += __shfl_xor(pre, o, 64);
            all += __shfl_xor(all, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            s_tot[threadIdx.x >> 6] = all;
            s_wave[threadIdx.x >> 6] = (uint32_t)min(pre, 0xFFFFFFFFull);
        }
        __syncthreads();
        total_keys = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
        gbase = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];   // used only when total fits
        __syncthreads();   // s_wave is reused by the block scan below
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *m_total = total_keys;
            if (total_keys > (unsigned long long)capacity) {
                *m_dev = 0u;
                atomicOr(flags, GSF_FLAG_CAPACITY);
            } else {
                *m_dev = (uint32_t)total_keys;
            }
        }
    } else {
        total_keys = *m_total;
        gbase = block_prefix[blockIdx.x];
    }
    if (total_keys > (unsigned long long)capacity) return;    // overflow: emit nothing
    const int rec0 = blockIdx.x * kScanTile;
    const int base = rec0 + threadIdx.x * kScanIpt;
    uint32_t cnt[kScanIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanIpt; k++) {
        cnt[k] = base + k < nrec ? count[base + k] : 0u;
        sum += cnt[k];
    }
    uint32_t total;
    uint32_t off = block_excl_scan_256(sum, s_wave, total);
#pragma unroll
    for (int k = 0; k < kScanIpt; k++) {
        const int i = threadIdx.x * kScanIpt + k;
        s_off[i] = off;
        if (cnt[k] != 0u) {
            const uint32_t r = (uint32_t)(base + k);
            koff[r] = gbase + off;             // the record's first key
            const uint2 rc = rect[r];
            s_rect[i] = rc;
            s_view[i] = (int)(r / (uint32_t)n);
            const int x0 = (int)(rc.x & 0xFFFFu), y0 = (int)(rc.x >> 16);
            const int x1 = (int)(rc.y & 0xFFFFu), y1 = (int)(rc.y >> 16);
            const uint2 pk = rspan[r];
            s_pack[i] = pk;
            if (y1 - y0 + 1 > kPackRows || x1 - x0 + 1 > kPackCols) {   // the row table
                const float4 ea = ell[r], a = sp.a[r], c = sp.c[r];
                const Ellipse e{ea.x, ea.y, ea.z, ea.w, sqrtf(ea.y / ea.z), a.x, a.y, (int)c.z, (int)c.w};
                const ViewDesc vd = views[r / (uint32_t)n];
                const int tl = 31 - __clz(tile);
                uint32_t j = 0, pre = 0;
                for (int ty = y0; ty <= y1 && j < pk.x; ty++) {
                    int c0, c1;
                    if (!row_span(e, ty, tl, vd.width, vd.height, x0, x1, c0, c1)) continue;
                    rowtab[gbase + off + j] = make_uint2((uint32_t)(ty - y0) | ((uint32_t)c0 << 16), pre);
                    pre += (uint32_t)(c1 - c0 + 1);
                    j++;
                }
            }
        }
        off += cnt[k];
    }
    __syncthreads();   // row tables written (the block's own global stores) and LDS filled
    for (uint32_t q = threadIdx.x; q < total; q += kScanBlock) {
        // the last record whose offset is <= q (records without keys share the
        // offset of the next record, so the last one is the owner)
        int lo = 0, hi = kScanTile - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= q) lo = mid; else hi = mid - 1;
        }
        uint32_t li = q - s_off[lo];              // index of the key within its record
        const uint32_t r = (uint32_t)(rec0 + lo);
        const uint2 rc = s_rect[lo];
        const int x0 = (int)(rc.x & 0xFFFFu), y0 = (int)(rc.x >> 16);
        const int x1 = (int)(rc.y & 0xFFFFu), y1 = (int)(rc.y >> 16);
        const ViewDesc vd = s_views[s_view[lo]];
        uint32_t key = 0u;
        if (y1 - y0 + 1 <= kPackRows && x1 - x0 + 1 <= kPackCols) {   // packed spans
            const uint2 pk = s_pack[lo];
            for (int k = 0; k < kPackRows; k++) {
                const uint32_t f = ((k < 2 ? pk.x : pk.y) >> (16 * (k & 1))) & 0xFFFFu;
                const uint32_t w = f >> 8;
                if (li < w) {
                    key = (uint32_t)vd.tile_off + (uint32_t)(y0 + k) * (uint32_t)vd.tiles_x +
                          (uint32_t)x0 + (f & 0xFFu) + li;
                    break;
                }
                li -= w;
            }
        } else {   // the last row-table entry whose key prefix is <= li holds key li
            const uint32_t tb = gbase + s_off[lo];
            int a = 0, b = (int)s_pack[lo].x - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (rowtab[tb + (uint32_t)mid].y <= li) a = mid; else b = mid - 1;
            }
            const uint2 te = rowtab[tb + (uint32_t)a];
            key = (uint32_t)vd.tile_off + ((uint32_t)y0 + (te.x & 0xFFFFu)) * (uint32_t)vd.tiles_x +
                  (te.x >> 16) + (li - te.y);
        }
        keys[gbase + q] = key;
        vals[gbase + q] = r;
    }
}

// ---- 3. tile ranges from the boundaries of the sorted keys -----------------------

// ranges[t] = [lower_bound(t), lower_bound(t + 1)) over the sorted keys, for every
// tile: an empty tile gets the position where its keys would be, so starts are
// non-decreasing in t (the checkpointed adjoint numbers its work units by them).
// A lane at a boundary owns the run of empty tiles before its key (and the last
// key the run after it); a run can be a thousand tiles long, so each wave writes
// its lanes' runs together, 64 tiles per store.  Tiles before the first key keep
// the (0, 0) the duplicate pass wrote.
__device__ __forceinline__ void fill_runs(uint2 *ranges, uint32_t lo, uint32_t hi, uint32_t value) {
    const int lane = __lane_id();
    uint64_t todo = __ballot(hi > lo);
    while (todo) {
        const int src = __builtin_ctzll(todo);
        const uint32_t a = __shfl(lo, src, 64), b = __shfl(hi, src, 64), v = __shfl(value, src, 64);
        for (uint32_t e = a + (uint32_t)lane; e < b; e += 64u) ranges[e] = make_uint2(v, v);
        todo &= todo - 1u;
    }
}

__global__ __launch_bounds__(256) void k_tile_bounds(const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ m_dev,
                                                     uint32_t m_host, int total_tiles,
                                                     uint2 *__restrict__ ranges) {
    const uint32_t m = m_dev ? *m_dev : m_host;
    const uint32_t stride = gridDim.x * blockDim.x;
    // wave-uniform trip count: every lane takes part in the run fills
    for (uint32_t base = blockIdx.x * blockDim.x; base < m; base += stride) {
        const uint32_t k = base + threadIdx.x;
        uint32_t lo = 0, hi = 0, lo2 = 0, hi2 = 0;
        if (k < m) {
            const uint32_t t = keys[k];
            if (k == 0 || keys[k - 1] != t) {
                lo = k == 0 ? t : keys[k - 1] + 1u;   // empty tiles before t
                hi = t;
                ranges[t].x = k;
            }
            if (k + 1 == m) {
                ranges[t].y = m;
                lo2 = t + 1u;                         // empty tiles after the last key
                hi2 = (uint32_t)total_tiles;
            } else if (keys[k + 1] != t) {
                ranges[t].y = k + 1;
            }
        }
        fill_runs(ranges, lo, hi, k);
        fill_runs(ranges, lo2, hi2, m);
    }
}

// ---- 3b. compositing order: tiles with more keys first ----------------------------

// Key-count class of a tile: 0 for an empty tile, else 1 + floor(log2(count)).
__device__ __forceinline__ uint32_t tile_class(const uint2 *__restrict__ ranges, int i) {
    const uint2 rg = ranges[i];
    const uint32_t len = rg.y - rg.x;
    return len ? 32u - (uint32_t)__clz(len) : 0u;
}

// Lanes of the wave with the same 6-bit class (valid lanes only).
__device__ __forceinline__ uint64_t class_peers(uint32_t c, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const uint64_t bal = __ballot((c >> k) & 1u);
        peers &= ((c >> k) & 1u) ? bal : ~bal;
    }
    return peers;
}

// One workgroup (at most 1024 kOrderU tiles): a counting sort of the tile ids
// by descending class, each wave aggregating its lanes per class before
// touching the LDS counters.  The classes of all rounds are loaded before any
// is used, so there is no chain of dependent global loads, and they and each
// wave's peer masks are kept from the counting to the placing; the 33 class
// counters are scanned by one wave.
constexpr int kOrderU = 8;

__global__ __launch_bounds__(1024) void k_tile_order(const uint2 *__restrict__ ranges, int total_tiles,
                                                     uint32_t *__restrict__ order) {
    __shared__ uint32_t s_cnt[64];
    const int t = threadIdx.x, lane = __lane_id();
    if (t < 64) s_cnt[t] = 0u;
    uint32_t c[kOrderU];
    uint64_t peers[kOrderU];
#pragma unroll
    for (int u = 0; u < kOrderU; u++) {
        const int i = u * 1024 + t;
        c[u] = i < total_tiles ? tile_class(ranges, i) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kOrderU; u++) {
        const bool valid = u * 1024 + t < total_tiles;
        peers[u] = class_peers(c[u], valid);
        if (valid && lanes_below(peers[u]) == 0u) atomicAdd(&s_cnt[c[u]], (uint32_t)__popcll(peers[u]));
    }
    __syncthreads();
    if (t < 64) {   // first slot of each class, class 32 first: exclusive scan over lanes 32 - c
        const int cls = 32 - lane;
        const uint32_t x = cls >= 0 ? s_cnt[cls] : 0u;
        uint32_t inc = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (cls >= 0) s_cnt[cls] = inc - x;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kOrderU; u++) {
        const int i = u * 1024 + t;
        const bool valid = i < total_tiles;
        const uint32_t below = lanes_below(peers[u]);
        uint32_t start = 0u;
        if (valid && below == 0u) start = atomicAdd(&s_cnt[c[u]], (uint32_t)__popcll(peers[u]));
        const int leader = peers[u] ? __builtin_ctzll(peers[u]) : lane;
        start = __shfl(start, leader, 64);
        if (valid) order[start + below] = (uint32_t)i;
    }
}

// Many tiles: the same counting sort over kOrderTiles tiles per workgroup.
// k_order_count writes each workgroup's class counts; k_order_place turns them
// into the workgroup's first slot per class (classes descending, workgroups in
// order) and places its tiles.
constexpr int kOrderTiles = 4096;

__device__ __forceinline__ void order_walk(const uint2 *__restrict__ ranges, int total_tiles,
                                           uint32_t *s_cnt, uint32_t *__restrict__ order) {
    const int t0 = blockIdx.x * kOrderTiles;
    const int t1 = min(total_tiles, t0 + kOrderTiles);
    for (int base = t0; base < t1; base += 256) {   // workgroup-uniform trip count
        const int i = base + (int)threadIdx.x;
        const bool valid = i < t1;
        const uint32_t c = valid ? tile_class(ranges, i) : 0u;
        const uint64_t peers = class_peers(c, valid);
        const uint32_t below = lanes_below(peers);
        uint32_t start = 0u;
        if (valid && below == 0u) start = atomicAdd(&s_cnt[c], (uint32_t)__popcll(peers));
        if (order) {
            const int leader = peers ? __builtin_ctzll(peers) : __lane_id();
            start = __shfl(start, leader, 64);
            if (valid) order[start + below] = (uint32_t)i;
        }
    }
}

__global__ __launch_bounds__(256) void k_order_count(const uint2 *__restrict__ ranges, int total_tiles,
                                                     uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_cnt[33];
    if (threadIdx.x < 33) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    order_walk(ranges, total_tiles, s_cnt, nullptr);
    __syncthreads();
    if (threadIdx.x < 33) counts[(size_t)blockIdx.x * 33 + threadIdx.x] = s_cnt[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_order_place(const uint2 *__restrict__ ranges, int total_tiles,
                                                     const uint32_t *__restrict__ counts, int groups,
                                                     uint32_t *__restrict__ order) {
    __shared__ uint32_t s_tot[33], s_cnt[33];
    const int c = threadIdx.x;
    if (c < 33) {
        uint32_t tot = 0, before = 0;
        for (int w = 0; w < groups; w++) {
            const uint32_t n = counts[(size_t)w * 33 + c];
            tot += n;
            if (w < (int)blockIdx.x) before += n;
        }
        s_tot[c] = tot;
        s_cnt[c] = before;
    }
    __syncthreads();
    if (c < 33) {
        uint32_t above = 0;
        for (int k = c + 1; k <= 32; k++) above += s_tot[k];
        s_cnt[c] += above;
    }
    __syncthreads();
    order_walk(ranges, total_tiles, s_cnt, order);
}

// ---- 4. per-tile sort by depth ----------------------------------------------------

struct SortShared {
    uint32_t hist[4][256];   // per-wave digit counts
    uint32_t base[256];      // running output offset per digit
    uint32_t tot[256];
    uint32_t wave[4];
    uint32_t skip;
};

// One stable pass by the 8-bit digit (k >> shift) & 0xFF.  Returns false (and
// moves nothing) when every key has the same digit.  Generic pointers: called
// on LDS arrays or on global scratch.
__device__ __forceinline__ bool sort_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                          uint32_t *vout, int n, int shift, SortShared &sh) {
    const int t = threadIdx.x, w = t >> 6, lane = __lane_id();
    for (int e = t; e < 4 * 256; e += kTileSortBlock) (&sh.hist[0][0])[e] = 0u;
    if (t == 0) sh.skip = 0u;
    __syncthreads();
    for (int i = t; i < n; i += kTileSortBlock) {
        const uint32_t d = (kin[i] >> shift) & 0xFFu;
        atomicAdd(&sh.hist[w][d], 1u);
    }
    __syncthreads();
    const uint32_t cnt = sh.hist[0][t] + sh.hist[1][t] + sh.hist[2][t] + sh.hist[3][t];
    if (cnt == (uint32_t)n) sh.skip = 1u;
    uint32_t all;
    sh.base[t] = block_excl_scan_256(cnt, sh.wave, all);   // (has barriers)
    const bool skip = sh.skip != 0u;
    __syncthreads();                       // all have read skip before a later pass resets it
    if (skip) return false;
    for (int c0 = 0; c0 < n; c0 += kTileSortBlock) {
        for (int e = t; e < 4 * 256; e += kTileSortBlock) (&sh.hist[0][0])[e] = 0u;
        __syncthreads();
        const int i = c0 + w * 64 + lane;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u, v = valid ? vin[i] : 0u;
        const uint32_t d = (k >> shift) & 0xFFu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = lanes_below(peers);
        if (valid && below == 0u) sh.hist[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {   // earlier waves of this chunk, per digit
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t c = sh.hist[q][t];
                sh.hist[q][t] = run;
                run += c;
            }
            sh.tot[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = sh.base[d] + sh.hist[w][d] + below;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        sh.base[t] += sh.tot[t];
    }
    __syncthreads();
    return true;
}

// Four stable passes over the 32 depth bits.  The list arrives in record order
// (stable tile sort of keys emitted in record order), so equal depths keep it.
__device__ __forceinline__ void sort_list(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                                          int n, SortShared &sh, bool &in_second) {
    bool second = false;
    for (int p = 0; p < 4; p++) {
        const bool moved = second ? sort_pass(k1, v1, k0, v0, n, 8 * p, sh)
                                  : sort_pass(k0, v0, k1, v1, n, 8 * p, sh);
        if (moved) second = !second;
    }
    in_second = second;
}

// Keys of s[j0, j1) below k (at most k when LE); j0 and j1 are multiples of 4.
template <bool LE>
__device__ __forceinline__ uint32_t count_keys(const uint32_t *s, int j0, int j1, uint32_t k) {
    const uint4 *q = reinterpret_cast<const uint4 *>(s);
    uint32_t c = 0u;
    for (int j = j0; j < j1; j += 4) {
        const uint4 v = q[j >> 2];
        if (LE)
            c += (uint32_t)(v.x <= k) + (uint32_t)(v.y <= k) + (uint32_t)(v.z <= k) + (uint32_t)(v.w <= k);
        else
            c += (uint32_t)(v.x < k) + (uint32_t)(v.y < k) + (uint32_t)(v.z < k) + (uint32_t)(v.w < k);
    }
    return c;
}

__global__ __launch_bounds__(kTileSortBlock) void k_tile_sort(
    const uint32_t *__restrict__ order, const uint2 *__restrict__ ranges,
    const uint32_t *__restrict__ depth_key,
    uint32_t *__restrict__ vals, uint32_t *__restrict__ gk0, uint32_t *__restrict__ gk1,
    uint32_t *__restrict__ gv1) {
    __shared__ SortShared sh;
    __shared__ __align__(16) uint32_t s_k0[kTileSortLds];
    __shared__ uint32_t s_v0[kTileSortLds], s_k1[kTileSortLds], s_v1[kTileSortLds];
    const uint2 rg = ranges[order[blockIdx.x]];   // tiles with the longest lists first
    const int n = (int)(rg.y - rg.x);
    if (n <= 1) return;
    uint32_t *lv = vals + rg.x;
    bool second;
    if (n <= kTileSortBlock) {
        // Short list: entry i goes to the count of entries before it in (depth
        // bits, list position) order, the order the stable passes give.  A
        // wave's entries are 64 consecutive positions, so earlier waves' keys
        // count when at most the entry's depth, later ones when below it, and
        // only the wave's own run compares positions.  The depths are padded to
        // a multiple of 4 with a key above every depth (depth bits of finite or
        // infinite floats are below 0x7F800001).
        const int i = threadIdx.x;
        const int np = (n + 3) & ~3;
        uint32_t r = 0u;
        if (i < n) {
            r = lv[i];
            s_k0[i] = depth_key[r];
        } else if (i < np) {
            s_k0[i] = 0xFFFFFFFFu;
        }
        __syncthreads();
        if (i < n) {
            const uint32_t k = s_k0[i];
            const int w0 = i & ~63, w1 = min(w0 + 64, np);
            uint32_t rank = count_keys<true>(s_k0, 0, w0, k) + count_keys<false>(s_k0, w1, np, k);
            const uint4 *q = reinterpret_cast<const uint4 *>(s_k0);
            for (int j = w0; j < w1; j += 4) {   // equal depths count when earlier
                const uint4 v = q[j >> 2];
                rank += (uint32_t)(v.x < k + (uint32_t)(j < i)) + (uint32_t)(v.y < k + (uint32_t)(j + 1 < i)) +
                        (uint32_t)(v.z < k + (uint32_t)(j + 2 < i)) + (uint32_t)(v.w < k + (uint32_t)(j + 3 < i));
            }
            lv[rank] = r;
        }
    } else if (n <= kTileSortLds) {
        for (int i = threadIdx.x; i < n; i += kTileSortBlock) {
            const uint32_t r = lv[i];
            s_v0[i] = r;
            s_k0[i] = depth_key[r];
        }
        __syncthreads();
        sort_list(s_k0, s_v0, s_k1, s_v1, n, sh, second);
        const uint32_t *res = second ? s_v1 : s_v0;
        for (int i = threadIdx.x; i < n; i += kTileSortBlock) lv[i] = res[i];
    } else {
        uint32_t *k0 = gk0 + rg.x, *k1 = gk1 + rg.x, *v1 = gv1 + rg.x;
        for (int i = threadIdx.x; i < n; i += kTileSortBlock) k0[i] = depth_key[lv[i]];
        __syncthreads();
        sort_list(k0, lv, k1, v1, n, sh, second);
        if (second)
            for (int i = threadIdx.x; i < n; i += kTileSortBlock) lv[i] = v1[i];
    }
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

int scan_blocks(int64_t nrec) { return (int)((nrec + kScanTile - 1) / kScanTile) + 1; }

void launch_scan_duplicate(hipStream_t s, const uint32_t *count, const uint2 *rect,
                           const float4 *ell, const uint2 *rspan, SplatPtrs sp, uint32_t *koff,
                           uint2 *rowtab, int nrec, int n, int tile,
                           const ViewDesc *views, uint32_t *block_sums, uint32_t *keys,
                           uint32_t *vals, uint32_t *m_dev, unsigned long long *m_total,
                           uint32_t *flags, int64_t capacity, uint2 *ranges, int total_tiles) {
    const int nb = (nrec + kScanTile - 1) / kScanTile;
    const bool own_prefix = nb >= 1 && nb <= kOwnPrefixBlocks;   // else k_scan_top writes the total
    if (!own_prefix) k_scan_top<<<1, 1024, 0, s>>>(block_sums, nb, m_dev, m_total, flags, capacity);
    k_scan_dup<<<nb, kScanBlock, 0, s>>>(count, rect, ell, rspan, sp, koff, rowtab, nrec, n, tile, views,
                                         block_sums, nb, own_prefix, m_dev, m_total, flags,
                                         capacity, keys, vals, ranges, total_tiles);
}

void launch_tile_bounds(hipStream_t s, const uint32_t *keys, const uint32_t *m_dev, uint32_t m_host,
                        int64_t capacity, int total_tiles, uint2 *ranges) {
    int64_t g = (capacity + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    k_tile_bounds<<<(int)g, 256, 0, s>>>(keys, m_dev, m_host, total_tiles, ranges);
}

int order_groups(int64_t total_tiles) { return (int)((total_tiles + kOrderTiles - 1) / kOrderTiles); }

void launch_tile_order(hipStream_t s, const uint2 *ranges, int total_tiles, uint32_t *order,
                       uint32_t *counts) {
    if (total_tiles <= 1024 * kOrderU) {
        k_tile_order<<<1, 1024, 0, s>>>(ranges, total_tiles, order);
        return;
    }
    const int g = order_groups(total_tiles);
    k_order_count<<<g, 256, 0, s>>>(ranges, total_tiles, counts);
    k_order_place<<<g, 256, 0, s>>>(ranges, total_tiles, counts, g, order);
}

void launch_tile_sort(hipStream_t s, const uint32_t *order, const uint2 *ranges, int total_tiles,
                      const uint32_t *depth_key, uint32_t *vals, uint32_t *gk0, uint32_t *gk1,
                      uint32_t *gv1) {
    k_tile_sort<<<total_tiles, kTileSortBlock, 0, s>>>(order, ranges, depth_key, vals, gk0, gk1, gv1);
}

}  // namespace gsf
