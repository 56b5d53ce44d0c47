// sort.hip - the discrete stage of tile-based splatting: one key per
// (tile, record) pair whose support ellipse reaches the tile, ordered by
// (global tile, camera depth, record), and per-tile [start, end) ranges.
//
//   1. record scan: an exclusive scan of the records' listed-tile counts in
//      record order (the projection writes each 256-record block's total) gives
//      each record its run of gradient slots (koff, where the adjoint stores the
//      per-key gradients and a record's row table lives); the key total is
//      checked against the capacity on the device; the records that list a tile
//      are compacted with their float32 depth bits.  No global atomics:
//      counters with thousands of writers serialise badly across the XCDs.
//   2. depth sort: a stable least-significant-digit radix sort of those
//      (depth bits, record) pairs (31 bits: depths are positive), so equal
//      depths keep the record order;
//   3. emission: every record's keys (key = global tile id, value = record id)
//      written in that depth order, placed by a second scan of the counts;
//   4. a stable LSD radix sort of the keys by tile id: each tile's list then
//      holds its records in (depth, record) order with no per-tile sort.
//      Both sorts use a fixed grid of G workgroups, each owning one contiguous
//      chunk whose size follows from the count read on the device (graph
//      capture).  Per pass of a digit of at most 11 bits: per-workgroup digit
//      histograms (per-wave LDS sub-histograms), a column scan per digit, and a
//      scatter that ranks each wave's 64 keys with one ballot per digit bit
//      (peer masks) and combines the waves in order (stable);
//   5. tile ranges from the boundaries of the sorted keys, and the compositing
//      order (tiles with more keys first).
// Depth bits of positive floats order like the floats.
#include "gs_internal.h"

namespace gsf {
namespace {

constexpr int kSortBlock = 256;              // threads per radix-sort workgroup (4 waves)
constexpr int kSortIpt = 16;                 // keys per thread per chunk tile
constexpr int kSortTile = kSortBlock * kSortIpt;
constexpr int kSortMaxGrid = 1024;
constexpr int kMaxDigit = 8;                 // radix digits of at most 256 bins
constexpr int kHistU = 16;                   // keys in flight per thread while counting digits
constexpr int kLocalScanGrid = 64;           // radix grids up to this sum their digit offsets in the scatter
constexpr int kScanBlock = 256;
constexpr int kScanIpt = 1;                  // 256 records per block: 50k records fill 196 blocks
constexpr int kScanTile = kScanBlock * kScanIpt;
static_assert(kScanTile == 256, "the projection writes the count totals of 256-record blocks");
constexpr int kScanRecRounds = 2;           // 256-record rounds per workgroup of the record scan
constexpr int kOwnPrefixBlocks = 1024;       // up to this many scan blocks, each sums its own prefix (no k_seg_scan)
constexpr int kSegBlocks = 1024;             // block totals per segment of k_seg_scan

// A depth-sort value holds the entry index in its low `ebits` bits and the
// record's tile count, saturated, above them, so that the emission's block
// totals read the sorted values instead of gathering an entry per record.
// ebits = 32: no room for a count (plans of more than 2^26 records).
int entry_bits(int nrec) {
    int b = 1;
    while ((int64_t(1) << b) < nrec) b++;
    return b > 26 ? 32 : b;
}
struct ValPack {
    uint32_t emask, cmax;
    int ebits;
    __host__ __device__ explicit ValPack(int eb)
        : emask(eb >= 32 ? 0xFFFFFFFFu : (1u << eb) - 1u), cmax(eb >= 32 ? 0u : (1u << (32 - eb)) - 1u),
          ebits(eb) {}
    __device__ uint32_t pack(uint32_t e, uint32_t c) const {
        return ebits >= 32 ? e : e | (min(c, cmax) << ebits);
    }
    __device__ uint32_t entry(uint32_t v) const { return v & emask; }
    // the count, or cmax (saturated: read the entry instead)
    __device__ uint32_t count(uint32_t v) const { return ebits >= 32 ? cmax : v >> ebits; }
};

__device__ __forceinline__ uint32_t chunk_size(uint32_t n, int G) {
    const uint32_t per = (n + (uint32_t)G - 1u) / (uint32_t)G;
    return (per + 255u) & ~255u;
}

// Optional controls of a radix pass (all null: a plain pass over the key bits).
//   base:  the digits are those of key - *base (the keys are written unchanged)
//   skip:  *skip != 0: the pass has nothing to do and returns at once
//   last:  *last != 0: this is the sort's last pass: the values go to vlast
//          and no keys are written
//   mm:    the histogram writes each workgroup's smallest and largest key
//          (mm[2 g], mm[2 g + 1]); with ctl, the scatter's last workgroup
//          reduces them to ctl[0] = the smallest key with its low 8 bits
//          cleared and ctl[1] = 1 when every key lies below ctl[0] + 2^24
struct RadixCtl {
    const uint32_t *base = nullptr;
    const uint32_t *skip = nullptr;
    const uint32_t *last = nullptr;
    uint32_t *vlast = nullptr;
    uint32_t *mm = nullptr;
    uint32_t *ctl = nullptr;
};

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

// ---- stable LSD radix sort of (key, value) pairs ------------------------------------
// A pass sorts by a digit of `bits` <= 8 bits at `shift`.

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ n_dev,
                                                           uint32_t n_host, int shift, int bits,
                                                           uint32_t *__restrict__ hist, int G,
                                                           RadixCtl ctl) {
    __shared__ uint32_t h[4][256];
    __shared__ uint32_t s_mm[8];
    if (ctl.skip && *ctl.skip) return;
    const uint32_t kb = ctl.base ? *ctl.base : 0u;
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t chunk = chunk_size(n, G);
    const uint32_t start = min(n, (uint32_t)blockIdx.x * chunk);
    const uint32_t end = min(n, start + chunk);
    const int w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < 4 * 256; d += kSortBlock) (&h[0][0])[d] = 0u;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
    // kHistU keys per thread are loaded before any is counted, so their loads
    // are in flight together
    for (uint32_t base = start; base < end; base += kSortBlock * kHistU) {
        uint32_t k[kHistU];
#pragma unroll
        for (int u = 0; u < kHistU; u++) {
            const uint32_t idx = base + (uint32_t)(u * kSortBlock) + threadIdx.x;
            k[u] = idx < end ? keys[idx] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistU; u++)
            if (base + (uint32_t)(u * kSortBlock) + threadIdx.x < end) {
                atomicAdd(&h[w][((k[u] - kb) >> shift) & mask], 1u);
                kmin = min(kmin, k[u]);
                kmax = max(kmax, k[u]);
            }
    }
    if (ctl.mm) {   // the workgroup's smallest and largest key
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            s_mm[w] = kmin;
            s_mm[4 + w] = kmax;
        }
    }
    __syncthreads();
    if (ctl.mm && threadIdx.x == 0) {
        ctl.mm[2 * blockIdx.x] = min(min(s_mm[0], s_mm[1]), min(s_mm[2], s_mm[3]));
        ctl.mm[2 * blockIdx.x + 1] = max(max(s_mm[4], s_mm[5]), max(s_mm[6], s_mm[7]));
    }
    const int nd = 1 << bits;
    for (int d = threadIdx.x; d < nd; d += kSortBlock)
        hist[(size_t)d * G + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// One workgroup per digit: exclusive scan of that digit's per-workgroup counts.
__global__ __launch_bounds__(256) void k_radix_colscan(uint32_t *__restrict__ hist, int G,
                                                       uint32_t *__restrict__ digit_tot,
                                                       const uint32_t *__restrict__ skip) {
    __shared__ uint32_t s_wave[4];
    if (skip && *skip) return;
    uint32_t *row = hist + (size_t)blockIdx.x * G;
    const int per = (G + 255) / 256;   // G <= kSortMaxGrid
    const int base = threadIdx.x * per;
    uint32_t local[(kSortMaxGrid + 255) / 256];
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

// Each workgroup ranks its chunk a round of up to kSortTile keys at a time,
// reorders the round by digit in LDS (stable) and then writes it out in that
// order: consecutive threads write consecutive addresses within each digit's
// run, so the stores coalesce.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ n_dev, uint32_t n_host, int shift,
    int bits, const uint32_t *__restrict__ hist, const uint32_t *__restrict__ digit_tot, int G,
    RadixCtl ctl) {
    __shared__ uint32_t s_base[256];      // next global position of each digit
    __shared__ uint32_t s_loc[256];       // first local position of each digit in the round
    __shared__ uint32_t s_cnt[4][256];
    __shared__ uint32_t s_tot[256];
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    if (ctl.skip && *ctl.skip) return;
    const uint32_t kb = ctl.base ? *ctl.base : 0u;
    // the sort's last pass: the values to vlast, no keys
    const bool lastp = ctl.last && *ctl.last;
    uint32_t *const ko = lastp ? nullptr : kout;
    uint32_t *const vo = lastp ? ctl.vlast : vout;
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint32_t chunk = chunk_size(n, G);
    const uint32_t start = min(n, (uint32_t)blockIdx.x * chunk);
    const uint32_t end = min(n, start + chunk);
    const int nd = 1 << bits;
    const uint32_t mask = (uint32_t)nd - 1u;
    const int t = threadIdx.x, w = t >> 6, lane = __lane_id();
    // the key range from the histogram's per-workgroup extremes, reduced by the
    // last workgroup (chunks are rounded up, so it holds the fewest keys)
    if (ctl.ctl && (int)blockIdx.x == G - 1) {
        uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
        for (int g = t; g < G; g += kSortBlock) {
            kmin = min(kmin, ctl.mm[2 * g]);
            kmax = max(kmax, ctl.mm[2 * g + 1]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
        }
        if (lane == 0) {
            s_base[w] = kmin;
            s_base[4 + w] = kmax;
        }
        __syncthreads();
        if (t == 0) {
            kmin = min(min(s_base[0], s_base[1]), min(s_base[2], s_base[3]));
            kmax = max(max(s_base[4], s_base[5]), max(s_base[6], s_base[7]));
            const uint32_t b = kmin <= kmax ? kmin & ~0xFFu : 0u;   // no keys: any base
            ctl.ctl[0] = b;
            ctl.ctl[1] = kmin > kmax || kmax - b < (1u << 24) ? 1u : 0u;
        }
        __syncthreads();   // s_base is free again
    }
    if (digit_tot) {   // global base of each digit for this workgroup (hist scanned per digit)
        const uint32_t tot = t < nd ? digit_tot[t] : 0u;
        uint32_t all;
        const uint32_t dp = block_excl_scan_256(tot, s_wave, all);
        if (t < nd) s_base[t] = dp + hist[(size_t)t * G + blockIdx.x];
    } else {   // few workgroups: each sums the raw counts itself (no scan launch)
        uint32_t tot = 0u, before = 0u;
        if (t < nd) {
            const uint32_t *row = hist + (size_t)t * G;
#pragma unroll 8
            for (int g = 0; g < G; g++) {
                const uint32_t c = row[g];
                tot += c;
                before += g < (int)blockIdx.x ? c : 0u;
            }
        }
        uint32_t all;
        const uint32_t dp = block_excl_scan_256(tot, s_wave, all);
        if (t < nd) s_base[t] = dp + before;
    }
    // Each round takes up to kSortTile keys; wave w ranks the contiguous run
    // [wbase, wbase + span) of them, span being the fewest whole rounds of 64
    // that cover the keys left, so a short chunk still spreads over the four
    // waves (earlier waves hold earlier keys, as the in-order combination needs).
    for (uint32_t tile0 = start, span; tile0 < end; tile0 += 4u * span) {
        const uint32_t left = end - tile0;
        span = min(64u * kSortIpt, (left + 255u) / 256u * 64u);
        const int rounds = (int)(span / 64u);   // workgroup-uniform
        for (int k = t; k < 4 * 256; k += kSortBlock) (&s_cnt[0][0])[k] = 0u;
        __syncthreads();
        uint32_t key[kSortIpt], val[kSortIpt], rank[kSortIpt];
        const uint32_t wbase = tile0 + (uint32_t)w * span;
        // every load of the round is issued before the ranking waits on any
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {
            const uint32_t idx = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            const bool valid = r < rounds && idx < end;
            key[r] = valid ? kin[idx] : 0u;
            val[r] = valid ? vin[idx] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {
            if (r >= rounds) break;
            const uint32_t idx = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            const bool valid = idx < end;
            const uint32_t d = ((key[r] - kb) >> shift) & mask;
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
        uint32_t run = 0;   // combine the waves of this round in order, per digit
        if (t < nd) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t c = s_cnt[k][t];
                s_cnt[k][t] = run;
                run += c;
            }
            s_tot[t] = run;
        }
        uint32_t nround;
        const uint32_t loc = block_excl_scan_256(t < nd ? run : 0u, s_wave, nround);
        if (t < nd) s_loc[t] = loc;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortIpt; r++) {   // the round in digit order, in LDS
            if (r >= rounds) break;
            const uint32_t idx = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            if (idx < end) {
                const uint32_t d = ((key[r] - kb) >> shift) & mask;
                const uint32_t lp = s_loc[d] + s_cnt[w][d] + rank[r];
                s_key[lp] = key[r];
                s_val[lp] = val[r];
            }
        }
        __syncthreads();
        for (uint32_t p = (uint32_t)t; p < nround; p += kSortBlock) {
            const uint32_t k = s_key[p];
            const uint32_t d = ((k - kb) >> shift) & mask;
            const uint32_t pos = s_base[d] + (p - s_loc[d]);
            if (ko) ko[pos] = k;
            vo[pos] = s_val[p];
        }
        __syncthreads();
        if (t < nd) s_base[t] += s_tot[t];
        __syncthreads();
    }
}

// ---- 1. scans of the touched-tile counts, depth order, key emission ------------------

// Top level of the two-level scans when there are more blocks than each block
// can sum itself: one workgroup per segment of kSegBlocks block totals scans its
// segment in place (exclusive, coalesced) and writes the segment's totals;
// each block then adds the totals of the segments before its own.
__global__ __launch_bounds__(kSegBlocks) void k_seg_scan(uint32_t *__restrict__ sums,
                                                         uint32_t *__restrict__ act, int nblocks,
                                                         unsigned long long *__restrict__ seg_tot,
                                                         uint32_t *__restrict__ seg_act) {
    __shared__ unsigned long long s_w[kSegBlocks / 64];
    __shared__ uint32_t s_a[kSegBlocks / 64];
    const int i = blockIdx.x * kSegBlocks + threadIdx.x;
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long c = i < nblocks ? sums[i] : 0ull;
    const uint32_t a = act && i < nblocks ? act[i] : 0u;
    unsigned long long ic = c;
    uint32_t ia = a;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(ic, o, 64);
        const uint32_t ya = __shfl_up(ia, o, 64);
        if (lane >= o) {
            ic += y;
            ia += ya;
        }
    }
    if (lane == 63) {
        s_w[w] = ic;
        s_a[w] = ia;
    }
    __syncthreads();
    if (w == 0) {   // the waves' totals
        constexpr int NW = kSegBlocks / 64;
        const unsigned long long x = lane < NW ? s_w[lane] : 0ull;
        const uint32_t y = lane < NW ? s_a[lane] : 0u;
        unsigned long long xi = x;
        uint32_t yi = y;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            const unsigned long long u = __shfl_up(xi, o, 64);
            const uint32_t ua = __shfl_up(yi, o, 64);
            if (lane >= o) {
                xi += u;
                yi += ua;
            }
        }
        if (lane < NW) {
            s_w[lane] = xi - x;
            s_a[lane] = yi - y;
        }
        if (lane == NW - 1) {
            seg_tot[blockIdx.x] = xi;
            if (seg_act) seg_act[blockIdx.x] = yi;
        }
    }
    __syncthreads();
    if (i < nblocks) {
        sums[i] = (uint32_t)min(s_w[w] + ic - c, 0xFFFFFFFFull);
        if (act) act[i] = s_a[w] + ia - a;
    }
}

// The first offsets of scan block `first` (a workgroup's first block of 256
// records) and the totals: with at most kOwnPrefixBlocks blocks each workgroup
// sums the totals of the blocks before it itself; otherwise k_seg_scan has
// scanned each segment in place and the workgroup adds the totals of the
// segments before its own.  With `publish`, block 0
// writes the totals (m_total; m_dev = key total, 0 on overflow with
// GSF_FLAG_CAPACITY; a_dev = active records, 0 on overflow).  Returns false on
// a key overflow.
__device__ __forceinline__ bool block_prefix(const uint32_t *__restrict__ sums,
                                             const uint32_t *__restrict__ act, int nblocks, int first,
                                             const unsigned long long *__restrict__ seg_tot,
                                             const uint32_t *__restrict__ seg_act,
                                             int64_t capacity, uint32_t *m_dev,
                                             unsigned long long *m_total, uint32_t *a_dev,
                                             uint32_t *flags, bool publish,
                                             unsigned long long *s_tot, uint32_t &gbase,
                                             uint32_t &abase) {
    const bool own = nblocks <= kOwnPrefixBlocks;
    const int n = own ? nblocks : (nblocks + kSegBlocks - 1) / kSegBlocks;
    const int mine = own ? first : first / kSegBlocks;
    unsigned long long pre = 0ull, all = 0ull, apre = 0ull, aall = 0ull;
    for (int b = threadIdx.x; b < n; b += kScanBlock) {
        const unsigned long long c = own ? sums[b] : seg_tot[b];
        const unsigned long long a = own ? (act ? act[b] : 0ull) : (seg_act ? seg_act[b] : 0ull);
        all += c;
        aall += a;
        if (b < mine) {
            pre += c;
            apre += a;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        pre += __shfl_xor(pre, o, 64);
        all += __shfl_xor(all, o, 64);
        apre += __shfl_xor(apre, o, 64);
        aall += __shfl_xor(aall, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_tot[threadIdx.x >> 6] = all;
        s_tot[4 + (threadIdx.x >> 6)] = aall;
        s_tot[8 + (threadIdx.x >> 6)] = pre;
        s_tot[12 + (threadIdx.x >> 6)] = apre;
    }
    __syncthreads();
    const unsigned long long total_keys = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
    const unsigned long long total_act = s_tot[4] + s_tot[5] + s_tot[6] + s_tot[7];
    unsigned long long g = s_tot[8] + s_tot[9] + s_tot[10] + s_tot[11];
    unsigned long long ga = s_tot[12] + s_tot[13] + s_tot[14] + s_tot[15];
    if (!own) {   // plus this block's place within its segment
        g += sums[first];
        ga += act ? act[first] : 0u;
    }
    gbase = (uint32_t)min(g, 0xFFFFFFFFull);   // used only when the total fits
    abase = (uint32_t)ga;
    __syncthreads();   // s_tot is free again
    if (publish && blockIdx.x == 0 && threadIdx.x == 0) {
        *m_total = total_keys;
        const bool over = total_keys > (unsigned long long)capacity;
        if (over) atomicOr(flags, GSF_FLAG_CAPACITY);
        *m_dev = over ? 0u : (uint32_t)total_keys;
        if (a_dev) *a_dev = over ? 0u : (uint32_t)total_act;
    }
    return total_keys <= (unsigned long long)capacity;
}

// One record with keys: its compacted entry e (depth key, value, arec) and,
// for a box not packed, its row table at its first gradient slot.
__device__ __forceinline__ void scan_rec_place(uint32_t r, uint32_t c, uint32_t first, uint32_t e,
                                               uint2 rc, uint2 pk, uint32_t dk, const SplatPtrs &sp,
                                               uint2 *__restrict__ rowtab, int n, int tile,
                                               const ViewDesc *__restrict__ views, const FoveaRows &fr,
                                               uint32_t *__restrict__ dkey, uint32_t *__restrict__ dval,
                                               uint4 *__restrict__ arec, const ValPack &vp) {
    dkey[e] = dk;
    dval[e] = vp.pack(e, c);
    arec[2 * e] = make_uint4(r, first, c, pk.x);
    arec[2 * e + 1] = make_uint4(rc.x, rc.y, pk.y, 0u);
    const int x0 = (int)(rc.x & 0xFFFFu), y0 = (int)(rc.x >> 16);
    const int x1 = (int)(rc.y & 0xFFFFu), y1 = (int)(rc.y >> 16);
    if (y1 - y0 + 1 > kPackRows || x1 - x0 + 1 > kPackCols) {   // the row table
        const float4 ea = *sp.at(r, kRecEll), a = *sp.at(r, kRecA),
                     cc = *sp.at(r, kRecC);
        const Ellipse el{ea.x, ea.y, ea.z, ea.w, sqrtf(ea.y / ea.z), a.x, a.y, (int)cc.z, (int)cc.w};
        const int v = (int)r / n;
        const ViewDesc vd = views[v];
        const int tl = 31 - __clz(tile);
        uint32_t j = 0, pre = 0;
        for (int ty = y0; ty <= y1 && j < pk.x; ty++) {
            int c0, c1;
            if (!row_span(el, ty, tl, vd.width, vd.height, x0, x1, c0, c1) ||
                !fovea_rows_clip(fr, v, ty, c0, c1))
                continue;
            rowtab[first + j] = make_uint2((uint32_t)(ty - y0) | ((uint32_t)c0 << 16), pre);
            pre += (uint32_t)(c1 - c0 + 1);
            j++;
        }
    }
}

// Record-order scan of the listed-tile counts: koff[r], the position of record
// r's first gradient slot (its keys in record order), the row tables of the
// boxes not packed (written at those slots), the key total and the capacity
// check; and the records that list a tile, compacted in record order: entry e
// holds (depth bits, e) in (dkey, dval) for the depth sort and, in arec, the
// record's data the emission needs (record id, first slot, count, packed spans
// or row-table size, box) as one 32-byte entry, so that the emission, which
// visits the records in depth order, gathers one cache line per record.
// a_dev: their number (0 on overflow).  Also clears the tile ranges
// (grid-stride).  The per-block totals of counts and of active records come
// from the projection.  A workgroup scans kScanRecRounds consecutive blocks of
// 256 records; their loads are all issued before its prefix is summed, so that
// they are in flight while it waits on the totals (nrec >= 1).
__global__ __launch_bounds__(kScanBlock) void k_scan_rec(
    const uint32_t *__restrict__ count, const uint2 *__restrict__ rect,
    const uint2 *__restrict__ rspan, SplatPtrs sp,
    const uint32_t *__restrict__ depth_key, uint32_t *__restrict__ koff, uint2 *__restrict__ rowtab,
    int nrec, int n, int tile, const ViewDesc *__restrict__ views, FoveaRows fr,
    const uint32_t *__restrict__ block_sums, const uint32_t *__restrict__ block_act, int nblocks,
    const unsigned long long *__restrict__ seg_tot, const uint32_t *__restrict__ seg_act,
    uint32_t *__restrict__ m_dev, unsigned long long *__restrict__ m_total,
    uint32_t *__restrict__ a_dev, uint32_t *__restrict__ flags, int64_t capacity,
    uint32_t *__restrict__ dkey, uint32_t *__restrict__ dval, uint4 *__restrict__ arec,
    uint2 *__restrict__ ranges, int total_tiles, ValPack vp) {
    __shared__ uint32_t s_wave[4];
    __shared__ unsigned long long s_tot[16];
    // kScanRecRounds rounds of 256 consecutive records per workgroup; every
    // record's entries are read first, with no branch (the lines hold records
    // with keys anyway; past the end, the last record's, unused)
    uint32_t c[kScanRecRounds], dk[kScanRecRounds];
    uint2 rc[kScanRecRounds], pk[kScanRecRounds];
#pragma unroll
    for (int k = 0; k < kScanRecRounds; k++) {
        const int r = (blockIdx.x * kScanRecRounds + k) * kScanTile + threadIdx.x;
        const int rl = min(r, nrec - 1);
        c[k] = r < nrec ? count[rl] : 0u;
        rc[k] = rect[rl];
        pk[k] = rspan[rl];
        dk[k] = depth_key[rl];
    }
    for (int t = blockIdx.x * kScanBlock + threadIdx.x; t < total_tiles; t += gridDim.x * kScanBlock)
        ranges[t] = make_uint2(0u, 0u);
    uint32_t gbase, abase;
    if (!block_prefix(block_sums, block_act, nblocks, (int)blockIdx.x * kScanRecRounds, seg_tot, seg_act,
                      capacity, m_dev, m_total, a_dev, flags, true, s_tot, gbase, abase))
        return;   // overflow: nothing placed, nothing to sort
#pragma unroll
    for (int k = 0; k < kScanRecRounds; k++) {
        const int r = (blockIdx.x * kScanRecRounds + k) * kScanTile + threadIdx.x;
        uint32_t total, atot;
        const uint32_t off = block_excl_scan_256(c[k], s_wave, total);
        const uint32_t apos = block_excl_scan_256(c[k] != 0u ? 1u : 0u, s_wave, atot);
        const uint32_t first = gbase + off, e = abase + apos;
        gbase += total;
        abase += atot;
        if (r < nrec) koff[r] = first;   // every record: whole 64-byte chunks are written
        if (c[k] != 0u) scan_rec_place((uint32_t)r, c[k], first, e, rc[k], pk[k], dk[k], sp, rowtab, n,
                                       tile, views, fr, dkey, dval, arec, vp);
    }
}

// Per view, the first tile (column, row) of its fovea box, into LDS (threads
// below nviews), for the compact keys of a fovea-culled forward.
__device__ __forceinline__ void fovea_origins(const TileMap &tm, const ViewDesc *__restrict__ views,
                                              int nviews, int2 *s_f0) {
    const int v = threadIdx.x;
    if (tm.gaze && v < nviews) {
        const ViewDesc vd = views[v];
        const FoveaTiles f = fovea_tiles(tm.gaze, v, tm.radius, vd.width, vd.height, tm.tile);
        s_f0[v] = make_int2(f.tx0, f.ty0);
    }
}

// Global tile id of a sort key (identity without a gaze).
__device__ __forceinline__ uint32_t global_tile(uint32_t c, const TileMap &tm,
                                                const ViewDesc *s_views, const int2 *s_f0) {
    if (!tm.gaze) return c;
    const uint32_t box = (uint32_t)tm.box, area = box * box;
    const uint32_t v = c / area, l = c - v * area, ly = l / box, lx = l - ly * box;
    const ViewDesc vd = s_views[v];
    return (uint32_t)vd.tile_off + ((uint32_t)s_f0[v].y + ly) * (uint32_t)vd.tiles_x +
           (uint32_t)s_f0[v].x + lx;
}

// Per block of 256 depth-ordered active records: the sum of their counts (the
// first level of the emission scan).
__global__ __launch_bounds__(kScanBlock) void k_emit_totals(const uint32_t *__restrict__ dval,
                                                            const uint32_t *__restrict__ a_dev,
                                                            const uint4 *__restrict__ arec,
                                                            uint32_t *__restrict__ sums, ValPack vp) {
    __shared__ uint32_t s_w[4];
    const uint32_t pos = blockIdx.x * kScanTile + threadIdx.x;
    uint32_t c = 0u;
    if (pos < *a_dev) {
        const uint32_t v = dval[pos];
        c = vp.count(v);
        if (c == vp.cmax) c = arec[2 * vp.entry(v)].z;   // saturated: the entry's count
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Keys of the active records in depth order (key = global tile id, value =
// record id): block b emits the keys of depth positions 256 b .. 256 b + 255,
// all its threads together, key q of the block by thread q mod 256, the record
// owning q found by binary search over the block's offsets in LDS (one record's
// many keys spread over the block, consecutive threads writing consecutive
// addresses).  Within a record the keys run over the box rows, each row's tiles
// being those its support ellipse reaches: from the packed spans, or the row
// table at the record's gradient slots.  The stable sort by tile that follows
// then leaves every tile's list in (depth, record) order.
__global__ __launch_bounds__(kScanBlock) void k_emit(
    const uint32_t *__restrict__ dval, const uint32_t *__restrict__ a_dev,
    const uint4 *__restrict__ arec, const uint2 *__restrict__ rowtab, int n,
    const ViewDesc *__restrict__ views, int nviews, const uint32_t *__restrict__ block_sums,
    int nblocks, const unsigned long long *__restrict__ seg_tot,
    const unsigned long long *__restrict__ m_total, int64_t capacity, TileMap tm,
    uint32_t *__restrict__ keys, uint32_t *__restrict__ vals, ValPack vp) {
    __shared__ uint32_t s_wave[4];
    __shared__ unsigned long long s_tot[16];
    __shared__ uint32_t s_off[kScanTile];   // block-local exclusive key offset per record
    __shared__ uint4 s_r0[kScanTile];       // record, first slot, count, spans.x / table size
    __shared__ uint4 s_r1[kScanTile];       // box, spans.y
    __shared__ ViewDesc s_views[kMaxViews];   // read per key: kept in LDS
    __shared__ int2 s_f0[kMaxViews];          // fovea box origins (compact keys)
    const uint32_t A = *a_dev;
    if ((uint32_t)blockIdx.x * kScanTile >= A) return;   // beyond the active records
    // the record's entry first, with no branch (past the end: the last one's,
    // unused), so that its gather is in flight while the block's prefix is summed
    const uint32_t pos = blockIdx.x * kScanTile + threadIdx.x;
    const uint32_t e = vp.entry(dval[min(pos, A - 1u)]);
    uint4 r0 = arec[2 * e], r1 = arec[2 * e + 1];
    if ((int)threadIdx.x < min(nviews, kMaxViews)) s_views[threadIdx.x] = views[threadIdx.x];
    fovea_origins(tm, views, nviews, s_f0);
    uint32_t gbase, abase;
    if (!block_prefix(block_sums, nullptr, nblocks, (int)blockIdx.x, seg_tot, nullptr, capacity, nullptr,
                      const_cast<unsigned long long *>(m_total), nullptr, nullptr, false, s_tot,
                      gbase, abase))
        return;
    if (pos < A) {
        r1.w = r0.x / (uint32_t)n;   // the record's view, once per record
    } else {
        r0 = make_uint4(0u, 0u, 0u, 0u);
        r1 = r0;
    }
    uint32_t total;
    const uint32_t off = block_excl_scan_256(r0.z, s_wave, total);
    s_off[threadIdx.x] = off;
    s_r0[threadIdx.x] = r0;
    s_r1[threadIdx.x] = r1;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < total; q += kScanBlock) {
        // the last record whose offset is <= q (every active record has keys;
        // slots past the active records hold the total): a fixed 8-step search
        int lo = 0;
#pragma unroll
        for (int step = kScanTile / 2; step > 0; step >>= 1)
            lo = s_off[lo + step] <= q ? lo + step : lo;
        uint32_t li = q - s_off[lo];              // index of the key within its record
        const uint4 a = s_r0[lo], b = s_r1[lo];
        const uint32_t rr = a.x;
        const int x0 = (int)(b.x & 0xFFFFu), y0 = (int)(b.x >> 16);
        const int x1 = (int)(b.y & 0xFFFFu), y1 = (int)(b.y >> 16);
        const uint32_t v = b.w;
        uint32_t ty = 0u, tx = 0u;   // the key's tile
        if (y1 - y0 + 1 <= kPackRows && x1 - x0 + 1 <= kPackCols) {   // packed spans
            for (int k = 0; k < kPackRows; k++) {
                const uint32_t f = ((k < 2 ? a.w : b.z) >> (16 * (k & 1))) & 0xFFFFu;
                const uint32_t w = f >> 8;
                if (li < w) {
                    ty = (uint32_t)(y0 + k);
                    tx = (uint32_t)x0 + (f & 0xFFu) + li;
                    break;
                }
                li -= w;
            }
        } else {   // the last row-table entry whose key prefix is <= li holds key li
            const uint32_t tb = a.y;
            int ta = 0, tz = (int)a.w - 1;
            while (ta < tz) {
                const int mid = (ta + tz + 1) >> 1;
                if (rowtab[tb + (uint32_t)mid].y <= li) ta = mid; else tz = mid - 1;
            }
            const uint2 te = rowtab[tb + (uint32_t)ta];
            ty = (uint32_t)y0 + (te.x & 0xFFFFu);
            tx = (te.x >> 16) + (li - te.y);
        }
        const ViewDesc vd = s_views[v];
        keys[gbase + q] = tm.gaze ? v * (uint32_t)(tm.box * tm.box) +
                                        (ty - (uint32_t)s_f0[v].y) * (uint32_t)tm.box +
                                        (tx - (uint32_t)s_f0[v].x)
                                  : (uint32_t)vd.tile_off + ty * (uint32_t)vd.tiles_x + tx;
        vals[gbase + q] = rr;
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

// Each thread takes kBoundKeys consecutive sorted keys (16-byte loads) and the
// keys on either side: a key opens its tile's range where it differs from the
// key before and closes it where it differs from the key after.  Only those
// keys (one in several hundred on large plans) map the key to its tile, write
// the range and fill the empty tiles since the previous tile with (k, k).
constexpr int kBoundKeys = 8;

__global__ __launch_bounds__(256) void k_tile_bounds(const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ m_dev,
                                                     uint32_t m_host, int total_tiles,
                                                     const ViewDesc *__restrict__ views, int nviews,
                                                     TileMap tm, uint2 *__restrict__ ranges) {
    __shared__ ViewDesc s_views[kMaxViews];
    __shared__ int2 s_f0[kMaxViews];
    if (tm.gaze) {
        if ((int)threadIdx.x < min(nviews, kMaxViews)) s_views[threadIdx.x] = views[threadIdx.x];
        fovea_origins(tm, views, nviews, s_f0);
        __syncthreads();
    }
    const uint32_t m = m_dev ? *m_dev : m_host;
    const uint32_t stride = gridDim.x * blockDim.x * kBoundKeys;
    // wave-uniform trip count: every lane takes part in the run fills
    for (uint32_t b0 = blockIdx.x * blockDim.x * kBoundKeys; b0 < m; b0 += stride) {
        const uint32_t k0 = b0 + threadIdx.x * kBoundKeys;
        uint32_t c[kBoundKeys + 2];   // c[0]: the key before k0; c[j + 1]: key k0 + j
        if (k0 + kBoundKeys <= m) {
            const uint4 u0 = *reinterpret_cast<const uint4 *>(keys + k0);
            const uint4 u1 = *reinterpret_cast<const uint4 *>(keys + k0 + 4);
            c[1] = u0.x; c[2] = u0.y; c[3] = u0.z; c[4] = u0.w;
            c[5] = u1.x; c[6] = u1.y; c[7] = u1.z; c[8] = u1.w;
        } else {
#pragma unroll
            for (int j = 0; j < kBoundKeys; j++) c[j + 1] = k0 + j < m ? keys[k0 + j] : 0u;
        }
        c[0] = k0 > 0 && k0 <= m ? keys[k0 - 1] : 0u;
        c[kBoundKeys + 1] = k0 + kBoundKeys < m ? keys[k0 + kBoundKeys] : 0u;
#pragma unroll
        for (int j = 0; j < kBoundKeys; j++) {
            const uint32_t k = k0 + (uint32_t)j;
            uint32_t lo = 0, hi = 0, lo2 = 0, hi2 = 0;
            if (k < m) {
                const bool first = k == 0 || c[j] != c[j + 1];
                const bool last = k + 1 == m || c[j + 2] != c[j + 1];
                if (first || last) {
                    const uint32_t t = global_tile(c[j + 1], tm, s_views, s_f0);
                    if (first) {
                        // empty tiles before t
                        lo = k == 0 ? t : global_tile(c[j], tm, s_views, s_f0) + 1u;
                        hi = t;
                        ranges[t].x = k;
                    }
                    if (k + 1 == m) {
                        ranges[t].y = m;
                        lo2 = t + 1u;                         // empty tiles after the last key
                        hi2 = (uint32_t)total_tiles;
                    } else if (last) {
                        ranges[t].y = k + 1;
                    }
                }
            }
            fill_runs(ranges, lo, hi, k);
            fill_runs(ranges, lo2, hi2, m);
        }
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
constexpr int kOrderTiles = 1024;

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
    constexpr int kStrips = 7;   // 33 classes x 7 strips of the workgroups <= 256 threads
    __shared__ uint32_t s_tot[33], s_cnt[33], s_part[2][kStrips][33];
    const int c = threadIdx.x;
    {   // the class totals over all workgroups and over those before this
        // one: thread (class, strip) sums every kStrips-th row, then the
        // strips are added (no atomics, which the compiler would serialise
        // over the lanes)
        const int cls = (int)threadIdx.x % 33, strip = (int)threadIdx.x / 33;
        if (strip < kStrips) {
            uint32_t tot = 0u, bef = 0u;
#pragma unroll 4
            for (int w = strip; w < groups; w += kStrips) {
                const uint32_t n = counts[(size_t)w * 33 + cls];
                tot += n;
                bef += w < (int)blockIdx.x ? n : 0u;
            }
            s_part[0][strip][cls] = tot;
            s_part[1][strip][cls] = bef;
        }
    }
    __syncthreads();
    if (c < 33) {
        uint32_t tot = 0u, bef = 0u;
#pragma unroll
        for (int k = 0; k < kStrips; k++) {
            tot += s_part[0][k][c];
            bef += s_part[1][k][c];
        }
        s_tot[c] = tot;
        s_cnt[c] = bef;
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

}  // namespace

int radix_grid_for(int64_t capacity) {
    int64_t g = (capacity + kSortTile - 1) / kSortTile;
    if (g < 1) g = 1;
    if (g > kSortMaxGrid) g = kSortMaxGrid;
    return (int)g;
}

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + kMaxDigit - 1) / kMaxDigit; }

namespace {

// One pass: histogram, digit scan (more than kLocalScanGrid workgroups) and
// scatter.
void radix_pass(hipStream_t s, const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                uint32_t *vout, const uint32_t *n_dev, uint32_t n_host, int shift, int bits, int grid,
                uint32_t *hist, uint32_t *digit_tot, const RadixCtl &ctl) {
    k_radix_hist<<<grid, kSortBlock, 0, s>>>(kin, n_dev, n_host, shift, bits, hist, grid, ctl);
    // up to kLocalScanGrid workgroups sum their digit offsets themselves
    const bool local = grid <= kLocalScanGrid;
    if (!local) k_radix_colscan<<<1 << bits, 256, 0, s>>>(hist, grid, digit_tot, ctl.skip);
    k_radix_scatter<<<grid, kSortBlock, 0, s>>>(kin, vin, kout, vout, n_dev, n_host, shift, bits, hist,
                                                local ? nullptr : digit_tot, grid, ctl);
}

}  // namespace

void launch_depth_sort(hipStream_t s, uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                       const uint32_t *n_dev, int grid, uint32_t *hist, uint32_t *digit_tot,
                       uint32_t *mm, uint32_t *ctl, uint32_t *vfinal) {
    // pass 1 sorts by the low 8 bits, which the base (low 8 bits clear) leaves
    // as they are, and finds the base and whether 24 bits above it hold every key
    RadixCtl c1;
    c1.mm = mm;
    c1.ctl = ctl;
    radix_pass(s, k0, v0, k1, v1, n_dev, 0u, 0, 8, grid, hist, digit_tot, c1);
    RadixCtl c2;
    c2.base = ctl;
    radix_pass(s, k1, v1, k0, v0, n_dev, 0u, 8, 8, grid, hist, digit_tot, c2);
    RadixCtl c3 = c2;   // the last pass when 24 bits hold the keys
    c3.last = ctl + 1;
    c3.vlast = vfinal;
    radix_pass(s, k0, v0, k1, v1, n_dev, 0u, 16, 8, grid, hist, digit_tot, c3);
    RadixCtl c4 = c2;   // otherwise bits 24 - 30
    c4.skip = ctl + 1;
    radix_pass(s, k1, v1, nullptr, vfinal, n_dev, 0u, 24, 7, grid, hist, digit_tot, c4);
}

int launch_radix_sort(hipStream_t s, const uint32_t *kin, const uint32_t *vin, uint32_t *ka,
                      uint32_t *va, uint32_t *kb, uint32_t *vb, const uint32_t *n_dev,
                      uint32_t n_host, int bits, int grid, uint32_t *hist, uint32_t *digit_tot) {
    int where = 0;
    const uint32_t *ks = kin, *vs = vin;
    const int passes = radix_passes(bits);
    // balanced digits: `passes` digits of at most kMaxDigit bits covering `bits`
    for (int p = 0, shift = 0; p < passes; p++) {
        const int b = (bits - shift + (passes - p) - 1) / (passes - p);
        uint32_t *kd = where == 1 ? kb : ka, *vd = where == 1 ? vb : va;
        radix_pass(s, ks, vs, kd, vd, n_dev, n_host, shift, b, grid, hist, digit_tot, RadixCtl{});
        where = where == 1 ? 2 : 1;
        ks = kd;
        vs = vd;
        shift += b;
    }
    return where;
}

int scan_blocks(int64_t nrec) { return (int)((nrec + kScanTile - 1) / kScanTile) + 1; }


int seg_count(int64_t nrec) {
    const int64_t nb = (nrec + kScanTile - 1) / kScanTile;
    return (int)((nb + kSegBlocks - 1) / kSegBlocks) + 1;
}

void launch_scan_records(hipStream_t s, const uint32_t *count, const uint2 *rect,
                         const uint2 *rspan, SplatPtrs sp, const uint32_t *depth_key, uint32_t *koff,
                         uint2 *rowtab, int nrec, int n, int tile, const ViewDesc *views,
                         const FoveaRows &fr, uint32_t *block_sums, uint32_t *block_act,
                         unsigned long long *seg_tot, uint32_t *seg_act, uint32_t *m_dev, unsigned long long *m_total,
                         uint32_t *a_dev, uint32_t *flags, int64_t capacity, uint32_t *dkey,
                         uint32_t *dval, uint4 *arec, uint2 *ranges, int total_tiles) {
    const int nb = (nrec + kScanTile - 1) / kScanTile;
    if (nb > kOwnPrefixBlocks)
        k_seg_scan<<<(nb + kSegBlocks - 1) / kSegBlocks, kSegBlocks, 0, s>>>(block_sums, block_act, nb,
                                                                            seg_tot, seg_act);
    k_scan_rec<<<(nb + kScanRecRounds - 1) / kScanRecRounds, kScanBlock, 0, s>>>(
        count, rect, rspan, sp, depth_key, koff, rowtab, nrec, n, tile, views, fr, block_sums,
        block_act, nb, seg_tot, seg_act, m_dev, m_total, a_dev, flags, capacity, dkey, dval, arec,
        ranges, total_tiles, ValPack(entry_bits(nrec)));
}

void launch_emit(hipStream_t s, const uint32_t *dval, const uint32_t *a_dev, const uint4 *arec,
                 const uint2 *rowtab, int nrec, int n, const ViewDesc *views, int nviews,
                 uint32_t *block_sums, unsigned long long *seg_tot, const unsigned long long *m_total,
                 int64_t capacity, const TileMap &tm, uint32_t *keys, uint32_t *vals) {
    const int nb = (nrec + kScanTile - 1) / kScanTile;
    const ValPack vp(entry_bits(nrec));   // as launch_scan_records packed them
    k_emit_totals<<<nb, kScanBlock, 0, s>>>(dval, a_dev, arec, block_sums, vp);
    if (nb > kOwnPrefixBlocks)
        k_seg_scan<<<(nb + kSegBlocks - 1) / kSegBlocks, kSegBlocks, 0, s>>>(block_sums, nullptr, nb,
                                                                            seg_tot, nullptr);
    k_emit<<<nb, kScanBlock, 0, s>>>(dval, a_dev, arec, rowtab, n, views, nviews, block_sums, nb,
                                     seg_tot, m_total, capacity, tm, keys, vals, vp);
}

void launch_tile_bounds(hipStream_t s, const uint32_t *keys, const uint32_t *m_dev, uint32_t m_host,
                        int64_t capacity, int total_tiles, const ViewDesc *views, int nviews,
                        const TileMap &tm, uint2 *ranges) {
    int64_t g = (capacity + 256 * kBoundKeys - 1) / (256 * kBoundKeys);
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    k_tile_bounds<<<(int)g, 256, 0, s>>>(keys, m_dev, m_host, total_tiles, views, nviews, tm, ranges);
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


}  // namespace gsf
