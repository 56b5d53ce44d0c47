// gs_internal.h - internal types, constants and launchers of the gfx950 fit path.
// Not part of the ABI (see include/gsfit.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsfit.h"

namespace gsf {

// Compositing constants of the 3DGS forward model the paper builds on (Related
// Work "Novel View Synthesis"; Method "Periphery Model Training").
constexpr float kAlphaMin = 1.0f / 255.0f;   // contributions below are skipped
constexpr float kAlphaMax = 0.99f;           // alpha clamp
constexpr float kTStop = 1e-4f;              // stop before T would fall below this
constexpr float kLowPass = 0.3f;             // px^2 added to the 2D covariance diagonal
constexpr float kJClamp = 1.3f;              // Jacobian evaluated at x/z within 1.3 tan(fov/2)
constexpr float kBoxRel = 1e-4f;             // support-box padding, relative
constexpr float kBoxAbs = 1.0f / 64.0f;      // support-box padding, pixels

constexpr int kMaxViews = 64;
constexpr int kMaxSeg = 16;

// Per-view launch descriptor (device copy made at plan creation).
struct ViewDesc {
    int32_t tile_off;   // first global tile id of the view
    int32_t tiles_x;
    int32_t tiles_y;
    int32_t pix_off;    // first global pixel of the view (images are concatenated)
    int32_t width;
    int32_t height;
    int32_t pad0, pad1;
};

// Per-record screen-space splat, three 16-byte loads per gather:
//   a = (hx, hy, A2, B2), b = (C2, opacity, red, green), c = (blue, h, ix, iy),
// h being the padded half height in pixel rows of the support box (the region
// where o e^power >= 1/255 can hold).
// The pixel mean mu' is computed in double precision and split into an integer
// pixel (ix, iy; exact floats) and the offset of mu' from that pixel's centre,
// hx = ix + 1/2 - mu'_x (likewise hy), so that the offset of pixel (x, y) from
// the mean, dx = (x - ix) + hx, is exact up to one float32 rounding of the
// result: the gradient with respect to the mean sums +dx and -dx terms from
// both sides of a small footprint, and float32 rounding of mu' itself (about
// 3e-5 px at 1000 px) would otherwise dominate it.  The conic is stored
// pre-scaled so that power2 = A2 dx^2 + C2 dy^2 + B2 dx dy = log2(e) * power,
// i.e. A2 = -log2(e) A / 2, B2 = -log2(e) B, C2 = -log2(e) C / 2; the
// compositing kernels compare power2 with tau = log2(1 / (255 opacity)), below
// which alpha < 1/255.
// The splat of a record (record = Gaussian x view) as one 64-byte aligned
// chunk, the four float4 that staging a key reads: a, b, c and the support
// ellipse.  A key's staging gathers one chunk instead of a piece of four
// arrays; the projection writes each chunk whole (a partial 64-byte chunk
// would cost the memory a read-modify-write).
constexpr int kRecF4 = 4;
constexpr int kRecA = 0, kRecB = 1, kRecC = 2, kRecEll = 3;
struct SplatPtrs {
    float4 *rec;   // [records][kRecF4]
    __host__ __device__ float4 *at(uint32_t r, int slot) const {
        return rec + (size_t)r * kRecF4 + slot;
    }
};
constexpr float kLog2e = 1.4426950408889634f;

struct SegTable {
    int64_t off[kMaxSeg + 1];
    float lr[kMaxSeg];
    int32_t n;
};

// Learning rate per parameter plane (11 + 3 * 16 planes at SH degree 3).
constexpr int kMaxPlanes = 64;
struct PlaneLr {
    float lr[kMaxPlanes];
};

// Support ellipse of a record for the tile lists, as the constants of its
// row-wise x extent: for a row offset d from the mean the ellipse (quadratic
// form <= Kp = 2 ln(255 o) (1 + kBoxRel)^2, covariance Sigma' = [sa sb; sb sc])
// spans x in slope d +- sqrt(kw - ws d^2), with slope = sb / sc,
// kw = Kp (sa - sb^2 / sc), ws = (sa - sb^2 / sc) / sc; its rightmost point
// lies at row offset dyr = sb sqrt(Kp / sa) and its rows within +-ey,
// ey = sqrt(Kp sc).  Plus the split-form mean (integer pixel ix, iy; offsets
// hxo, hyo of that pixel's centre from the mean).
// Number of set bits of a wave mask below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

struct Ellipse {
    float slope, kw, ws, dyr, ey;
    float hxo, hyo;
    int ix, iy;
};
__device__ __forceinline__ float4 ellipse_pack(float sa, float sb, float sc, float Kp, float &ey) {
    const float slope = sb / sc, wid = sa - sb * (sb / sc);
    ey = sqrtf(Kp * sc);
    return make_float4(slope, Kp * wid, wid / sc, sb * sqrtf(Kp / sa));
}
// Every box lists, in each of its tile rows, only the tiles its padded
// support ellipse reaches (row_span).  Boxes of at most kPackRows tile rows
// and kPackCols tile columns carry their row spans packed (per row: first
// column - x0 in the low byte, tile count in the high byte of a 16-bit field),
// so the duplicate pass needs no arithmetic.  Every other box gets a row table
// at its own key positions: the duplicate pass writes, for the j-th row that
// lists a tile, entry koff[r] + j = (row - y0 | first column << 16, keys of the
// rows before it).  A listed row holds at least one key, so the entries fit in
// the record's count[r] key slots; rspan[r].x holds the entry count.
constexpr int kPackRows = 4;
constexpr int kPackCols = 255;

// Tile columns [c0, c1] of tile row ty that the padded support ellipse
// reaches (false: none).  Over the row's band of pixel centres (rows ty T ..
// min(ty T + T, H) - 1) the ellipse's x extent is taken where its boundary is
// right- (left-)most within the band, widened by kBoxAbs; the pixel columns
// whose centres lie in it, clamped to the image width W and to the box's tile
// columns [x0, x1], give the tiles.  Every pixel with alpha >= 1/255 lies in
// such a tile.
// tile = 1 << tile_log2.  The square roots are the hardware's (within an ulp):
// the same code counts the tiles in the projection and emits them in the
// duplicate pass, so both agree exactly.
// Pixel columns [a, b] (not clamped to the image) whose centres lie in the
// padded ellipse's x extent over the band of pixel rows ja..jb.
__device__ __forceinline__ void ellipse_cols(const Ellipse &e, int ja, int jb, int &a, int &b) {
    const float ya = (float)(ja - e.iy) + e.hyo, yb = (float)(jb - e.iy) + e.hyo;
    float lo = fmaxf(ya, -e.ey), hi = fminf(yb, e.ey);
    if (lo > hi) lo = hi = ya > e.ey ? e.ey : -e.ey;   // band beside the ellipse: its tip
    const float d1 = fminf(fmaxf(e.dyr, lo), hi), d2 = fminf(fmaxf(-e.dyr, lo), hi);
    const float xr = e.slope * d1 + __builtin_amdgcn_sqrtf(fmaxf(e.kw - e.ws * (d1 * d1), 0.f)) + kBoxAbs;
    const float xl = e.slope * d2 - __builtin_amdgcn_sqrtf(fmaxf(e.kw - e.ws * (d2 * d2), 0.f)) - kBoxAbs;
    a = e.ix + (int)ceilf(xl - e.hxo);
    b = e.ix + (int)floorf(xr - e.hxo);
}

__device__ __forceinline__ bool row_span(const Ellipse &e, int ty, int tile_log2, int W, int H,
                                         int x0, int x1, int &c0, int &c1) {
    const int ja = ty << tile_log2, jb = min((ty + 1) << tile_log2, H) - 1;
    int a, b;
    ellipse_cols(e, ja, jb, a, b);
    a = max(a, 0);
    b = min(b, W - 1);
    if (a > b) return false;
    c0 = max(a >> tile_log2, x0);
    c1 = min(b >> tile_log2, x1);
    return c0 <= c1;
}

// The compositing kernels of 16-pixel tiles give each wave one 8 x 8 quadrant
// (q = 0..3: column half q & 1, row half q >> 1) and skip the splats whose
// padded ellipse reaches no pixel centre of it: bit q of the mask is set when
// the ellipse's x extent over the quadrant's rows meets its columns.  The same
// bound as the tile lists, so every pixel with alpha >= 1/255 lies in a
// quadrant whose bit is set.  (x0, y0): the tile's first pixel.
__device__ __forceinline__ bool quad_meets(const Ellipse &e, int xa, int ya) {
    int a, b;
    ellipse_cols(e, ya, ya + 7, a, b);
    return max(a, xa) <= min(b, xa + 7);
}
__device__ __forceinline__ uint32_t quadrant_mask(const Ellipse &e, int x0, int y0) {
    uint32_t m = 0u;
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (quad_meets(e, x0 + (q & 1) * 8, y0 + (q >> 1) * 8)) m |= 1u << q;
    return m;
}

// Where the adjoint puts each key's screen-space gradient: the duplicate pass
// writes a record's count[r] keys at consecutive positions (its first at
// koff[r]), box rows top to bottom and each row's listed tiles left to right;
// the adjoint writes key (r, tile) at that position of pg, one 64-byte chunk
// per key (fields 0-3, 4-7, then 8 and seven zeros, plain stores of the whole
// chunk: a key's slots are written by different workgroups at different times,
// and a partial chunk would cost the memory a read-modify-write), and one pass
// per record sums its positions into g2d.  After a key overflow
// (m_total > capacity) nothing was listed and g2d is zero.
constexpr int kKeyGradF4 = 4;
struct KeyPlace {
    const uint32_t *koff = nullptr, *count = nullptr;
    const uint2 *rect = nullptr, *rspan = nullptr;
    const uint2 *rowtab = nullptr;              // row tables of the boxes not packed
    float4 *pg = nullptr;                       // [capacity][kKeyGradF4]
    const unsigned long long *m_total = nullptr;
    int64_t capacity = 0;
};

// Position of the key of record r in tile (ty, tx) of its view: koff[r] plus
// the tile's rank among the record's listed tiles, from the packed row spans
// or (other boxes) the row table entry of row ty, found by binary search.
__device__ __forceinline__ uint32_t key_slot(const KeyPlace &kp, uint32_t r, int ty, int tx) {
    const uint2 rc = kp.rect[r], pk = kp.rspan[r];
    const int x0 = (int)(rc.x & 0xFFFFu), y0 = (int)(rc.x >> 16);
    const int x1 = (int)(rc.y & 0xFFFFu), y1 = (int)(rc.y >> 16);
    const int rows = y1 - y0 + 1, cols = x1 - x0 + 1;
    const uint32_t base = kp.koff[r];
    uint32_t rank = 0;
    if (rows <= kPackRows && cols <= kPackCols) {
        const int kr = ty - y0;
        for (int k = 0; k < kr; k++) rank += (((k < 2 ? pk.x : pk.y) >> (16 * (k & 1))) >> 8) & 0xFFu;
        const uint32_t f = ((kr < 2 ? pk.x : pk.y) >> (16 * (kr & 1))) & 0xFFFFu;
        rank += (uint32_t)(tx - x0) - (f & 0xFFu);
    } else {
        const uint32_t row = (uint32_t)(ty - y0);
        int lo = 0, hi = (int)pk.x - 1;   // the last entry of a row <= ty (it is row ty: listed)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((kp.rowtab[base + (uint32_t)mid].x & 0xFFFFu) <= row) lo = mid; else hi = mid - 1;
        }
        const uint2 e = kp.rowtab[base + (uint32_t)lo];
        rank = e.y + (uint32_t)tx - (e.x >> 16);
    }
    return base + rank;
}

// ---- wave-level helpers shared by the adjoint passes ------------------------------

// Value of x from the lane the DPP control names (zero where it names none or
// the row is masked off).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                                 ROW_MASK, 0xf, true));
}

// OR over the wave's lanes (DPP row prefix, then the rows folded together).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_shift_u(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, true);
}
__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
    x |= dpp_shift_u<0x111, 0xf>(x);   // row_shr:1
    x |= dpp_shift_u<0x112, 0xf>(x);   // row_shr:2
    x |= dpp_shift_u<0x114, 0xf>(x);   // row_shr:4
    x |= dpp_shift_u<0x118, 0xf>(x);   // row_shr:8
    x |= dpp_shift_u<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x |= dpp_shift_u<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// True when bits a..l (0 <= a <= l <= 63) of the mask are all clear.
__device__ __forceinline__ bool bits_clear(uint64_t m, int a, int l) {
    return ((m << (63 - l)) >> (63 - l + a)) == 0ull;
}

// One step of the segmented inclusive scan: add the value the DPP control
// brings (zero where it brings none) unless a segment starts between.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_step(float (&v)[9], bool join) {
#pragma unroll
    for (int f = 0; f < 9; f++) {
        const float t = dpp_shift<CTRL, ROW_MASK>(v[f]);
        v[f] = join ? v[f] + t : v[f];
    }
}

// Sum of the per-key screen-space gradients of each lane's record r (valid
// lanes; all 64 lanes of the wave take part): record r's keys sit at
// koff[r] .. koff[r] + count[r] - 1, so the records of consecutive lanes own
// one run of consecutive keys.  The wave reads that run 64 keys a step
// (coalesced), sums each record's part of the step with a segmented scan
// across the lanes, and the record's lane takes its part from the part's last
// lane.  After a key overflow nothing was listed and the sums are zero.
__device__ __forceinline__ void wave_key_sum(const KeyPlace &kp, uint32_t r, bool valid, float (&S)[9]) {
    const int lane = __lane_id();
    const bool over = *kp.m_total > (unsigned long long)kp.capacity;
    uint32_t cnt = 0u, base = 0u;
    if (valid && !over) {
        cnt = kp.count[r];
        if (cnt != 0u) base = kp.koff[r];
    }
    // wave-local key range [beg, end) of each lane's record
    uint32_t end = cnt;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const uint32_t t = __shfl_up(end, m, 64);
        if (lane >= m) end += t;
    }
    const uint32_t beg = end - cnt;
    const uint32_t K = __shfl(end, 63, 64);
    const uint64_t nz = __ballot(cnt != 0u);
    const uint32_t start = nz ? __shfl(base, __builtin_ctzll(nz), 64) : 0u;   // the run's first key
#pragma unroll
    for (int f = 0; f < 9; f++) S[f] = 0.f;
    // the next step's keys are loaded while this step is scanned
    float4 na = make_float4(0.f, 0.f, 0.f, 0.f), nb = na;
    float nc = 0.f;
    if ((uint32_t)lane < K) {
        const float4 *g = kp.pg + (size_t)(start + lane) * kKeyGradF4;
        na = g[0];
        nb = g[1];
        nc = g[2].x;
    }
    for (uint32_t c0 = 0; c0 < K; c0 += 64u) {   // wave-uniform
        float v[9] = {na.x, na.y, na.z, na.w, nb.x, nb.y, nb.z, nb.w, nc};
        const uint32_t pn = c0 + 64u + (uint32_t)lane;
        if (pn < K) {
            const float4 *g = kp.pg + (size_t)(start + pn) * kKeyGradF4;
            na = g[0];
            nb = g[1];
            nc = g[2].x;
        } else {
            na = nb = make_float4(0.f, 0.f, 0.f, 0.f);
            nc = 0.f;
        }
        // segment starts in this step: lane 0 and each record's first key
        const bool starts = cnt != 0u && beg >= c0 && beg < c0 + 64u;
        const uint32_t bit = starts ? beg - c0 : 64u;
        const uint64_t heads = 1ull | ((uint64_t)wave_or(bit < 32u ? 1u << bit : 0u)) |
                               ((uint64_t)wave_or(bit >= 32u && bit < 64u ? 1u << (bit - 32u) : 0u) << 32);
        // within rows of 16 lanes, then rows 0 -> 1 and 2 -> 3, then rows 0-1 -> 2-3
        seg_step<0x111, 0xf>(v, lane >= 1 && bits_clear(heads, lane, lane));
        seg_step<0x112, 0xf>(v, lane >= 2 && bits_clear(heads, lane - 1, lane));
        seg_step<0x114, 0xf>(v, lane >= 4 && bits_clear(heads, lane - 3, lane));
        seg_step<0x118, 0xf>(v, lane >= 8 && bits_clear(heads, lane - 7, lane));
        seg_step<0x142, 0xa>(v, lane >= 16 && bits_clear(heads, lane & ~15, lane));
        seg_step<0x143, 0xc>(v, lane >= 32 && bits_clear(heads, 32, lane));
        // each record adds its part of the step, held by the part's last lane
        const bool mine = cnt != 0u && beg < c0 + 64u && end > c0;
        const int src = mine ? (int)(min(end, c0 + 64u) - 1u - c0) : lane;
#pragma unroll
        for (int f = 0; f < 9; f++) {
            const float t = __shfl(v[f], src, 64);
            S[f] = mine ? S[f] + t : S[f];
        }
    }
}

// Tiles [tx0, tx1] x [ty0, ty1] of a view that meet its fovea: the pixels whose
// centre can lie within radius_frac * width of the gaze point, with one pixel of
// slack (the mask test itself is done per pixel by the loss).  Empty when
// tx0 > tx1.
struct FoveaTiles {
    int tx0, tx1, ty0, ty1;
};

__host__ __device__ __forceinline__ FoveaTiles fovea_tiles(const float *__restrict__ gaze, int v,
                                                  float radius_frac, int width, int height, int tile) {
    const float r = radius_frac * (float)width;
    const float gx = gaze[2 * v], gy = gaze[2 * v + 1];
    const float x0 = fmaxf(floorf(gx - r - 0.5f) - 1.f, 0.f);
    const float x1 = fminf(ceilf(gx + r - 0.5f) + 1.f, (float)(width - 1));
    const float y0 = fmaxf(floorf(gy - r - 0.5f) - 1.f, 0.f);
    const float y1 = fminf(ceilf(gy + r - 0.5f) + 1.f, (float)(height - 1));
    FoveaTiles f{1, 0, 1, 0};
    const int tl = __builtin_ctz((unsigned)tile);   // tile: a power of two; x0, y0 >= 0
    if (x0 <= x1 && y0 <= y1) f = FoveaTiles{(int)x0 >> tl, (int)x1 >> tl, (int)y0 >> tl, (int)y1 >> tl};
    return f;
}

// Tile (tx, ty) of a view may hold a pixel of the fovea disk: the nearest point
// of its rectangle of pixel centres lies within radius_frac * width + 1 of the
// gaze point.  The pixel of slack covers the rounding of the per-pixel FP32
// test (the loss's mask), so no tile holding a masked-in pixel is left out; a
// fovea-culled step composites only these tiles of the fovea box (the box's
// corners lie outside the disk).
__host__ __device__ __forceinline__ bool fovea_tile_live(const float *__restrict__ gaze, int v,
                                                        float radius_frac, int width, int height,
                                                        int tile, int tx, int ty) {
    const float r = radius_frac * (float)width + 1.f;
    const float gx = gaze[2 * v], gy = gaze[2 * v + 1];
    const float x0 = (float)(tx * tile) + 0.5f, x1 = (float)min((tx + 1) * tile, width) - 0.5f;
    const float y0 = (float)(ty * tile) + 0.5f, y1 = (float)min((ty + 1) * tile, height) - 0.5f;
    const float dx = fmaxf(fmaxf(x0 - gx, gx - x1), 0.f);
    const float dy = fmaxf(fmaxf(y0 - gy, gy - y1), 0.f);
    return dx * dx + dy * dy <= r * r;
}

// Tile columns [c0, c1] of tile row ty clipped to the tiles that can hold a
// pixel of the fovea disk (false: none remain).  Along a row those tiles form
// one interval (the distance test is monotone in the column on either side of
// the gaze point), so the ends move inwards until they pass it.
__host__ __device__ __forceinline__ bool fovea_row_clip(const float *__restrict__ gaze, int v,
                                                       float radius_frac, int width, int height,
                                                       int tile, int ty, int &c0, int &c1) {
    while (c0 <= c1 && !fovea_tile_live(gaze, v, radius_frac, width, height, tile, c0, ty)) c0++;
    while (c1 >= c0 && !fovea_tile_live(gaze, v, radius_frac, width, height, tile, c1, ty)) c1--;
    return c0 <= c1;
}

// Per view and tile row, the tile columns [lo, hi] that can hold a pixel of the
// fovea disk (lo > hi: none), the clip of every record's row spans in a
// fovea-culled step: entry v * rows + ty.  rows = null: no culling.
struct FoveaRows {
    const uint2 *rows = nullptr;
    int per_view = 0;
};
// Clip tile columns [c0, c1] of view v's tile row ty to the disk's (false: none
// remain).  Without culling, unchanged.
__device__ __forceinline__ bool fovea_rows_clip(const FoveaRows &fr, int v, int ty, int &c0, int &c1) {
    if (!fr.rows) return c0 <= c1;
    const uint2 lr = fr.rows[v * fr.per_view + ty];
    c0 = max(c0, (int)lr.x);
    c1 = min(c1, (int)lr.y);
    return c0 <= c1;
}

// Sort keys of a fovea-culled forward: only the tiles of each view's fovea box
// receive keys, so the key is the tile's place in a compact space instead of
// its global id - view v's box of box x box tiles (from its first fovea tile)
// at v box^2, row-major.  The map is increasing in the global id, so sorting
// by it sorts by tile; the tile ranges are written at the global ids.
struct TileMap {
    const float *gaze = nullptr;   // null: keys are global tile ids
    float radius = 0.f;            // fovea radius as a fraction of the width
    int box = 0;                   // tiles per side of the compact box
    int tile = 16;
};

// ---- launchers (all asynchronous on `s`) -----------------------------------------

// Projection of n Gaussians into V views: records r = v*n + i.  Writes the
// splat and the ellipse constants (slope, kw, ws, dyr; ey follows as
// sqrt(kw / ws)) into the record (kRecA-kRecEll), the depth key (float32 bits
// of the camera depth, 0xFFFFFFFF when culled), the tile rectangle of the
// support box, the number of its tiles the support ellipse reaches (row_span)
// and the packed row spans of short boxes (other boxes: the number of their
// rows that list a tile).
// With cull_gaze (nullable) the rectangle is clipped to the view's
// fovea tiles (fovea_tiles with cull_radius) and each row's span to the tiles
// that can hold a pixel of the disk (fr, which launch_fovea_rows must have
// written for the same gaze and radius).  block_sums[b] / block_act[b]
// receive the total count / the number of records with a nonzero count among
// records 256 b .. 256 b + 255 (scan_blocks(nrec) words each), the input of
// launch_scan_records.
void launch_project_fwd(hipStream_t s, const float *P, int n, int nviews, int deg,
                        const gsf_camera *cams, const ViewDesc *views, int tile, SplatPtrs sp,
                        uint32_t *depth_key, uint2 *rect, uint32_t *count, uint2 *rspan,
                        const float *cull_gaze, float cull_radius, const FoveaRows &fr,
                        uint32_t *block_sums, uint32_t *block_act);
// The row table of fovea culling: fr.rows[v * fr.per_view + ty] for every view
// and tile row up to fr.per_view (rows past a view's last: none).
void launch_fovea_rows(hipStream_t s, const float *gaze, float radius_frac, const ViewDesc *views,
                       int nviews, int tile, const FoveaRows &fr);

// Parameter gradient from the per-key screen-space gradients the compositing
// adjoint left in kp: for SH degrees 0-1 summed per record (wave_key_sum) on
// the way; for degrees 2-3, whose larger state leaves no registers for the
// sum, read from g2d, which launch_grad_sum must have written.
bool project_bwd_sums_keys(int deg);
// accumulate: grads += the gradient (else grads = it).
void launch_project_bwd(hipStream_t s, const float *P, int n, int nviews, int deg,
                        const gsf_camera *cams, const KeyPlace &kp, const float *g2d, float *grads,
                        bool accumulate = false);

// Record-order exclusive scan of the per-record tile counts: koff[r] (record
// r's gradient slots, its keys in record order), the row tables of the boxes
// not packed (rowtab, key capacity entries, at those slots), the key total to
// m_total and (0 on overflow, with GSF_FLAG_CAPACITY) to m_dev; the records with
// keys compacted in record order: entry e = (dkey = depth bits, dval = e) and
// arec[2e], arec[2e + 1] = (record, first slot, count, spans.x or row-table
// size), (box x0 | y0 << 16, x1 | y1 << 16, spans.y, 0); their number to a_dev
// (0 on overflow).  Clears ranges[total_tiles].  block_sums, block_act: the
// per-256-record totals launch_project_fwd wrote, scanned in place; seg_tot,
// seg_act: seg_count(nrec) entries of scratch.  fr: as the projection took it
// (the row tables clip the rows alike).
void launch_scan_records(hipStream_t s, const uint32_t *count, const uint2 *rect,
                         const uint2 *rspan, SplatPtrs sp, const uint32_t *depth_key, uint32_t *koff,
                         uint2 *rowtab, int nrec, int n, int tile, const ViewDesc *views,
                         const FoveaRows &fr,
                         uint32_t *block_sums, uint32_t *block_act, unsigned long long *seg_tot,
                         uint32_t *seg_act, uint32_t *m_dev, unsigned long long *m_total,
                         uint32_t *a_dev, uint32_t *flags, int64_t capacity, uint32_t *dkey,
                         uint32_t *dval, uint4 *arec, uint2 *ranges, int total_tiles);
// Keys of the a_dev active records in the order dval lists their entries
// (depth order): key = global tile id, value = record id, each record's keys
// over its box rows, each row's listed tiles left to right.  block_sums:
// scratch of scan_blocks(nrec) words, seg_tot of seg_count(nrec).  Emits
// nothing after a key overflow.
void launch_emit(hipStream_t s, const uint32_t *dval, const uint32_t *a_dev, const uint4 *arec,
                 const uint2 *rowtab, int nrec, int n, const ViewDesc *views, int nviews,
                 uint32_t *block_sums, unsigned long long *seg_tot, const unsigned long long *m_total,
                 int64_t capacity, const TileMap &tm, uint32_t *keys, uint32_t *vals);
int seg_count(int64_t nrec);
int scan_blocks(int64_t nrec);

// Stable LSD radix sort of (key, value) pairs by the low `bits` key bits in
// radix_passes(bits) passes of at most 8-bit digits; the count is read from
// n_dev (or n_host when n_dev is null).  Passes write a, b, a, ... (b may alias
// the input); returns 1 when the result is in (ka, va), 2 when in (kb, vb), 0
// when no pass ran (the input).  hist: kRadixBins * grid words; digit_tot:
// kRadixBins words.
int launch_radix_sort(hipStream_t s, const uint32_t *kin, const uint32_t *vin, uint32_t *ka,
                      uint32_t *va, uint32_t *kb, uint32_t *vb, const uint32_t *n_dev,
                      uint32_t n_host, int bits, int grid, uint32_t *hist, uint32_t *digit_tot);
// Stable sort of the (depth bits, value) pairs (k0, v0) of the records that
// list a tile (count n_dev; positive float bits, below 2^31) by depth: pass 1
// by the low 8 bits, passes 2 and 3 by bits 8 - 23 of key - base, where base
// is the smallest key with its low 8 bits clear (found by pass 1: mm holds 2
// grid words, ctl 2), and a fourth pass by bits 24 - 30 of key - base only
// when some key lies 2^24 or more above base (else it returns at once).  The
// sorted values end in vfinal; the keys of the last pass are not written.
// (k1, v1) and (k0, v0) are the passes' intermediates.
void launch_depth_sort(hipStream_t s, uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                       const uint32_t *n_dev, int grid, uint32_t *hist, uint32_t *digit_tot,
                       uint32_t *mm, uint32_t *ctl, uint32_t *vfinal);
int radix_grid_for(int64_t capacity);
int radix_passes(int bits);
constexpr int kRadixBins = 256;

// ranges[t] = [lower_bound(t), lower_bound(t + 1)) in the sorted keys for every
// tile (ranges cleared beforehand); keys mapped by tm when it has a gaze.
void launch_tile_bounds(hipStream_t s, const uint32_t *keys, const uint32_t *m_dev, uint32_t m_host,
                        int64_t capacity, int total_tiles, const ViewDesc *views, int nviews,
                        const TileMap &tm, uint2 *ranges);

// order = all tile ids, tiles with more keys first (by floor(log2(key count)),
// empty tiles last; order within a class unspecified).  counts: scratch of
// 33 * order_groups(total_tiles) words.
void launch_tile_order(hipStream_t s, const uint2 *ranges, int total_tiles, uint32_t *order,
                       uint32_t *counts);
int order_groups(int64_t total_tiles);

// Everything the compositing kernels share.
struct RenderArgs {
    int tile = 16, batch = 128, total_tiles = 0, nviews = 1, nrec = 0;
    int t_mode = 0;                       // 0 recompute, 1 checkpointed, 2 stored transmittance
    int bwd_grid = 1;                     // workgroups of the checkpointed adjoint (unit ids)
    int cus = 256;                        // compute units of the device
    const uint32_t *order = nullptr;      // tile ids, heavy tiles first
    const float *bg = nullptr;            // per-view background [V][3] replacing the cameras' bg
    const float *cull_gaze = nullptr;     // fovea culling: only tiles meeting the fovea are composited
    float cull_radius = 0.f;
    const uint2 *ranges = nullptr;
    const uint32_t *vals = nullptr;
    SplatPtrs sp{};
    const ViewDesc *views = nullptr;
    const gsf_camera *cams = nullptr;
    float *tfinal = nullptr;
    uint32_t *ncontrib = nullptr;
    float4 *ckpt = nullptr;               // [key capacity / B + 1][T*T]
    float4 *fstate = nullptr;             // [pixels]: final (T, colour)
    float *tstore = nullptr;              // [key capacity][T*T]: T in front of each included pair
    const uint32_t *m_dev = nullptr;      // key count on the device, or
    uint32_t m_host = 0;                  //   on the host when m_dev is null
    KeyPlace kp{};                        // where the adjoint writes each key's gradient
    // the launch tiles (total_tiles of them, which ranges and order index):
    // global tile ids, or (tm.gaze, a fovea-culled forward) the compact
    // fovea-box ids of the sort keys
    TileMap tm{};
};

// Front-to-back compositing of all tiles of all views.
void launch_render_fwd(hipStream_t s, const RenderArgs &a, float *out_rgba);

// Back-to-front adjoint of the compositing: every key's screen-space gradient
// into a.kp (zeros for keys it does not reach).
void launch_render_bwd(hipStream_t s, const RenderArgs &a, const float *dl_drgba);
// Their sum per record into g2d [9][nrec] (every entry written).
void launch_grad_sum(hipStream_t s, const KeyPlace &kp, int nrec, float *g2d);

// Pair accounting of the last forward: counters[3] (visited, included, adjoint
// visited), over the tiles and pixels it composited (cull_gaze, nullable: its
// fovea culling).
void launch_count_pairs(hipStream_t s, int tile, int total_tiles, const uint2 *ranges,
                        const uint32_t *vals, SplatPtrs sp, const ViewDesc *views, int nviews,
                        const TileMap &tm, const float *cull_gaze, float cull_radius,
                        unsigned long long *counters);

// Masked L1 loss.  partial: scratch of loss_partials(total_pix) floats.
int loss_partials(int64_t total_pix);
// step_inc (nullable): step counter the final reduction advances by one.
// box > 0 (fovea culling, gaze required): only the box x box pixel window of each
// view starting at its first fovea tile is visited (every pixel of the tiles
// that meet the fovea; nviews * box^2 <= total_pix); dl elsewhere is not written.
// RGBA targets (tgt_planes 4): the target colour is composited over bg
// ([V][3], nullable = black) and, with alpha_term, alpha is a fourth L1 channel.
void launch_loss_l1(hipStream_t s, const float *rgba, const float *target, const float *gaze,
                    float radius_frac, const ViewDesc *views, int nviews, int64_t total_pix,
                    float *dl, float *partial, uint32_t *mask_count, float *loss, uint32_t *flags,
                    int32_t *step_inc, int box, int tile, int tgt_planes, bool alpha_term,
                    const float *bg, uint32_t norm_count, bool accumulate, int max_height);
// norm_count > 0: the mean divides by it (entries over all plans of a multi-plan
// loss) instead of the plan's own masked count; accumulate: loss[0] += the share.
// max_height: the tallest view's height.
// The masked entry count alone (gaze required) into mask_count[0].
void launch_loss_count(hipStream_t s, const float *gaze, float radius_frac, const ViewDesc *views,
                       int nviews, int max_height, int box, int tile, uint32_t channels,
                       uint32_t *mask_count);

// bg[v][c] = top 24 bits of output 1 + (step[0] * kMaxViews + v) * 4 + c of
// SplitMix64(seed), scaled to [0, 1).
void launch_draw_bg(hipStream_t s, uint64_t seed, const int32_t *step, int nviews, float *bg);

// Adam with bias correction for step step[0]; when advance is true a one-thread
// kernel first advances step[0] by one.  skip (nullable): device flags; the
// update is skipped while GSF_FLAG_CAPACITY is set.
void launch_adam(hipStream_t s, float *p, const float *g, float *m, float *v, int64_t n,
                 const SegTable &seg, float b1, float b2, float eps, int32_t *step, bool advance,
                 const uint32_t *skip = nullptr);

// vis[i] = 1 when a record of Gaussian i (count[v * n + i], v < nviews) touched a tile.
void launch_visible(hipStream_t s, const uint32_t *count, int n, int nviews, uint8_t *vis);

// Adam on planar [planes][n] state for the Gaussians with vis[i] != 0 only
// (others untouched), plane c at lr.lr[c]; advance as in launch_adam.
void launch_adam_masked(hipStream_t s, float *p, const float *g, float *m, float *v, int64_t n,
                        int planes, const PlaneLr &lr, const uint8_t *vis, float b1, float b2,
                        float eps, int32_t *step, bool advance, const uint32_t *skip = nullptr);

// m[0..n) = v[0..n) = 0 and step[0] = 0, by a kernel (graph-capturable).
void launch_adam_reset(hipStream_t s, float *m, float *v, int64_t n, int32_t *step);

// Depth-guided reprojection constants (matrices composed and inverted on the
// host in double, stored as float), opaque outside reproject.hip.
struct ReprojConstOpaque {
    alignas(16) unsigned char bytes[160];
};
// False when P_old V_old is singular or a value is not finite.
bool make_reproj(const float *p_old, const float *v_old, const float *pos_old, const float *p_new,
                 const float *v_new, int width, int height, ReprojConstOpaque *out);
// clip [4][H][W] of every pixel (NaN where the depth is not finite and positive).
void launch_reproject(hipStream_t s, const ReprojConstOpaque &k, const float *depth, float *clip);
// Output pixels the no-allocation warp's device-resident z-buffer holds
// (2048 x 2304, which covers one 2064 x 2208 head-mounted-display eye).
constexpr int64_t kWarpScratchPixels = 2048ll * 2304ll;
constexpr int kMaxDevices = 64;
// Device address of that z-buffer on `device` (must be current); looked up
// once per device, the same address returned afterwards.
hipError_t warp_scratch_address(int device, unsigned long long **out);
// Forward warp of rgba [4][H][W] to [4][out_h][out_w] (zbuf: out_w * out_h words).
void launch_reproject_warp(hipStream_t s, const ReprojConstOpaque &k, const float *rgba,
                           const float *depth, int out_w, int out_h, unsigned long long *zbuf,
                           float *out_rgba, int32_t *src);

// First-hit point cloud (synchronises): Gaussians at the first significant hit
// of every pixel ray of the cameras, capped by ray priority; scratch:
// first_hit_scratch_bytes(total rays).
size_t first_hit_scratch_bytes(int64_t nrays);
hipError_t run_first_hits(hipStream_t s, const uint16_t *vol, int n, const gsf_camera *cams,
                          int nviews, const int32_t *widths, const int32_t *heights, float step,
                          float extinction, float thr, float range, const float *lo, const float *hi,
                          float hit_alpha, int color_steps, double opacity, int64_t cap,
                          uint64_t seed, float *params, int64_t *count, int32_t *ray_ids,
                          void *scratch);

// Seeding from a device volume (synchronises); scratch: seed_scratch_bytes(n^3).
hipError_t run_seed(hipStream_t s, const uint16_t *vol, int n, double thr, double range,
                    const double *lo, const double *hi, double opacity, int64_t cap, uint64_t seed,
                    float *params, int64_t *count, void *scratch);
size_t seed_scratch_bytes(int64_t nvox);
// Emission-absorption targets of n_views cameras (asynchronous).
hipError_t run_raymarch(hipStream_t s, const uint16_t *vol, int n, const gsf_camera *cams, int nviews,
                        const int32_t *widths, const int32_t *heights, float step, float extinction,
                        float t_stop, float thr, float range, const float *lo, const float *hi,
                        float *out);

void launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t value);
void launch_fill_f32(hipStream_t s, float *p, int64_t n, float value);

}  // namespace gsf
