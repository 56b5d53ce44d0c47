// raster.hip - per-tile front-to-back alpha compositing, its back-to-front
// adjoint, and the masked L1 image loss.
//
// One workgroup per screen tile (T x T pixels, T in {8, 16, 32}); one thread
// per pixel (T = 32: four pixels per thread).  The tile's depth-ordered list of
// splats is staged through LDS in batches of B records (B in {64, 128, 256})
// that every wave then reads by broadcast.  Per pixel and splat, with the
// projection's conic pre-scaled by log2(e) so that power2 = log2(e) * power:
//   skip if power2 > 0 or power2 < tau, tau = log2(1 / (255 o))
//        (the second test is o e^power < 1/255 without the exponential);
//   alpha = min(0.99, o 2^power2);
//   stop before the splat if T (1 - alpha) < 1e-4;
//   C += colour alpha T;  T *= 1 - alpha.
// A wave leaves the batch once all its pixels have stopped (checked every four
// splats) and the workgroup leaves the tile once all waves have.  A pixel's
// arithmetic sequence does not depend on T, B or the tile's other pixels, so
// images are bitwise independent of the tile size and the batch size.
//
// The adjoint walks the same list back to front from each pixel's last
// included splat.  Transmittance modes: recompute (the transmittance in front
// of each splat is rebuilt as T_i = T_{i+1} / (1 - alpha_i) from the final
// state; one workgroup per tile), checkpointed ((T, colour) stored by the
// forward at every LDS-batch boundary; persistent workgroups over (tile, batch)
// units, each rebuilding T within its batch) and stored (the forward stores
// T_i of every included (splat, pixel) pair at [key position][pixel of tile];
// the adjoint reads it; one workgroup per tile).  The nine per-splat screen-space
// gradient terms of a wave are summed across its lanes with DPP row
// operations, kept per row in LDS, and stored once per (key, field) at the
// key's own position; a separate pass sums each record's keys (no atomics).
// With 16-pixel tiles each wave covers an 8x8 quadrant of the tile and skips
// the splats whose padded support ellipse misses it.
#include "gs_internal.h"

namespace gsf {
namespace {

constexpr float kLn2 = 0.69314718055994531f;

// Shared by every kernel that walks a tile list so all take identical decisions.
// a = (hx, hy, A2, B2), b = (C2, opacity, red, green), c = (blue, tau, ix, iy)
// with A2 = -log2(e) A / 2, B2 = -log2(e) B, C2 = -log2(e) C / 2; (x, y) is
// the integer pixel (as float) and (dx, dy) its centre's offset from the mean.
__device__ __forceinline__ float splat_dx(float x, float ix, float hx) { return (x - ix) + hx; }

// power2 = A2 dx^2 + B2 dx dy + C2 dy^2, evaluated as dx (A2 dx + B2 dy) + (C2 dy) dy
// (five operations); every kernel that decides inclusion uses this one form.
__device__ __forceinline__ float splat_power2(const float4 &a, const float4 &b, float dx, float dy) {
    return fmaf(dx, fmaf(a.z, dx, a.w * dy), (b.x * dy) * dy);
}

__device__ __forceinline__ bool splat_alpha(const float4 &a, const float4 &b, const float4 &c,
                                            float x, float y, float &alpha, float &ae, float &ex,
                                            float &dx, float &dy) {
    dx = splat_dx(x, c.z, a.x);
    dy = splat_dx(y, c.w, a.y);
    const float power2 = splat_power2(a, b, dx, dy);
    if (power2 > 0.f || power2 < c.y) return false;
    ex = __builtin_amdgcn_exp2f(power2);
    ae = b.y * ex;
    alpha = fminf(kAlphaMax, ae);
    return true;
}

// Threads of an adjoint workgroup: one wave per 8x8 or 16x16 tile (1 or 4 pixels
// per lane), two waves per 32x32 tile (8 pixels per lane).  Each lane first sums
// its own pixels' contributions, so the per-splat cross-lane reductions, the
// bulk of the adjoint's VALU work, are shared by more pixels.
template <int T>
constexpr int bwd_threads() { return T == 32 ? 128 : 64; }

// A record's c = (blue, tau, ix, iy): tau = -log2(255 o) is the alpha
// threshold of the base-2 exponent, computed once by the projection.  The
// padded half height of the support (where o e^power >= 1/255 can hold) is
// the ellipse's y extent plus the absolute padding.
// Half height of the padded ellipse for the quadrant test, with the hardware
// reciprocal and square root: their few-ulp error lies far inside the padding,
// and the forward and the adjoint both use this form, so they skip the same
// quadrants.  (Tile enumeration keeps the exact form everywhere.)
__device__ __forceinline__ float quad_half_height(const float4 &e0) {
    return __builtin_amdgcn_sqrtf(e0.y * __builtin_amdgcn_rcpf(e0.z));
}

__device__ __forceinline__ float support_half_height(const float4 &e0) {
    return sqrtf(e0.y / e0.z) + kBoxAbs;
}

typedef __attribute__((address_space(3))) void *lds_void_ptr;
__device__ __forceinline__ lds_void_ptr lds_ptr(void *p) { return (lds_void_ptr)p; }

// Whether rows with offsets [lo, lo + span] from a splat's mean can meet its
// support of half height h (NaN-safe: only a definite miss returns false).
// Rows farther away are skipped as a block: the per-pixel test would skip
// every pair there.
__device__ __forceinline__ bool rows_meet(float lo, float span, float h) {
    return !(lo > h) && !(lo + span < -h);
}

__device__ __forceinline__ int view_of_tile(const ViewDesc *__restrict__ views, int nviews, int gt) {
    int v = 0;
    while (v + 1 < nviews && gt >= views[v + 1].tile_off) v++;
    return v;
}

// Launch tile c of the compositing kernels: a global tile id, or (tm.gaze) a
// compact fovea-box id (view c / box^2, then row-major from the view's first
// fovea tile, as the fovea-culled sort keys).  False for a box tile past the
// view's fovea tiles (no pixel of it is composited).
__device__ __forceinline__ bool launch_tile(uint32_t c, const TileMap &tm,
                                            const ViewDesc *__restrict__ views, int nviews, int T,
                                            int &v, ViewDesc &vd, int &ty, int &tx) {
    if (tm.gaze) {
        const uint32_t box = (uint32_t)tm.box, area = box * box;
        v = (int)(c / area);
        const uint32_t l = c - (uint32_t)v * area, ly = l / box;
        vd = views[v];
        const FoveaTiles f = fovea_tiles(tm.gaze, v, tm.radius, vd.width, vd.height, T);
        ty = f.ty0 + (int)ly;
        tx = f.tx0 + (int)(l - ly * box);
        return tx <= f.tx1 && ty <= f.ty1;
    }
    v = view_of_tile(views, nviews, (int)c);
    vd = views[v];
    const int local = (int)c - vd.tile_off;
    ty = local / vd.tiles_x;
    tx = local - ty * vd.tiles_x;
    return true;
}

// Pixel (x, y) of view v lies in the fovea disk (the loss's mask): its centre
// within `radius` pixels of the gaze point, tested in FP32; no gaze: every pixel.
__device__ __forceinline__ bool in_fovea(const float *__restrict__ gaze, int v, int x, int y,
                                         float radius) {
    if (!gaze) return true;
    const float dx = (float)x + 0.5f - gaze[2 * v], dy = (float)y + 0.5f - gaze[2 * v + 1];
    return dx * dx + dy * dy <= radius * radius;
}

// Sum of x over the 64 lanes of a wave, valid in lane 63: four row shifts
// (DPP row_shr 1, 2, 4, 8) leave each 16-lane row's total in its lane 15, then
// row_bcast:15 and row_bcast:31 fold the rows together.  All steps are VALU
// instructions with DPP operands (no LDS traffic).

// Sum over each 16-lane row, left in the row's last lane (15, 31, 47, 63).
__device__ __forceinline__ float row_sum_lane15(float x) {
    x += dpp_shift<0x111, 0xf>(x);   // row_shr:1
    x += dpp_shift<0x112, 0xf>(x);   // row_shr:2
    x += dpp_shift<0x114, 0xf>(x);   // row_shr:4
    x += dpp_shift<0x118, 0xf>(x);   // row_shr:8
    return x;
}

// Wave sums of two splats' nine per-lane terms a and b at once.  A
// v_permlane32_swap per field halves the 18 values (lanes 0-31 then hold
// splat a's partial sums, lanes 32-63 splat b's), a v_permlane16_swap per
// pair of fields leaves one (splat, field) per 16-lane row, and a row sum
// (four DPP adds) finishes: lane 15 of row 0 holds a's fields 0, 2, 4, 6, 8
// in out[0..4], row 1 a's fields 1, 3, 5, 7 in out[0..3], rows 2 and 3 the
// same of b.  24 VALU instructions per splat against 36 for nine row sums.
// (Written as inline assembly: this compiler folds the two results of the
// permlane-swap builtins into one when both feed the same expression.  The
// swap is a register-only VALU operation; the s_nop gives it the two wait
// states it needs after the VALU writes of its operands.)
__device__ __forceinline__ float swap_add32(float x, float y) {
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(x), "+v"(y));
    return x + y;
}
__device__ __forceinline__ float swap_add16(float x, float y) {
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(x), "+v"(y));
    return x + y;
}
__device__ __forceinline__ void pair_sums(const float (&a)[9], const float (&b)[9], float (&out)[5]) {
    float L[9];
#pragma unroll
    for (int f = 0; f < 9; f++) L[f] = swap_add32(a[f], b[f]);
#pragma unroll
    for (int k = 0; k < 4; k++) out[k] = row_sum_lane15(swap_add16(L[2 * k], L[2 * k + 1]));
    out[4] = row_sum_lane15(swap_add16(L[8], 0.f));
}

// MODE 1 (checkpointed): also store (T, colour) of every pixel after each LDS
// batch that is not the tile's last (slot = boundary position / B, unique over
// all tiles) and the final (T, colour), so the adjoint can start at any batch.
// MODE 2 (stored): also store T in front of every included pair at
// tstore[key position * T*T + pixel of tile].
// One workgroup per tile, workgroup i taking tile order[i]: the order lists
// tiles with more keys first, so the dispatcher starts the heavy tiles on
// different CUs at once and fills in with light ones as slots free up, however
// the keys cluster on screen.
// Threads of a forward workgroup: one per pixel (at most 256).  A 16-pixel
// tile is composited by four waves, one per 8x8 quadrant, each skipping the
// splats whose padded ellipse misses its quadrant.  SPLIT (16-pixel tiles):
// the four quadrants are four one-wave workgroups instead; they run
// independently, each with no barrier shared with the others, at the cost of
// staging every batch four times, which pays only where the heaviest tiles,
// not throughput, set the time (few tiles; the launcher's choice).
// Workgroups are dealt to the 8 XCDs round robin (workgroup g to XCD g mod
// 8), so workgroup g takes quadrant (g >> 3) & 3 of the tile at position
// 8 (g >> 5) + (g & 7) of the order: the four quadrants of a tile share an
// XCD and its L2, and the order's heaviest tiles still come first.
template <int T, bool SPLIT>
constexpr int fwd_threads() { return SPLIT ? 64 : (T * T < 256 ? T * T : 256); }

template <int T, int B, int MODE, bool SPLIT>
__global__ __launch_bounds__((fwd_threads<T, SPLIT>())) void k_render_fwd(
    const uint32_t *__restrict__ order,
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, const gsf_camera *__restrict__ cams,
    float *__restrict__ out_rgba, float *__restrict__ tfinal, uint32_t *__restrict__ ncontrib,
    float4 *__restrict__ ckpt, float4 *__restrict__ fstate, float *__restrict__ tstore,
    const float *__restrict__ bg, const float *__restrict__ cull_gaze, float cull_radius,
    int total_tiles, TileMap tm) {
    constexpr bool CKPT = MODE == 1;
    constexpr bool QUAD = T == 16;   // a wave composites one 8 x 8 quadrant
    static_assert(!SPLIT || QUAD, "only 16-pixel tiles are split");
    constexpr int NT = fwd_threads<T, SPLIT>();
    constexpr int PPT = QUAD ? 1 : T * T / NT;
    constexpr int ROWS = NT / T;
    constexpr int U = 4;   // splats between wave-level completion checks
    static_assert(U == 4, "a group of splat indices is read as one int4");
    constexpr int kListLen = 64 + U;   // per wave: one 64-splat chunk, padded
    // PREF (a batch no larger than the workgroup): two LDS buffers; the
    // records of the next batch are copied from global memory straight into
    // the other buffer (global_load_lds, no registers; wave w copies entries
    // 64 w .. 64 w + 63) while the current batch composites, the record ids
    // being read one batch further ahead.
    constexpr bool PREF = B <= NT;
    // A buffer holds the batch's records a, b, c and support ellipses
    // (slope, kw, ws, dyr) at sections 0, 1, 2, 3 of B + 1 entries.  Buffers
    // 0 and 1 are separate arrays, so the compiler sees that reads of one do
    // not wait for copies into the other.  Entry B of a, b, c: an inert splat
    // (power2 = 0 < tau = +inf: never included) that pads a wave's last
    // group of U.
    // (Entry 0 of each array is unused: a copy addressed at an array's very
    // start loses the alias information that lets reads of the other buffer
    // proceed while it is in flight.)
    constexpr int SEC = B + 1;
    constexpr int NW = NT / 64;
    __shared__ __align__(16) int s_list[NW * kListLen];
    // the waves' votes of a workgroup-wide test, two rows used in turn: a row is
    // written again only two votes later, after a barrier that every wave
    // reaches once it has read the row
    __shared__ __align__(16) uint32_t s_vote[2][NW < 4 ? 4 : NW];
    __shared__ float4 s_buf0_[1 + 4 * SEC];
    __shared__ float4 s_buf1_[PREF ? 1 + 4 * SEC : 1];
    float4 *const s_buf0 = s_buf0_ + 1;
    float4 *const s_buf1 = s_buf1_ + 1;

    const int quad = SPLIT ? (int)((blockIdx.x >> 3) & 3u) : (int)(threadIdx.x >> 6);
    const uint32_t oi = SPLIT ? (blockIdx.x >> 5) * 8u + (blockIdx.x & 7u) : blockIdx.x;
    if (oi >= (uint32_t)total_tiles) return;   // the split grid is padded to whole groups of 8 tiles
    const uint32_t ti = order[oi];
    int v, ty, tx;
    ViewDesc vd;
    if (!launch_tile(ti, tm, views, nviews, T, v, vd, ty, tx)) return;
    // Fovea culling: only the pixels of the fovea disk are composited; the others,
    // which carry no loss, start stopped (background, no contributor).  Over the
    // compact fovea-box tiles, a tile that cannot hold a pixel of the disk is not
    // visited at all (the adjoint skips it alike); over global tiles every tile
    // is, so that each holds its pixels' state.
    if (tm.gaze && !fovea_tile_live(tm.gaze, v, tm.radius, vd.width, vd.height, T, tx, ty)) return;
    const float disk_r = cull_gaze ? cull_radius * (float)vd.width : 0.f;
    const uint2 rg = ranges[ti];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lx = QUAD ? (quad & 1) * 8 + (lane & 7) : threadIdx.x % T;
    const int ly = QUAD ? (quad >> 1) * 8 + (lane >> 3) : threadIdx.x / T;
    if (threadIdx.x == 0) {
        s_buf0[B] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_buf0[SEC + B] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_buf0[2 * SEC + B] = make_float4(0.f, __builtin_inff(), 0.f, 0.f);
        if constexpr (PREF) {
            s_buf1[B] = make_float4(0.f, 0.f, 0.f, 0.f);
            s_buf1[SEC + B] = make_float4(0.f, 0.f, 0.f, 0.f);
            s_buf1[2 * SEC + B] = make_float4(0.f, __builtin_inff(), 0.f, 0.f);
        }
    }

    // Whether `pred` holds on every thread of the workgroup: one barrier (the
    // waves' votes in LDS), which also ends the batch's copies into LDS and its
    // reads of the buffer.
    uint32_t vrow = 0u;
    auto block_all = [&](bool pred) -> bool {
        const bool w = __all(pred);
        if constexpr (NW == 1) {
            __syncthreads();
            return w;
        } else {
            if (lane == 0) s_vote[vrow][wave] = w ? 1u : 0u;
            __syncthreads();
            uint32_t r = 1u;
#pragma unroll
            for (int i = 0; i < NW; i++) r &= s_vote[vrow][i];
            vrow ^= 1u;
            return r != 0u;
        }
    };

    // Tr[k] is the pixel's transmittance while it composites; a pixel that has
    // stopped (or lies outside the image) holds -T instead, so one compare
    // gives its state and no flag is carried from splat to splat.
    float px[PPT], py[PPT], Tr[PPT], cr[PPT], cg[PPT], cb[PPT];
    uint32_t last[PPT];
    int pix[PPT];   // the pixel's row-major index in the tile
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int x = tx * T + lx, y = ty * T + ly + k * ROWS;
        px[k] = (float)x;   // integer pixel; its centre's offset from a mean is splat_dx
        py[k] = (float)y;
        pix[k] = (ly + k * ROWS) * T + lx;
        Tr[k] = x < vd.width && y < vd.height && in_fovea(cull_gaze, v, x, y, disk_r) ? 1.f : -1.f;
        cr[k] = cg[k] = cb[k] = 0.f;
        last[k] = 0u;
    }

    // Composite the batch at bs from one LDS buffer; true once every pixel of
    // the tile has stopped.  Ends with a barrier, after which the buffer is free.
    auto composite = [&](uint32_t bs, const float4 *buf) -> bool {
        const float4 *SA = buf, *SB = buf + SEC, *SC = buf + 2 * SEC, *SE = buf + 3 * SEC;
        const int nb = (int)min((uint32_t)B, rg.y - bs);
        // list entries are the byte offset 16 j of the splat's slot j in a
        // section, which the LDS reads take as their address (the section's
        // start being the constant part); slot j is the splat's 1-based place
        // j + off in the tile's list, what last[] records: within the batch the
        // pixel keeps the offset (lastb, ~0 for none) and converts it at the end
        const int off = (int)(bs - rg.x) + 1;
        uint32_t lastb[PPT];
#pragma unroll
        for (int k = 0; k < PPT; k++) lastb[k] = ~0u;
        // a wave whose pixels have all stopped (or start outside the disk or
        // the image) skips the batch: no quadrant tests, no list
        bool stopped = true;
#pragma unroll
        for (int k = 0; k < PPT; k++) stopped &= !(Tr[k] > 0.f);
        bool done = __all(stopped);
        // the batch 64 splats at a time: the wave's splats are the set bits of
        // m (with 16-pixel tiles, those whose padded ellipse reaches the wave's
        // quadrant)
        for (int cb0 = 0; cb0 < nb && !done; cb0 += 64) {
            const int jl = cb0 + lane;
            bool meet = jl < nb;
            if (QUAD && meet) {
                const float4 e0 = SE[jl], a0 = SA[jl], c0 = SC[jl];
                const Ellipse e{e0.x, e0.y, e0.z, e0.w, quad_half_height(e0), a0.x, a0.y, (int)c0.z, (int)c0.w};
                meet = quad_meets(e, tx * T + (quad & 1) * 8, ty * T + (quad >> 1) * 8);
            }
            // the wave's list of them in LDS, padded with the inert slot to whole
            // groups of U, read back a group at a time (the indices stay in
            // vector registers: no scalar bookkeeping per splat)
            const uint64_t m = __ballot(meet);
            const int cnt = (int)__popcll(m);
            int *list = s_list + wave * kListLen;
            if (meet) list[lanes_below(m)] = jl * (int)sizeof(float4);
            if (lane < U) list[cnt + lane] = B * (int)sizeof(float4);
            for (int g = 0; g < cnt; g += U) {
                bool all = true;
#pragma unroll
                for (int k = 0; k < PPT; k++) all &= !(Tr[k] > 0.f);
                if (__all(all)) {
                    done = true;
                    break;
                }
                const int4 j4 = *(const int4 *)(list + g);
                const uint32_t bo[U] = {(uint32_t)j4.x, (uint32_t)j4.y, (uint32_t)j4.z, (uint32_t)j4.w};
                // Phase 1: the U splats' alphas are independent of each other and of
                // the pixel state; computed without branches (skipped splats get
                // valid = false; every operand is read whatever the outcome).
                float4 a[U], b[U];
                float4 c[U];
#pragma unroll
                for (int u = 0; u < U; u++) {
                    a[u] = *(const float4 *)((const char *)SA + bo[u]);
                    b[u] = *(const float4 *)((const char *)SB + bo[u]);
                    c[u] = *(const float4 *)((const char *)SC + bo[u]);
                }
#pragma unroll
                for (int k = 0; k < PPT; k++) {
                    float alpha[U];
                    bool valid[U];
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const float dx = splat_dx(px[k], c[u].z, a[u].x);
                        const float dy = splat_dx(py[k], c[u].w, a[u].y);
                        const float power2 = splat_power2(a[u], b[u], dx, dy);
                        valid[u] = !(power2 > 0.f) & !(power2 < c[u].y);
                        alpha[u] = fminf(kAlphaMax, b[u].y * __builtin_amdgcn_exp2f(power2));
                    }
                    // Phase 2: the sequential front-to-back update.  An included
                    // splat performs exactly the float operations of the definition
                    // (Tn = T (1 - alpha), w = alpha T, C += colour w); any other
                    // gets w = 0, which leaves the (non-negative) colour sums as
                    // they are bit for bit.
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        // A stopped pixel holds -T < 0, so its Tn < 0 < kTStop: it is
                        // never included, and -|T| keeps it stopped.  A running pixel
                        // stops where Tn < kTStop and then holds -T.
                        const float Tn = Tr[k] * (1.f - alpha[u]);
                        const bool inc = valid[u] && !(Tn < kTStop);
                        const bool stop = valid[u] && !inc;
                        if (MODE == 2 && inc)
                            tstore[(size_t)(bs + bo[u] / (uint32_t)sizeof(float4)) * (T * T) + pix[k]] = Tr[k];
                        const float w = (inc ? alpha[u] : 0.f) * Tr[k];
                        cr[k] = fmaf(b[u].z, w, cr[k]);
                        cg[k] = fmaf(b[u].w, w, cg[k]);
                        cb[k] = fmaf(c[u].x, w, cb[k]);
                        Tr[k] = inc ? Tn : (stop ? -fabsf(Tr[k]) : Tr[k]);
                        lastb[k] = inc ? bo[u] : lastb[k];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PPT; k++)
            if (lastb[k] != ~0u) last[k] = lastb[k] / (uint32_t)sizeof(float4) + (uint32_t)off;
        if (CKPT && bs + B < rg.y) {
            float4 *slot = ckpt + (size_t)((bs + B) / B) * (T * T);
#pragma unroll
            for (int k = 0; k < PPT; k++)
                slot[pix[k]] = make_float4(fabsf(Tr[k]), cr[k], cg[k], cb[k]);
        }
        bool all = true;
#pragma unroll
        for (int k = 0; k < PPT; k++) all &= !(Tr[k] > 0.f);
        return block_all(all);
    };

    // A workgroup none of whose pixels composites (all outside the fovea disk or
    // the image) stages nothing: its pixels are written as they start.
    bool any_px = false;
#pragma unroll
    for (int k = 0; k < PPT; k++) any_px |= Tr[k] > 0.f;
    if (!block_all(!any_px)) {
        if constexpr (PREF) {
            // copy record r of entry threadIdx.x into a buffer (this wave's 64 slots)
            auto stage = [&](float4 *buf, uint32_t r) {
                float4 *d = buf + (threadIdx.x & ~63u);
                const float4 *rr = sp.at(r, 0);   // one 64-byte chunk: a, b, c, ellipse
                __builtin_amdgcn_global_load_lds((const void *)(rr + kRecA), lds_ptr(d), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((const void *)(rr + kRecB), lds_ptr(d + SEC), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((const void *)(rr + kRecC), lds_ptr(d + 2 * SEC), 16, 0, 0);
                if constexpr (QUAD)
                    __builtin_amdgcn_global_load_lds((const void *)(rr + kRecEll), lds_ptr(d + 3 * SEC), 16, 0, 0);
            };
            const uint32_t j = threadIdx.x;
            uint32_t rnext = 0u;
            if (j < (uint32_t)B && rg.x + j < rg.y) stage(s_buf0, vals[rg.x + j]);
            if (j < (uint32_t)B && rg.x + B + j < rg.y) rnext = vals[rg.x + B + j];
            __syncthreads();   // the inert slots and the first batch
            // Batches alternate between the buffers.  A batch has arrived before
            // the barrier that ended the previous one, after which the other
            // buffer is free: the next batch is copied there while this one
            // composites.
            for (uint32_t bs = rg.x; bs < rg.y;) {
                if (j < (uint32_t)B && bs + B + j < rg.y) stage(s_buf1, rnext);
                if (j < (uint32_t)B && bs + 2 * B + j < rg.y) rnext = vals[bs + 2 * B + j];
                if (composite(bs, s_buf0)) break;
                if ((bs += B) >= rg.y) break;
                if (j < (uint32_t)B && bs + B + j < rg.y) stage(s_buf0, rnext);
                if (j < (uint32_t)B && bs + 2 * B + j < rg.y) rnext = vals[bs + 2 * B + j];
                if (composite(bs, s_buf1)) break;
                bs += B;
            }
        } else {
            __syncthreads();   // the inert slots
            for (uint32_t bs = rg.x; bs < rg.y; bs += B) {
                const int nb = (int)min((uint32_t)B, rg.y - bs);
                for (int j = threadIdx.x; j < nb; j += NT) {
                    const float4 *rr = sp.at(vals[bs + j], 0);
                    s_buf0[j] = rr[kRecA];
                    s_buf0[SEC + j] = rr[kRecB];
                    s_buf0[2 * SEC + j] = rr[kRecC];
                    if constexpr (QUAD) s_buf0[3 * SEC + j] = rr[kRecEll];
                }
                __syncthreads();
                if (composite(bs, s_buf0)) break;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; k++) Tr[k] = fabsf(Tr[k]);

    const float *bgv = bg ? bg + 3 * v : cams[v].bg;
    const float bg0 = bgv[0], bg1 = bgv[1], bg2 = bgv[2];
    const size_t plane = (size_t)vd.width * vd.height;
    float *img = out_rgba + 4 * (size_t)vd.pix_off;
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int x = tx * T + lx, y = ty * T + ly + k * ROWS;
        if (!(x < vd.width && y < vd.height)) continue;
        const size_t q = (size_t)y * vd.width + x;
        img[q] = fmaf(Tr[k], bg0, cr[k]);
        img[plane + q] = fmaf(Tr[k], bg1, cg[k]);
        img[2 * plane + q] = fmaf(Tr[k], bg2, cb[k]);
        img[3 * plane + q] = 1.f - Tr[k];
        tfinal[vd.pix_off + q] = Tr[k];
        ncontrib[vd.pix_off + q] = last[k];
        if (CKPT) fstate[vd.pix_off + q] = make_float4(Tr[k], cr[k], cg[k], cb[k]);
    }
}

// Per-splat gradient sums of one adjoint wave, for a block of R = 64
// consecutive splats (stored as soon as a block is done, one lane per splat,
// so that every lane of the wave stores): nine fields of R splats, plus one
// word so that two waves' slots fall in different LDS banks.  A checkpointed
// unit (one LDS batch of up to 64) stores once.
template <int MODE>
constexpr int kRing = 64;
template <int MODE>
constexpr int kGradSlot = 9 * kRing<MODE> + 1;
static_assert(kRing<0> % 2 == 0 && kRing<1> % 2 == 0, "splat pairs stay within a block");

// Unit of adjoint work: the entries [us, ue) of launch tile ti's list (tm maps
// it to its view and tile).  With
// checkpoints (MODE 1) a unit is one LDS batch of B entries and starts from the
// state the forward stored at the batch's end; otherwise a unit is the whole
// list and starts from the final state.  MODE 2 reads each included pair's
// transmittance from tstore instead of dividing.
template <int T, int B, int MODE>
__device__ __forceinline__ void render_bwd_unit(
    uint32_t ti, const TileMap &tm, uint32_t us, uint32_t ue, bool last_unit, const uint2 &rg,
    const uint32_t *__restrict__ vals, SplatPtrs sp, const ViewDesc *__restrict__ views,
    int nviews, const gsf_camera *__restrict__ cams, const float *__restrict__ tfinal,
    const uint32_t *__restrict__ ncontrib, const float4 *__restrict__ fstate,
    const float4 *__restrict__ ckpt, const float *__restrict__ tstore, const float *__restrict__ bg,
    const float *__restrict__ dl, const KeyPlace &kp, float4 *s_a, float4 *s_b, float4 *s_c,
    uint32_t *s_q, uint8_t *s_m, float *s_g, uint64_t *s_hit, float *s_h, uint32_t *s_nmax) {
    constexpr bool CKPT = MODE == 1;
    constexpr int TL = T == 8 ? 3 : T == 16 ? 4 : 5;
    constexpr int R = kRing<MODE>, GS = kGradSlot<MODE>;
    constexpr int NT = bwd_threads<T>();
    constexpr int PPT = T * T / NT;
    constexpr int ROWS = NT / T;
    constexpr int NW = NT / 64;
    // 16-pixel tiles: one wave, pixel block k = quadrant k of the tile (8 x 8),
    // and a splat skips the quadrants its padded ellipse does not reach
    constexpr bool QUAD = T == 16;
    static_assert(!QUAD || (NT == 64 && PPT == 4), "quadrant layout: one wave, four blocks");
    int v, ty, tx;
    ViewDesc vd;
    launch_tile(ti, tm, views, nviews, T, v, vd, ty, tx);   // a tile with keys: valid
    // a fovea-culled forward over compact tiles composited only the disk's pixels
    // of the tiles that may hold some (the others carry no loss): the rest have no
    // contributor here (over global tiles the forward left them stopped, with no
    // contributor, which the pixel state says)
    const bool live = !tm.gaze || fovea_tile_live(tm.gaze, v, tm.radius, vd.width, vd.height, T, tx, ty);
    const float disk_r = tm.gaze ? tm.radius * (float)vd.width : 0.f;
    const int lane = threadIdx.x & 63;
    const float *bgv = bg ? bg + 3 * v : cams[v].bg;
    const float bg0 = bgv[0], bg1 = bgv[1], bg2 = bgv[2];
    const size_t plane = (size_t)vd.width * vd.height;
    const float *dimg = dl + 4 * (size_t)vd.pix_off;

    // gR: dL/dC-weighted colour behind the current splat, less gA Tf (the alpha
    // plane's share), carried as one value since only that difference is used
    float px[PPT], py[PPT], Tr[PPT], Tf[PPT], gR[PPT], g0[PPT], g1[PPT], g2[PPT], gA[PPT];
    uint32_t nc[PPT];
    int pix[PPT];   // the pixel's row-major index in the tile
    uint32_t my_max = 0;
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int lx = QUAD ? (k & 1) * 8 + (lane & 7) : threadIdx.x % T;
        const int ly = QUAD ? (k >> 1) * 8 + (lane >> 3) : threadIdx.x / T + k * ROWS;
        pix[k] = ly * T + lx;
        const int x = tx * T + lx, y = ty * T + ly;
        const bool inside = live && x < vd.width && y < vd.height && in_fovea(tm.gaze, v, x, y, disk_r);
        const size_t q = inside ? (size_t)y * vd.width + x : 0;
        px[k] = (float)x;   // integer pixel; its centre's offset from a mean is splat_dx
        py[k] = (float)y;
        if (inside) {
            Tf[k] = tfinal[vd.pix_off + q];
            nc[k] = ncontrib[vd.pix_off + q];
            g0[k] = dimg[q];
            g1[k] = dimg[plane + q];
            g2[k] = dimg[2 * plane + q];
            gA[k] = dimg[3 * plane + q];
        }
        // a pixel no splat reached passes no gradient, whatever its dL/dimage
        // (which a fovea-culled loss may not have written): it starts at zero
        if (!inside || nc[k] == 0u) {
            Tf[k] = 1.f;
            nc[k] = 0u;
            g0[k] = g1[k] = g2[k] = gA[k] = 0.f;
        }
        const float gbg = Tf[k] * (g0[k] * bg0 + g1[k] * bg1 + g2[k] * bg2);
        if (CKPT && !last_unit && rg.x + nc[k] > us) {
            // colour behind the unit = final colour - colour accumulated at its end
            const float4 fs = fstate[vd.pix_off + q];
            const float4 cp = ckpt[(size_t)(ue / B) * (T * T) + pix[k]];
            Tr[k] = cp.x;
            gR[k] = gbg + g0[k] * (fs.y - cp.y) + g1[k] * (fs.z - cp.z) + g2[k] * (fs.w - cp.w);
        } else {
            Tr[k] = Tf[k];
            gR[k] = gbg;
        }
        gR[k] -= gA[k] * Tf[k];
        my_max = max(my_max, nc[k]);
    }
    // 16-pixel tiles: per quadrant (one per pixel block of the wave) the largest
    // contributor count; a splat at or past it reaches no pixel of the quadrant
    // (each would add exact zeros and keep its state), so the quadrant is skipped
    uint32_t qmax[PPT];
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        uint32_t x = nc[k];
        if (QUAD) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
            x = __builtin_amdgcn_readfirstlane(x);
        }
        qmax[k] = x;
    }
    // the tile's largest contributor count: a wave reduction, then (several
    // waves) their maximum through LDS (an LDS atomic with per-lane values
    // would be serialised over the lanes)
    uint32_t nmax;
    if (QUAD) {
        nmax = max(max(qmax[0], qmax[1]), max(qmax[2], qmax[3]));
    } else {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) my_max = max(my_max, (uint32_t)__shfl_xor((int)my_max, o, 64));
        nmax = __builtin_amdgcn_readfirstlane(my_max);
        if (NW > 1) {
            __syncthreads();
            if (lane == 0) s_nmax[threadIdx.x >> 6] = nmax;
            __syncthreads();
#pragma unroll
            for (int w = 0; w < NW; w++) nmax = max(nmax, s_nmax[w]);
        }
    }
    const uint32_t top = min(ue, rg.x + nmax);

    for (uint32_t be = top; be > us;) {
        const uint32_t bs = be - us > (uint32_t)B ? be - (uint32_t)B : us;
        const int nb = (int)(be - bs);
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += NT) {
            const uint32_t r = vals[bs + j];
            const float4 *rr = sp.at(r, 0);   // one 64-byte chunk: splat and ellipse
            const float4 ra = rr[kRecA], rb = rr[kRecB], rc = rr[kRecC], e0 = rr[kRecEll];
            s_a[j] = ra;
            s_b[j] = rb;
            s_c[j] = rc;
            s_q[j] = key_slot(kp, r, ty, tx);
            if (QUAD) {
                const Ellipse e{e0.x, e0.y, e0.z, e0.w, quad_half_height(e0), ra.x, ra.y, (int)rc.z, (int)rc.w};
                s_m[j] = (uint8_t)quadrant_mask(e, tx * T, ty * T);
            } else {
                s_h[j] = support_half_height(e0);
            }
        }
        __syncthreads();
        uint64_t hit = 0ull;   // splats of the current block of R some pixel of the wave took
        // Splat j's per-lane sums: te dx, te dy, te dx^2, te dx dy, te dy^2 (te =
        // dL/do, so that o te = dL/dpower), dL/do, dL/dcolour; the opacity and
        // the conic factors of the mean gradient are applied once per splat when
        // the sums are flushed.  True if some pixel of the wave took the splat.
        auto splat_terms = [&](int j, float (&acc)[9]) -> bool {
            const uint32_t pos = bs + (uint32_t)j - rg.x;   // list position in the tile
            const float4 a = s_a[j];
            const float4 b = s_b[j];
            const float4 c = s_c[j];
            const float hy = QUAD ? 0.f : s_h[j];
            // the splat's quadrant mask, wave-uniform: tested in scalar registers
            const uint32_t qm = QUAD ? __builtin_amdgcn_readfirstlane((uint32_t)s_m[j]) : 0u;
            // row offset of the tile's first row from the mean; block k adds k ROWS
            const float dy0 = splat_dx((float)(ty * T), c.w, a.y);
            // (-0 is the exact identity of addition, so the first term needs no add)
#pragma unroll
            for (int f = 0; f < 9; f++) acc[f] = -0.f;
            // some pixel of the wave took the splat: with quadrants, known
            // (wave-uniform) from the quadrant skip; else from a per-lane flag
            bool took = false, any = false;
#pragma unroll
            for (int k = 0; k < PPT; k++) {
                if (QUAD ? (!((qm >> k) & 1u) || pos >= qmax[k])                     // wave-uniform
                         : !rows_meet(dy0 + (float)(k * ROWS), (float)(ROWS - 1), hy)) continue;
                // Branch-free per lane: every value is computed and a pixel the
                // splat does not reach (behind its last contributor, or alpha
                // below 1/255) adds exact zeros and keeps its state.  An
                // included pixel does exactly the float operations of the adjoint.
                const float dx = splat_dx(px[k], c.z, a.x);
                const float dy = splat_dx(py[k], c.w, a.y);
                const float power2 = splat_power2(a, b, dx, dy);
                const bool inc = (pos < nc[k]) & !(power2 > 0.f) & !(power2 < c.y);
                // no pixel of the block takes the splat: every lane would add
                // zeros and keep its state (wave-uniform)
                if (QUAD) {
                    if (!__any(inc)) continue;
                    took = true;
                } else {
                    any |= inc;
                }
                // Recomputed transmittance: a pixel the splat does not reach
                // takes power -inf instead, so exp2 = 0, alpha = 0, 1 / (1 - alpha)
                // = 1 and its state passes through unchanged bit for bit (Tr x 1,
                // gR + gc x 0) with zero sums, without a select per quantity.
                const float ex = __builtin_amdgcn_exp2f(MODE == 2 || inc ? power2 : -__builtin_inff());
                const float ae = b.y * ex;
                const float alpha = fminf(kAlphaMax, ae);
                const float inv = __builtin_amdgcn_rcpf(1.f - alpha);   // alpha <= 0.99
                float Tb;
                if (MODE == 2)
                    Tb = inc ? tstore[(size_t)(bs + (uint32_t)j) * (T * T) + pix[k]] : 0.f;
                else
                    Tb = Tr[k] * inv;
                const float gc = fmaf(g2[k], c.x, fmaf(g1[k], b.w, g0[k] * b.z));
                const float dalpha = fmaf(Tb, gc, -(gR[k] * inv));
                const float wT = MODE != 2 || inc ? alpha * Tb : 0.f;
                acc[6] = fmaf(wT, g0[k], acc[6]);
                acc[7] = fmaf(wT, g1[k], acc[7]);
                acc[8] = fmaf(wT, g2[k], acc[8]);
                gR[k] = fmaf(gc, wT, gR[k]);
                if (MODE == 2) Tr[k] = inc ? Tb : Tr[k];
                else Tr[k] = Tb;
                // a clamped alpha passes no gradient to the opacity or the power;
                // te = dL/do, and dL/dpower (natural units) = o te, the opacity
                // factor being applied to the sums once per splat at the flush
                const bool open = (MODE != 2 || inc) & !(ae > kAlphaMax);
                const float te = open ? ex * dalpha : 0.f;
                acc[5] += te;
                const float ux = te * dx, uy = te * dy;
                acc[0] += ux;
                acc[1] += uy;
                acc[2] = fmaf(ux, dx, acc[2]);
                acc[3] = fmaf(ux, dy, acc[3]);
                acc[4] = fmaf(uy, dy, acc[4]);
            }
            return QUAD ? took : __any(any);
        };
        // Wave sums of the pair of splats (j + 1, j), j even, at once
        // (pair_sums); the row leaders store them into the wave's slots, and the
        // wave notes the splats some pixel took in its hit mask (a splat none
        // took is read as zero).
        auto store_pair = [&](int j, const float (&accA)[9], bool hitA, const float (&acc)[9],
                              bool hitj) {
            if (!(hitA || hitj)) return;
            float out[5];
            pair_sums(accA, acc, out);
            const int lane = __lane_id();
            if ((lane & 15) == 15) {
                const int row = lane >> 4, par = row & 1;
                const int js = row < 2 ? j + 1 : j;
                float *g = s_g + (threadIdx.x >> 6) * GS + (js & (R - 1)) * 9 + par;
                g[0] = out[0];
                g[2] = out[1];
                g[4] = out[2];
                g[6] = out[3];
                if (!par) g[8] = out[4];
            }
            if (hitA) hit |= 1ull << ((j + 1) & (R - 1));
            if (hitj) hit |= 1ull << (j & (R - 1));
        };
        // after splat j (even): at a multiple of R, splats j .. j + R - 1 are
        // done: one lane per splat adds the waves' sums, applies the conic
        // factors and stores them at the key's own position (no other workgroup
        // writes it)
        auto flush = [&](int j) {
            if ((j & (R - 1)) != 0) return;
            if (NW > 1) {
                if (__lane_id() == 0) s_hit[threadIdx.x >> 6] = hit;
                __syncthreads();
            }
            const int t = (int)threadIdx.x, jj = j + t;
            if (t < R && jj < nb) {
                float S[9];
#pragma unroll
                for (int f = 0; f < 9; f++) S[f] = 0.f;
#pragma unroll
                for (int w = 0; w < NW; w++) {
                    const uint64_t hw = NW > 1 ? s_hit[w] : hit;
                    if (!((hw >> t) & 1ull)) continue;
#pragma unroll
                    for (int f = 0; f < 9; f++) S[f] += s_g[w * GS + t * 9 + f];
                }
                const float A2 = s_a[jj].z, B2 = s_a[jj].w, C2 = s_b[jj].x, o = s_b[jj].y;
                const uint32_t q = s_q[jj];
#pragma unroll
                for (int f = 0; f < 5; f++) S[f] *= o;   // te sums -> dL/dpower sums
                // dpower/dmean = (A dx + B dy, B dx + C dy) = -ln2 (2 A2 dx + B2 dy, B2 dx + 2 C2 dy);
                // dpower/d(A, B, C) = (-dx^2 / 2, -dx dy, -dy^2 / 2)
                float4 *g = kp.pg + (size_t)q * kKeyGradF4;
                g[0] = make_float4(-kLn2 * (2.f * A2 * S[0] + B2 * S[1]),
                                   -kLn2 * (B2 * S[0] + 2.f * C2 * S[1]), -0.5f * S[2], -S[3]);
                g[1] = make_float4(-0.5f * S[4], S[5], S[6], S[7]);
                g[2] = make_float4(S[8], 0.f, 0.f, 0.f);
                g[3] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            if (NW > 1) __syncthreads();   // the slots are free again
            hit = 0ull;
        };
        // back to front by pairs (2 g + 1, 2 g), both splats' sums in registers
        // of their own; with an odd count the top splat (even) pairs with zeros
        int j = nb - 1;
        if (!(j & 1)) {
            float accA[9], acc[9];
#pragma unroll
            for (int f = 0; f < 9; f++) accA[f] = -0.f;
            const bool hitj = splat_terms(j, acc);
            store_pair(j, accA, false, acc, hitj);
            flush(j);
            j--;
        }
        for (; j > 0; j -= 2) {
            float accA[9], acc[9];
            const bool hitA = splat_terms(j, accA);
            const bool hitj = splat_terms(j - 1, acc);
            store_pair(j - 1, accA, hitA, acc, hitj);
            flush(j - 1);
        }
        be = bs;
    }
    // keys behind every pixel's last included splat pass no gradient
    for (uint32_t e = max(top, us) + threadIdx.x; e < ue; e += NT) {
        const uint32_t q = key_slot(kp, vals[e], ty, tx);
        float4 *g = kp.pg + (size_t)q * kKeyGradF4;
#pragma unroll
        for (int f = 0; f < kKeyGradF4; f++) g[f] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Recompute (MODE 0) and stored (MODE 2) modes: one workgroup per tile, the
// whole list back to front; workgroup i takes tile order[i] like the forward.
template <int T, int B, int MODE>
__global__ __launch_bounds__(bwd_threads<T>()) void k_render_bwd(
    const uint32_t *__restrict__ order,
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, const gsf_camera *__restrict__ cams,
    const float *__restrict__ tfinal, const uint32_t *__restrict__ ncontrib,
    const float *__restrict__ tstore, const float *__restrict__ bg, const float *__restrict__ dl,
    KeyPlace kp, TileMap tm) {
    constexpr int NT = bwd_threads<T>();
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];
    __shared__ float4 s_c[B];
    __shared__ uint32_t s_q[B];
    __shared__ uint8_t s_m[B];
    __shared__ float s_g[NT / 64 * kGradSlot<MODE>];
    __shared__ uint64_t s_hit[NT / 64];
    __shared__ float s_h[B];
    __shared__ uint32_t s_nmax[NT / 64];
    const uint32_t ti = order[blockIdx.x];
    const uint2 rg = ranges[ti];
    // a tile without keys passes no gradient (and a fovea-culled step's tiles
    // away from the fovea hold no pixel state to read)
    if (rg.x == rg.y) return;
    render_bwd_unit<T, B, MODE>(ti, tm, rg.x, rg.y, true, rg, vals, sp, views, nviews, cams, tfinal,
                                ncontrib, nullptr, nullptr, tstore, bg, dl, kp, s_a, s_b, s_c, s_q,
                                s_m, s_g, s_hit, s_h, s_nmax);
}

// Checkpoint mode: one workgroup per (tile, batch) unit id.  Unit u of tile t
// has id floor(start_t / B) + t + u (strictly increasing, below M / B + tiles);
// a workgroup maps its id back to its tile by binary search.  The grid covers
// the key capacity; ids at or above M / B + tiles (M read on the device) and
// ids that fall in no tile's units exit at once.
template <int T, int B>
__global__ __launch_bounds__(bwd_threads<T>()) void k_render_bwd_ckpt(
    const uint2 *__restrict__ ranges, int total_tiles, const uint32_t *__restrict__ m_dev,
    uint32_t m_host, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, const gsf_camera *__restrict__ cams,
    const float *__restrict__ tfinal, const uint32_t *__restrict__ ncontrib,
    const float4 *__restrict__ fstate, const float4 *__restrict__ ckpt,
    const float *__restrict__ bg, const float *__restrict__ dl, KeyPlace kp, TileMap tm) {
    constexpr int NT = bwd_threads<T>();
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];
    __shared__ float4 s_c[B];
    __shared__ uint32_t s_q[B];
    __shared__ uint8_t s_m[B];
    __shared__ float s_g[NT / 64 * kGradSlot<1>];
    __shared__ uint64_t s_hit[NT / 64];
    __shared__ float s_h[B];
    __shared__ uint32_t s_nmax[NT / 64];
    const uint32_t m = m_dev ? *m_dev : m_host;
    const uint32_t n_ids = m / B + (uint32_t)total_tiles;
    for (uint32_t id = blockIdx.x; id < n_ids; id += gridDim.x) {   // one trip when the grid covers n_ids
        // largest tile t with first id floor(start_t / B) + t <= id
        int lo = 0, hi = total_tiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ranges[mid].x / B + (uint32_t)mid <= id) lo = mid; else hi = mid - 1;
        }
        const uint2 rg = ranges[lo];
        const uint32_t u = id - (rg.x / B + (uint32_t)lo);
        const uint32_t units = (rg.y - rg.x + B - 1) / B;
        if (u >= units) continue;
        const uint32_t us = rg.x + u * B;
        const uint32_t ue = min(rg.y, us + B);
        render_bwd_unit<T, B, 1>((uint32_t)lo, tm, us, ue, u + 1 == units, rg, vals, sp, views, nviews, cams,
                                 tfinal, ncontrib, fstate, ckpt, nullptr, bg, dl, kp, s_a, s_b,
                                 s_c, s_q, s_m, s_g, s_hit, s_h, s_nmax);
    }
}

// Per-record sum of the per-key screen-space gradients into g2d [9][nrec]
// (wave_key_sum; one wave per workgroup, so that small record counts still
// spread over every CU).  The fit step sums inside the projection adjoint
// instead; this pass serves the debug readout of g2d.
__global__ __launch_bounds__(64) void k_grad_sum(KeyPlace kp, int nrec, float *__restrict__ g2d) {
    const int r = blockIdx.x * 64 + threadIdx.x;
    float S[9];
    wave_key_sum(kp, (uint32_t)r, r < nrec, S);
    if (r < nrec) {
#pragma unroll
        for (int f = 0; f < 9; f++) g2d[(size_t)f * nrec + r] = S[f];
    }
}

// Work accounting: the same per-pixel walk as k_render_fwd, counting instead
// of compositing.  counters: visited (forward), included, visited (adjoint).
template <int T>
__global__ __launch_bounds__(T * T < 256 ? T * T : 256) void k_count_pairs(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, TileMap tm, const float *__restrict__ cull_gaze,
    float cull_radius, unsigned long long *__restrict__ counters) {
    constexpr int NT = T * T < 256 ? T * T : 256;
    constexpr int PPT = T * T / NT;
    constexpr int ROWS = NT / T;
    __shared__ unsigned long long s_cnt[3];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0ull;
    __syncthreads();
    int v, ty, tx;
    ViewDesc vd;
    // the tiles and pixels the compositing kernels take (fovea-culled: the disk's)
    const bool valid = launch_tile(blockIdx.x, tm, views, nviews, T, v, vd, ty, tx) &&
                       (!tm.gaze || fovea_tile_live(tm.gaze, v, tm.radius, vd.width, vd.height, T, tx, ty));
    const float disk_r = cull_gaze ? cull_radius * (float)vd.width : 0.f;
    const uint2 rg = valid ? ranges[blockIdx.x] : make_uint2(0u, 0u);
    unsigned long long visit = 0, incl = 0, visit_bwd = 0;
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int x = tx * T + threadIdx.x % T, y = ty * T + threadIdx.x / T + k * ROWS;
        if (!(x < vd.width && y < vd.height)) continue;
        if (!in_fovea(cull_gaze, v, x, y, disk_r)) continue;
        const float px = (float)x, py = (float)y;
        float Tr = 1.f;
        uint32_t last = 0;
        for (uint32_t e = rg.x; e < rg.y; e++) {
            const uint32_t r = vals[e];
            visit++;
            float alpha, ae, ex, dx, dy;
            const float4 *rr = sp.at(r, 0);
            const float4 ra = rr[kRecA], rb = rr[kRecB], c = rr[kRecC];
            if (!splat_alpha(ra, rb, c, px, py, alpha, ae, ex, dx, dy)) continue;
            const float Tn = Tr * (1.f - alpha);
            if (Tn < kTStop) break;
            Tr = Tn;
            incl++;
            last = e - rg.x + 1u;
        }
        visit_bwd += last;
    }
    atomicAdd(&s_cnt[0], visit);
    atomicAdd(&s_cnt[1], incl);
    atomicAdd(&s_cnt[2], visit_bwd);
    __syncthreads();
    if (threadIdx.x < 3) atomicAdd(&counters[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ---- loss -----------------------------------------------------------------------

constexpr int kLossBlock = 256;
constexpr int kLossPx = 4;                         // pixels per thread of a loss launch
constexpr int kLossSpan = kLossBlock * kLossPx;    // pixels per block

__device__ __forceinline__ int view_of_pixel(const ViewDesc *__restrict__ views, int nviews, uint32_t p) {
    int v = 0;
    while (v + 1 < nviews && p >= (uint32_t)views[v + 1].pix_off) v++;
    return v;
}


// Blocks per view of a fovea-window loss launch: each view's box x box window
// is covered by whole blocks, so a block's view is uniform.
__host__ __device__ __forceinline__ int loss_blocks_per_view(int box) {
    return (box * box + kLossSpan - 1) / kLossSpan;
}

// Pixel t (< kLossSpan) of block bi of a loss launch: every pixel of every view
// (box == 0: pixel bi kLossSpan + t), or in view bi / bpv the pixel
// (bi mod bpv) kLossSpan + t of its box x box window, which starts at its
// first fovea tile (fovea culling; false for window pixels outside the view or
// past its last fovea tile).  f: the view's fovea tiles (box mode, computed once
// per block by the caller).  Plans hold fewer than 2^31 pixels: 32-bit
// arithmetic.
__device__ __forceinline__ bool loss_pixel(uint32_t bi, uint32_t t, uint32_t total_pix, int box,
                                           int tile, const FoveaTiles &f,
                                           const ViewDesc *__restrict__ views, int nviews, int &v,
                                           int &x, int &y) {
    if (box == 0) {
        const uint32_t p = bi * kLossSpan + t;
        if (p >= total_pix) return false;
        v = view_of_pixel(views, nviews, p);
        const ViewDesc vd = views[v];
        const uint32_t q = p - (uint32_t)vd.pix_off;
        y = (int)(q / (uint32_t)vd.width);
        x = (int)(q - (uint32_t)y * (uint32_t)vd.width);
        return true;
    }
    const int bpv = loss_blocks_per_view(box);
    v = (int)(bi / (uint32_t)bpv);
    if (v >= nviews || f.tx0 > f.tx1) return false;
    const uint32_t l = (bi - (uint32_t)v * (uint32_t)bpv) * kLossSpan + t;
    if (l >= (uint32_t)(box * box)) return false;
    // l / box by a float reciprocal: exact, since l < 2^23 and box < 2^12 keep the
    // quotient's fraction at least 1 / (2 box) from an integer
    const uint32_t ly = (uint32_t)(((float)l + 0.5f) * __builtin_amdgcn_rcpf((float)box));
    x = f.tx0 * tile + (int)(l - ly * (uint32_t)box);
    y = f.ty0 * tile + (int)ly;
    const ViewDesc vd = views[v];
    return x < vd.width && y < vd.height && x < (f.tx1 + 1) * tile && y < (f.ty1 + 1) * tile;
}

// The fovea tiles of block bi's view (box mode), computed once per block.
__device__ __forceinline__ FoveaTiles block_fovea(uint32_t bi, int box, int tile,
                                                  const float *__restrict__ gaze, float radius_frac,
                                                  const ViewDesc *__restrict__ views, int nviews,
                                                  FoveaTiles *s_f) {
    __syncthreads();   // s_f of the previous block is no longer read
    if (threadIdx.x == 0) {
        FoveaTiles f{1, 0, 1, 0};
        const int v = box ? (int)(bi / (uint32_t)loss_blocks_per_view(box)) : 0;
        if (box && v < nviews) {
            const ViewDesc vd = views[v];
            f = fovea_tiles(gaze, v, radius_frac, vd.width, vd.height, tile);
        }
        *s_f = f;
    }
    __syncthreads();
    return *s_f;
}

// The masked entries, one thread per (view, row of the pixels the loss visits):
// every pixel of the view (box == 0) or of its box x box window from its first
// fovea tile, clipped to the view and to the fovea tiles (as loss_pixel).  On a
// row the mask is an interval: in_fovea compares fl(dx)^2 + dy^2 with r^2, where
// dx = fl(x + 0.5 - gaze_x), and rounding is monotone, so the test can only turn
// false as |x + 0.5 - gaze_x| grows.  The row's pixel nearest the gaze column
// decides whether it has any, and a binary search each way (on that same test)
// finds the ends: the count equals the pixel-by-pixel count exactly.
__global__ __launch_bounds__(kLossBlock) void k_loss_count(const float *__restrict__ gaze,
                                                           float radius_frac,
                                                           const ViewDesc *__restrict__ views,
                                                           int nviews, int rows, int box, int tile,
                                                           uint32_t channels,
                                                           uint32_t *__restrict__ mask_count) {
    __shared__ uint32_t s_red[kLossBlock / 64];
    const uint32_t i = blockIdx.x * kLossBlock + threadIdx.x;
    const int v = (int)(i / (uint32_t)rows);
    const int row = (int)(i - (uint32_t)v * (uint32_t)rows);
    uint32_t n = 0u;
    if (v < nviews) {
        const ViewDesc vd = views[v];
        int x0 = 0, x1 = vd.width - 1, y = row;
        bool ok = row < vd.height;
        if (box) {
            const FoveaTiles f = fovea_tiles(gaze, v, radius_frac, vd.width, vd.height, tile);
            x0 = f.tx0 * tile;
            x1 = min(min((f.tx1 + 1) * tile, vd.width), x0 + box) - 1;
            y = f.ty0 * tile + row;
            ok = f.tx0 <= f.tx1 && y < min((f.ty1 + 1) * tile, vd.height);
        }
        if (ok) {
            const float rad = radius_frac * (float)vd.width;
            // the row's pixel nearest the gaze column (fmaxf takes x0 for a NaN gaze)
            const int xm = (int)fminf(fmaxf(rintf(gaze[2 * v] - 0.5f), (float)x0), (float)x1);
            if (in_fovea(gaze, v, xm, y, rad)) {
                int lo = xm, hi = x1 + 1;   // in at lo, out at hi (or past the row)
                while (hi - lo > 1) {
                    const int mid = lo + (hi - lo) / 2;
                    if (in_fovea(gaze, v, mid, y, rad)) lo = mid;
                    else hi = mid;
                }
                const int xr = lo;
                lo = x0 - 1;   // out at lo (or before the row), in at hi
                hi = xm;
                while (hi - lo > 1) {
                    const int mid = lo + (hi - lo) / 2;
                    if (in_fovea(gaze, v, mid, y, rad)) hi = mid;
                    else lo = mid;
                }
                n = (uint32_t)(xr - hi + 1) * channels;
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) n += (uint32_t)__shfl_xor((int)n, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0u;
#pragma unroll
        for (int w = 0; w < kLossBlock / 64; w++) tot += s_red[w];
        if (tot) atomicAdd(mask_count, tot);
    }
}

// Per-pixel L1 terms and sign gradient, and one partial sum per workgroup.
// The count of masked entries comes from mask_count (device) or count_host.
// (A last-workgroup-done reduction would need an agent-scope release fence per
// workgroup, which writes back the L2 just filled with dL/dRGBA; a second
// one-workgroup kernel is cheaper.)
__global__ __launch_bounds__(kLossBlock) void k_loss_l1(
    const float *__restrict__ rgba, const float *__restrict__ target, const float *__restrict__ gaze,
    float radius_frac, const ViewDesc *__restrict__ views, int nviews, int64_t total_pix, int box,
    int tile, int tgt_planes, bool alpha_term, const float *__restrict__ bg,
    const uint32_t *__restrict__ mask_count, uint32_t count_host, float *__restrict__ dl,
    float *__restrict__ partial) {
    __shared__ float s_red[kLossBlock / 64];
    __shared__ FoveaTiles s_f;
    const uint32_t cnt = mask_count ? *mask_count : count_host;
    const FoveaTiles f = box ? block_fovea(blockIdx.x, box, tile, gaze, radius_frac, views, nviews, &s_f)
                             : FoveaTiles{1, 0, 1, 0};
    float s = 0.f;
    const float inv = 1.f / (float)max(cnt, 1u);
    // kLossPx pixels per thread, kLossBlock apart (each step coalesced); all
    // their loads are issued before any is used
    bool ok[kLossPx], in[kLossPx];
    int vk[kLossPx];
    uint32_t qk[kLossPx], plk[kLossPx], offk[kLossPx];
    if (box) {   // the block's view is uniform: its descriptor is read once
        const int vb = min((int)(blockIdx.x / (uint32_t)loss_blocks_per_view(box)), nviews - 1);
        const ViewDesc vd = views[vb];
        const float rad = radius_frac * (float)vd.width;
#pragma unroll
        for (int k = 0; k < kLossPx; k++) {
            int v = 0, x = 0, y = 0;
            ok[k] = loss_pixel(blockIdx.x, (uint32_t)(k * kLossBlock) + threadIdx.x, (uint32_t)total_pix,
                               box, tile, f, views, nviews, v, x, y);
            vk[k] = vb;
            qk[k] = (uint32_t)(y * vd.width + x);
            plk[k] = (uint32_t)vd.width * (uint32_t)vd.height;
            offk[k] = (uint32_t)vd.pix_off;
            in[k] = ok[k] && in_fovea(gaze, vb, x, y, rad);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kLossPx; k++) {
            int v = 0, x = 0, y = 0;
            ok[k] = loss_pixel(blockIdx.x, (uint32_t)(k * kLossBlock) + threadIdx.x, (uint32_t)total_pix,
                               box, tile, f, views, nviews, v, x, y);
            const ViewDesc vd = views[ok[k] ? v : 0];
            vk[k] = v;
            qk[k] = (uint32_t)(y * vd.width + x);
            plk[k] = (uint32_t)vd.width * (uint32_t)vd.height;
            offk[k] = (uint32_t)vd.pix_off;
            in[k] = ok[k] && in_fovea(gaze, v, x, y, radius_frac * (float)vd.width);
        }
    }
    // RGBA targets: colour premultiplied, composited over the view background.
    // A pixel outside the mask reads nothing (a fovea-culled forward did not
    // composite it) and gets a zero gradient - written only on full frames:
    // after a fovea-culled forward (box > 0) the adjoint does not read it (no
    // splat reached the pixel).
    float im[kLossPx][4], tg[kLossPx][4], bk[kLossPx][3];
#pragma unroll
    for (int k = 0; k < kLossPx; k++) {
        const size_t plane = plk[k], q = qk[k];
        const float *img = rgba + 4 * (size_t)offk[k];
        const float *tgt = target + (size_t)tgt_planes * offk[k];
        if (in[k]) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                im[k][c] = img[c * plane + q];
                tg[k][c] = tgt[c * plane + q];
            }
            im[k][3] = alpha_term ? img[3 * plane + q] : 0.f;
            tg[k][3] = tgt_planes == 4 || alpha_term ? tgt[3 * plane + q] : 1.f;
            if (bg) {
#pragma unroll
                for (int c = 0; c < 3; c++) bk[k][c] = bg[3 * vk[k] + c];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kLossPx; k++) {
        if (!(ok[k] && (in[k] || !box))) continue;
        const size_t plane = plk[k], q = qk[k];
        float *g = dl + 4 * (size_t)offk[k];
        const float ta = in[k] && tgt_planes == 4 ? tg[k][3] : 1.f;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            float gv = 0.f;
            if (in[k] && (c < 3 || alpha_term)) {
                float t = tg[k][c];
                if (c < 3 && bg) t = fmaf(1.f - ta, bk[k][c], t);
                const float d = im[k][c] - t;
                s += fabsf(d);
                gv = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            }
            g[c * plane + q] = gv;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);   // fixed tree: deterministic
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < kLossBlock / 64; w++) tot += s_red[w];
        partial[blockIdx.x] = tot;
    }
}

// Sum of the partials in a fixed order (deterministic) -> loss; optionally
// advances the optimiser step counter (the fit step's Adam runs after it).
__global__ __launch_bounds__(1024) void k_loss_final(const float *__restrict__ partial, int nparts,
                                                     const uint32_t *__restrict__ mask_count,
                                                     uint32_t count_host, float *__restrict__ loss,
                                                     uint32_t *__restrict__ flags,
                                                     int32_t *__restrict__ step_inc, bool accumulate) {
    __shared__ float s_part[16];
    // four partials per thread and step (16-byte loads; the tail one by one),
    // in four sums: a fixed order, so the loss is deterministic
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    const int n4 = nparts / 4;
    for (int k = threadIdx.x; k < n4; k += 1024) {
        const float4 v = reinterpret_cast<const float4 *>(partial)[k];
        s0 += v.x;
        s1 += v.y;
        s2 += v.z;
        s3 += v.w;
    }
    for (int k = 4 * n4 + (int)threadIdx.x; k < nparts; k += 1024) s0 += partial[k];
    float s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);   // same tree on every lane
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < 16; w++) tot += s_part[w];
        const uint32_t cnt = mask_count ? *mask_count : count_host;
        const float L = tot / (float)max(cnt, 1u);
        loss[0] = accumulate ? loss[0] + L : L;   // accumulate: one share of a multi-plan loss
        if (!isfinite(L)) atomicOr(flags, GSF_FLAG_NONFINITE);
        // a step whose keys overflowed the capacity is not counted (its Adam
        // update is skipped too, so it can be repeated after a re-plan)
        if (step_inc && !(*flags & GSF_FLAG_CAPACITY)) step_inc[0] = step_inc[0] + 1;
    }
}

// Per-view random background: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
// output k = 1 + (step * kMaxViews + v) * 4 + c from state seed, i.e. the
// state seed + k * golden-ratio increment passed through the published
// finaliser; the top 24 bits scaled to [0, 1) (exact in float).
__global__ void k_draw_bg(uint64_t seed, const int32_t *__restrict__ step, int nviews,
                          float *__restrict__ bg) {
    const int e = threadIdx.x;
    if (e >= 3 * nviews) return;
    const int v = e / 3, c = e - 3 * v;
    const uint64_t k = 1ull + ((uint64_t)step[0] * kMaxViews + (uint64_t)v) * 4ull + (uint64_t)c;
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    bg[e] = (float)(uint32_t)(z >> 40) * (1.f / 16777216.f);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t value) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = value;
}

__global__ void k_fill_f32(float *p, int64_t n, float value) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = value;
}

template <int T, int B, bool SPLIT>
void render_fwd_tbs(hipStream_t s, const RenderArgs &a, float *out) {
    constexpr int NT = fwd_threads<T, SPLIT>();
    const int g = SPLIT ? 4 * ((a.total_tiles + 7) / 8 * 8) : a.total_tiles;
    if (a.t_mode == 1)
        k_render_fwd<T, B, 1, SPLIT><<<g, NT, 0, s>>>(a.order, a.ranges, a.vals, a.sp, a.views,
                                                     a.nviews, a.cams, out, a.tfinal, a.ncontrib, a.ckpt,
                                                     a.fstate, nullptr, a.bg, a.cull_gaze, a.cull_radius,
                                                     a.total_tiles, a.tm);
    else if (a.t_mode == 2)
        k_render_fwd<T, B, 2, SPLIT><<<g, NT, 0, s>>>(a.order, a.ranges, a.vals, a.sp, a.views,
                                                     a.nviews, a.cams, out, a.tfinal, a.ncontrib, nullptr,
                                                     nullptr, a.tstore, a.bg, a.cull_gaze, a.cull_radius,
                                                     a.total_tiles, a.tm);
    else
        k_render_fwd<T, B, 0, SPLIT><<<g, NT, 0, s>>>(a.order, a.ranges, a.vals, a.sp, a.views,
                                                     a.nviews, a.cams, out, a.tfinal, a.ncontrib, nullptr,
                                                     nullptr, nullptr, a.bg, a.cull_gaze, a.cull_radius,
                                                     a.total_tiles, a.tm);
}

// Split 16-pixel tiles into one workgroup per quadrant when the plan has at
// most kSplitTilesPerCu tiles per compute unit: measured on one 1024^2 view
// (4096 tiles) it shortens the forward by 5%, on 16 views of 1920^2 (230k
// tiles) it lengthens it by 2.5% and on 8 views of 0.25-4 Mpix (63k tiles)
// by 6-18%.
constexpr int kSplitTilesPerCu = 16;

template <int T, int B>
void render_fwd_tb(hipStream_t s, const RenderArgs &a, float *out) {
    if (T == 16 && (int64_t)a.total_tiles <= (int64_t)kSplitTilesPerCu * a.cus)
        render_fwd_tbs<T, B, T == 16>(s, a, out);
    else
        render_fwd_tbs<T, B, false>(s, a, out);
}

template <int T, int B>
void render_bwd_tb(hipStream_t s, const RenderArgs &a, const float *dl) {
    constexpr int NT = bwd_threads<T>();
    if (a.t_mode == 1)
        k_render_bwd_ckpt<T, B><<<a.bwd_grid, NT, 0, s>>>(a.ranges, a.total_tiles, a.m_dev, a.m_host,
                                                         a.vals, a.sp, a.views, a.nviews, a.cams,
                                                         a.tfinal, a.ncontrib, a.fstate, a.ckpt, a.bg,
                                                         dl, a.kp, a.tm);
    else if (a.t_mode == 2)
        k_render_bwd<T, B, 2><<<a.total_tiles, NT, 0, s>>>(a.order, a.ranges, a.vals, a.sp,
                                                        a.views, a.nviews, a.cams, a.tfinal,
                                                        a.ncontrib, a.tstore, a.bg, dl, a.kp, a.tm);
    else
        k_render_bwd<T, B, 0><<<a.total_tiles, NT, 0, s>>>(a.order, a.ranges, a.vals, a.sp,
                                                        a.views, a.nviews, a.cams, a.tfinal,
                                                        a.ncontrib, nullptr, a.bg, dl, a.kp, a.tm);
}

template <int T>
void render_fwd_t(hipStream_t s, const RenderArgs &a, float *out) {
    if (a.batch == 64) render_fwd_tb<T, 64>(s, a, out);
    else if (a.batch == 128) render_fwd_tb<T, 128>(s, a, out);
    else render_fwd_tb<T, 256>(s, a, out);
}

template <int T>
void render_bwd_t(hipStream_t s, const RenderArgs &a, const float *dl) {
    if (a.batch == 64) render_bwd_tb<T, 64>(s, a, dl);
    else if (a.batch == 128) render_bwd_tb<T, 128>(s, a, dl);
    else render_bwd_tb<T, 256>(s, a, dl);
}

}  // namespace

void launch_render_fwd(hipStream_t s, const RenderArgs &a, float *out_rgba) {
    if (a.tile == 8) render_fwd_t<8>(s, a, out_rgba);
    else if (a.tile == 16) render_fwd_t<16>(s, a, out_rgba);
    else render_fwd_t<32>(s, a, out_rgba);
}

void launch_render_bwd(hipStream_t s, const RenderArgs &a, const float *dl_drgba) {
    if (a.tile == 8) render_bwd_t<8>(s, a, dl_drgba);
    else if (a.tile == 16) render_bwd_t<16>(s, a, dl_drgba);
    else render_bwd_t<32>(s, a, dl_drgba);
}

void launch_grad_sum(hipStream_t s, const KeyPlace &kp, int nrec, float *g2d) {
    if (nrec <= 0) return;
    k_grad_sum<<<(nrec + 63) / 64, 64, 0, s>>>(kp, nrec, g2d);
}

void launch_count_pairs(hipStream_t s, int tile, int total_tiles, const uint2 *ranges,
                        const uint32_t *vals, SplatPtrs sp, const ViewDesc *views, int nviews,
                        const TileMap &tm, const float *cull_gaze, float cull_radius,
                        unsigned long long *counters) {
    k_zero_u64<<<1, 64, 0, s>>>(counters, 3);
    if (tile == 8)
        k_count_pairs<8><<<total_tiles, 64, 0, s>>>(ranges, vals, sp, views, nviews, tm, cull_gaze, cull_radius, counters);
    else if (tile == 16)
        k_count_pairs<16><<<total_tiles, 256, 0, s>>>(ranges, vals, sp, views, nviews, tm, cull_gaze, cull_radius, counters);
    else
        k_count_pairs<32><<<total_tiles, 256, 0, s>>>(ranges, vals, sp, views, nviews, tm, cull_gaze, cull_radius, counters);
}

// Partial sums of a loss launch: one per block (a fovea-window launch's views
// are padded to whole blocks, at most one more block per view).
int loss_partials(int64_t total_pix) {
    return (int)((total_pix + kLossBlock - 1) / kLossBlock) + kMaxViews;
}

int loss_launch_blocks(int64_t total_pix, int nviews, int box) {
    return box ? nviews * loss_blocks_per_view(box) : (int)((total_pix + kLossSpan - 1) / kLossSpan);
}

void launch_loss_l1(hipStream_t s, const float *rgba, const float *target, const float *gaze,
                    float radius_frac, const ViewDesc *views, int nviews, int64_t total_pix,
                    float *dl, float *partial, uint32_t *mask_count, float *loss, uint32_t *flags,
                    int32_t *step_inc, int box, int tile, int tgt_planes, bool alpha_term,
                    const float *bg, uint32_t norm_count, bool accumulate, int max_height) {
    if (!gaze) box = 0;
    const uint32_t channels = alpha_term ? 4u : 3u;
    const int nb = loss_launch_blocks(total_pix, nviews, box);
    if (gaze && norm_count == 0u)
        launch_loss_count(s, gaze, radius_frac, views, nviews, max_height, box, tile, channels,
                          mask_count);
    const uint32_t *mc = gaze && norm_count == 0u ? mask_count : nullptr;
    const uint32_t cnt = norm_count ? norm_count : (uint32_t)(channels * total_pix);
    k_loss_l1<<<nb, kLossBlock, 0, s>>>(rgba, target, gaze, radius_frac, views, nviews, total_pix, box,
                                        tile, tgt_planes, alpha_term, bg, mc, cnt, dl, partial);
    k_loss_final<<<1, 1024, 0, s>>>(partial, nb, mc, cnt, loss, flags, step_inc, accumulate);
}

void launch_loss_count(hipStream_t s, const float *gaze, float radius_frac, const ViewDesc *views,
                       int nviews, int max_height, int box, int tile, uint32_t channels,
                       uint32_t *mask_count) {
    const int rows = box ? box : max_height;
    const int64_t threads = (int64_t)nviews * rows;
    k_fill_u32<<<1, 64, 0, s>>>(mask_count, 1, 0u);
    if (threads > 0)
        k_loss_count<<<(int)((threads + kLossBlock - 1) / kLossBlock), kLossBlock, 0, s>>>(
            gaze, radius_frac, views, nviews, rows, box, tile, channels, mask_count);
}

void launch_draw_bg(hipStream_t s, uint64_t seed, const int32_t *step, int nviews, float *bg) {
    k_draw_bg<<<1, 3 * kMaxViews, 0, s>>>(seed, step, nviews, bg);
}

void launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t value) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    k_fill_u32<<<(int)g, 256, 0, s>>>(p, n, value);
}

void launch_fill_f32(hipStream_t s, float *p, int64_t n, float value) {
    if (n <= 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    k_fill_f32<<<(int)g, 256, 0, s>>>(p, n, value);
}

}  // namespace gsf
