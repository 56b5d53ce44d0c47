// raster.hip - per-tile front-to-back alpha compositing, its back-to-front
// adjoint, and the masked L1 image loss.
//
// One workgroup per screen tile (T x T pixels, T in {8, 16, 32}); one thread
// per pixel (T = 32: four pixels per thread).  The tile's depth-ordered list of
// splats is staged through LDS in batches of B records (B in {64, 128, 256})
// that every wave then reads by broadcast.  Per pixel and splat:
//   power = -(A dx^2 + C dy^2) / 2 - B dx dy, skip if power > 0;
//   alpha = min(0.99, o e^power), skip if alpha < 1/255;
//   stop before the splat if T (1 - alpha) < 1e-4;
//   C += colour alpha T;  T *= 1 - alpha.
// A wave leaves the batch loop once all its pixels have stopped and the
// workgroup leaves the tile once all waves have.  Because a pixel's arithmetic
// sequence does not depend on T, B or the tile's other pixels, images are
// bitwise independent of the tile size and the batch size.
//
// The adjoint walks the same list back to front from each pixel's last
// included splat, rebuilding the transmittance in front of each splat as
// T_i = T_{i+1} / (1 - alpha_i) from the stored final transmittance.  The nine
// per-splat screen-space gradient terms of a wave are summed across lanes,
// added into an LDS accumulator per batch entry, and flushed with one global
// atomic per (tile, splat, field).
#include "gs_internal.h"

namespace gsf {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

// Shared by the forward and backward kernels so both take identical decisions.
__device__ __forceinline__ bool splat_alpha(const float4 &a, const float4 &b, float px, float py,
                                            float &alpha, float &ae, float &ex, float &dx,
                                            float &dy) {
    dx = px - a.x;
    dy = py - a.y;
    const float q = fmaf(a.z * dx, dx, (b.x * dy) * dy);
    const float power = fmaf(-0.5f, q, -((a.w * dx) * dy));
    if (power > 0.f) return false;
    ex = __builtin_amdgcn_exp2f(power * kLog2e);
    ae = b.y * ex;
    alpha = fminf(kAlphaMax, ae);
    return alpha >= kAlphaMin;
}

__device__ __forceinline__ int view_of_tile(const ViewDesc *__restrict__ views, int nviews, int gt) {
    int v = 0;
    while (v + 1 < nviews && gt >= views[v + 1].tile_off) v++;
    return v;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int T, int B>
__global__ __launch_bounds__(T * T < 256 ? T * T : 256) void k_render_fwd(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, const gsf_camera *__restrict__ cams,
    float *__restrict__ out_rgba, float *__restrict__ tfinal, uint32_t *__restrict__ ncontrib) {
    constexpr int NT = T * T < 256 ? T * T : 256;
    constexpr int PPT = T * T / NT;
    constexpr int ROWS = NT / T;
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];
    __shared__ float s_c[B];

    const int gt = blockIdx.x;
    const int v = view_of_tile(views, nviews, gt);
    const ViewDesc vd = views[v];
    const int local = gt - vd.tile_off;
    const int ty = local / vd.tiles_x, tx = local - ty * vd.tiles_x;
    const uint2 rg = ranges[gt];
    const int lx = threadIdx.x % T, ly = threadIdx.x / T;

    float px[PPT], py[PPT], Tr[PPT], cr[PPT], cg[PPT], cb[PPT];
    uint32_t last[PPT];
    bool done[PPT];
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int x = tx * T + lx, y = ty * T + ly + k * ROWS;
        done[k] = !(x < vd.width && y < vd.height);
        px[k] = (float)x + 0.5f;
        py[k] = (float)y + 0.5f;
        Tr[k] = 1.f;
        cr[k] = cg[k] = cb[k] = 0.f;
        last[k] = 0u;
    }

    for (uint32_t bs = rg.x; bs < rg.y; bs += B) {
        const int nb = (int)min((uint32_t)B, rg.y - bs);
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += NT) {
            const uint32_t r = vals[bs + j];
            s_a[j] = sp.a[r];
            s_b[j] = sp.b[r];
            s_c[j] = sp.c[r];
        }
        __syncthreads();
        for (int j = 0; j < nb; j++) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < PPT; k++) all &= done[k];
            if (__all(all)) break;
            const float4 a = s_a[j];
            const float4 b = s_b[j];
            const float c2 = s_c[j];
#pragma unroll
            for (int k = 0; k < PPT; k++) {
                if (done[k]) continue;
                float alpha, ae, ex, dx, dy;
                if (!splat_alpha(a, b, px[k], py[k], alpha, ae, ex, dx, dy)) continue;
                const float Tn = Tr[k] * (1.f - alpha);
                if (Tn < kTStop) {
                    done[k] = true;
                    continue;
                }
                const float w = alpha * Tr[k];
                cr[k] = fmaf(b.z, w, cr[k]);
                cg[k] = fmaf(b.w, w, cg[k]);
                cb[k] = fmaf(c2, w, cb[k]);
                Tr[k] = Tn;
                last[k] = bs + (uint32_t)j - rg.x + 1u;
            }
        }
        bool all = true;
#pragma unroll
        for (int k = 0; k < PPT; k++) all &= done[k];
        if (__syncthreads_and(all)) break;
    }

    const gsf_camera &cam = cams[v];
    const float bg0 = cam.bg[0], bg1 = cam.bg[1], bg2 = cam.bg[2];
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
    }
}

template <int T, int B>
__global__ __launch_bounds__(T * T < 256 ? T * T : 256) void k_render_bwd(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, SplatPtrs sp,
    const ViewDesc *__restrict__ views, int nviews, const gsf_camera *__restrict__ cams,
    const float *__restrict__ tfinal, const uint32_t *__restrict__ ncontrib,
    const float *__restrict__ dl, float *__restrict__ g2d, int nrec) {
    constexpr int NT = T * T < 256 ? T * T : 256;
    constexpr int PPT = T * T / NT;
    constexpr int ROWS = NT / T;
    __shared__ float4 s_a[B];
    __shared__ float4 s_b[B];
    __shared__ float s_c[B];
    __shared__ uint32_t s_r[B];
    __shared__ float s_g[B * 9];
    __shared__ uint32_t s_nmax;

    const int gt = blockIdx.x;
    const int v = view_of_tile(views, nviews, gt);
    const ViewDesc vd = views[v];
    const int local = gt - vd.tile_off;
    const int ty = local / vd.tiles_x, tx = local - ty * vd.tiles_x;
    const uint2 rg = ranges[gt];
    const int lx = threadIdx.x % T, ly = threadIdx.x / T;
    const gsf_camera &cam = cams[v];
    const float bg0 = cam.bg[0], bg1 = cam.bg[1], bg2 = cam.bg[2];
    const size_t plane = (size_t)vd.width * vd.height;
    const float *dimg = dl + 4 * (size_t)vd.pix_off;

    float px[PPT], py[PPT], Tr[PPT], Tf[PPT], gR[PPT], g0[PPT], g1[PPT], g2[PPT], gA[PPT];
    uint32_t nc[PPT];
    uint32_t my_max = 0;
#pragma unroll
    for (int k = 0; k < PPT; k++) {
        const int x = tx * T + lx, y = ty * T + ly + k * ROWS;
        px[k] = (float)x + 0.5f;
        py[k] = (float)y + 0.5f;
        if (x < vd.width && y < vd.height) {
            const size_t q = (size_t)y * vd.width + x;
            Tf[k] = tfinal[vd.pix_off + q];
            nc[k] = ncontrib[vd.pix_off + q];
            g0[k] = dimg[q];
            g1[k] = dimg[plane + q];
            g2[k] = dimg[2 * plane + q];
            gA[k] = dimg[3 * plane + q];
        } else {
            Tf[k] = 1.f;
            nc[k] = 0u;
            g0[k] = g1[k] = g2[k] = gA[k] = 0.f;
        }
        Tr[k] = Tf[k];
        gR[k] = Tf[k] * (g0[k] * bg0 + g1[k] * bg1 + g2[k] * bg2);
        my_max = max(my_max, nc[k]);
    }
    if (threadIdx.x == 0) s_nmax = 0u;
    __syncthreads();
    atomicMax(&s_nmax, my_max);
    __syncthreads();
    const uint32_t nmax = s_nmax;

    for (uint32_t be = rg.x + nmax; be > rg.x;) {
        const uint32_t bs = be - rg.x > (uint32_t)B ? be - (uint32_t)B : rg.x;
        const int nb = (int)(be - bs);
        __syncthreads();
        for (int j = threadIdx.x; j < nb; j += NT) {
            const uint32_t r = vals[bs + j];
            s_a[j] = sp.a[r];
            s_b[j] = sp.b[r];
            s_c[j] = sp.c[r];
            s_r[j] = r;
        }
        for (int e = threadIdx.x; e < nb * 9; e += NT) s_g[e] = 0.f;
        __syncthreads();
        for (int j = nb - 1; j >= 0; j--) {
            const uint32_t pos = bs + (uint32_t)j - rg.x;   // list position in the tile
            const float4 a = s_a[j];
            const float4 b = s_b[j];
            const float c2 = s_c[j];
            float acc[9];
#pragma unroll
            for (int f = 0; f < 9; f++) acc[f] = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPT; k++) {
                if (pos >= nc[k]) continue;
                float alpha, ae, ex, dx, dy;
                if (!splat_alpha(a, b, px[k], py[k], alpha, ae, ex, dx, dy)) continue;
                any = true;
                const float oma = 1.f - alpha;
                const float Tb = Tr[k] / oma;
                const float gc = g0[k] * b.z + g1[k] * b.w + g2[k] * c2;
                const float dalpha = (Tb * gc - gR[k] / oma) + gA[k] * Tf[k] / oma;
                const float wT = alpha * Tb;
                acc[6] += wT * g0[k];
                acc[7] += wT * g1[k];
                acc[8] += wT * g2[k];
                gR[k] = fmaf(gc, wT, gR[k]);
                Tr[k] = Tb;
                if (ae > kAlphaMax) continue;      // clamped alpha: no gradient to o, power
                const float dpw = ae * dalpha;
                acc[5] += ex * dalpha;
                acc[2] += -0.5f * dx * dx * dpw;
                acc[3] += -dx * dy * dpw;
                acc[4] += -0.5f * dy * dy * dpw;
                acc[0] += (a.z * dx + a.w * dy) * dpw;
                acc[1] += (a.w * dx + b.x * dy) * dpw;
            }
            if (__any(any)) {
#pragma unroll
                for (int f = 0; f < 9; f++) {
                    const float sum = wave_sum(acc[f]);
                    if (__lane_id() == 0 && sum != 0.f) atomicAdd(&s_g[j * 9 + f], sum);
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * 9; e += NT) {
            const float val = s_g[e];
            if (val != 0.f) {
                const int j = e / 9, f = e - 9 * (e / 9);
                unsafeAtomicAdd(&g2d[(size_t)f * nrec + s_r[j]], val);
            }
        }
        be = bs;
    }
}

// ---- loss -----------------------------------------------------------------------

constexpr int kLossBlock = 256;

__device__ __forceinline__ int view_of_pixel(const ViewDesc *__restrict__ views, int nviews, int64_t p) {
    int v = 0;
    while (v + 1 < nviews && p >= views[v + 1].pix_off) v++;
    return v;
}

__device__ __forceinline__ bool in_fovea(const float *__restrict__ gaze, int v, int x, int y,
                                         float radius) {
    if (!gaze) return true;
    const float dx = (float)x + 0.5f - gaze[2 * v], dy = (float)y + 0.5f - gaze[2 * v + 1];
    return dx * dx + dy * dy <= radius * radius;
}

__global__ __launch_bounds__(kLossBlock) void k_loss_count(const float *__restrict__ gaze,
                                                           float radius_frac,
                                                           const ViewDesc *__restrict__ views,
                                                           int nviews, int64_t total_pix,
                                                           uint32_t *__restrict__ mask_count) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
    if (p < total_pix) {
        const int v = view_of_pixel(views, nviews, p);
        const ViewDesc vd = views[v];
        const int q = (int)(p - vd.pix_off);
        const int y = q / vd.width, x = q - y * vd.width;
        if (in_fovea(gaze, v, x, y, radius_frac * (float)vd.width)) atomicAdd(&s_cnt, 3u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(mask_count, s_cnt);
}

__global__ __launch_bounds__(kLossBlock) void k_loss_l1(const float *__restrict__ rgba,
                                                        const float *__restrict__ target,
                                                        const float *__restrict__ gaze,
                                                        float radius_frac,
                                                        const ViewDesc *__restrict__ views,
                                                        int nviews, int64_t total_pix,
                                                        const uint32_t *__restrict__ mask_count,
                                                        float *__restrict__ dl,
                                                        float *__restrict__ partial) {
    __shared__ float s_wave[kLossBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
    float s = 0.f;
    if (p < total_pix) {
        const int v = view_of_pixel(views, nviews, p);
        const ViewDesc vd = views[v];
        const int q = (int)(p - vd.pix_off);
        const int y = q / vd.width, x = q - y * vd.width;
        const size_t plane = (size_t)vd.width * vd.height;
        const float *img = rgba + 4 * (size_t)vd.pix_off;
        const float *tgt = target + 3 * (size_t)vd.pix_off;
        float *g = dl + 4 * (size_t)vd.pix_off;
        const bool in = in_fovea(gaze, v, x, y, radius_frac * (float)vd.width);
        const float inv = 1.f / (float)max(*mask_count, 1u);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float d = img[c * plane + q] - tgt[c * plane + q];
            float gv = 0.f;
            if (in) {
                s += fabsf(d);
                gv = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            }
            g[c * plane + q] = gv;
        }
        g[3 * plane + q] = 0.f;
    }
    // deterministic block reduction
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (__lane_id() == 0) s_wave[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < kLossBlock / 64; w++) t += s_wave[w];
        partial[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_loss_final(const float *__restrict__ partial, int nparts,
                                                     const uint32_t *__restrict__ mask_count,
                                                     float *__restrict__ loss,
                                                     uint32_t *__restrict__ flags) {
    __shared__ float s_part[1024];
    float s = 0.f;
    for (int k = threadIdx.x; k < nparts; k += 1024) s += partial[k];
    s_part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (threadIdx.x < o) s_part[threadIdx.x] += s_part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float L = s_part[0] / (float)max(*mask_count, 1u);
        loss[0] = L;
        if (!isfinite(L)) atomicOr(flags, GSF_FLAG_NONFINITE);
    }
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

template <int T>
void render_fwd_t(hipStream_t s, int batch, int total_tiles, const uint2 *ranges, const uint32_t *vals,
                  SplatPtrs sp, const ViewDesc *views, int nviews, const gsf_camera *cams,
                  float *out, float *tfinal, uint32_t *ncontrib) {
    constexpr int NT = T * T < 256 ? T * T : 256;
    if (batch == 64)
        k_render_fwd<T, 64><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, out, tfinal, ncontrib);
    else if (batch == 128)
        k_render_fwd<T, 128><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, out, tfinal, ncontrib);
    else
        k_render_fwd<T, 256><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, out, tfinal, ncontrib);
}

template <int T>
void render_bwd_t(hipStream_t s, int batch, int total_tiles, const uint2 *ranges, const uint32_t *vals,
                  SplatPtrs sp, const ViewDesc *views, int nviews, const gsf_camera *cams,
                  const float *tfinal, const uint32_t *ncontrib, const float *dl, float *g2d, int nrec) {
    constexpr int NT = T * T < 256 ? T * T : 256;
    if (batch == 64)
        k_render_bwd<T, 64><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl, g2d, nrec);
    else if (batch == 128)
        k_render_bwd<T, 128><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl, g2d, nrec);
    else
        k_render_bwd<T, 256><<<total_tiles, NT, 0, s>>>(ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl, g2d, nrec);
}

}  // namespace

void launch_render_fwd(hipStream_t s, int tile, int batch, int total_tiles, const uint2 *ranges,
                       const uint32_t *vals, SplatPtrs sp, const ViewDesc *views, int nviews,
                       const gsf_camera *cams, float *out_rgba, float *tfinal, uint32_t *ncontrib) {
    if (tile == 8)
        render_fwd_t<8>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, out_rgba, tfinal, ncontrib);
    else if (tile == 16)
        render_fwd_t<16>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, out_rgba, tfinal, ncontrib);
    else
        render_fwd_t<32>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, out_rgba, tfinal, ncontrib);
}

void launch_render_bwd(hipStream_t s, int tile, int batch, int total_tiles, const uint2 *ranges,
                       const uint32_t *vals, SplatPtrs sp, const ViewDesc *views, int nviews,
                       const gsf_camera *cams, const float *tfinal, const uint32_t *ncontrib,
                       const float *dl_drgba, float *g2d, int nrec) {
    if (tile == 8)
        render_bwd_t<8>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl_drgba, g2d, nrec);
    else if (tile == 16)
        render_bwd_t<16>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl_drgba, g2d, nrec);
    else
        render_bwd_t<32>(s, batch, total_tiles, ranges, vals, sp, views, nviews, cams, tfinal, ncontrib, dl_drgba, g2d, nrec);
}

int loss_partials(int64_t total_pix) { return (int)((total_pix + kLossBlock - 1) / kLossBlock); }

void launch_loss_l1(hipStream_t s, const float *rgba, const float *target, const float *gaze,
                    float radius_frac, const ViewDesc *views, int nviews, int64_t total_pix,
                    float *dl, float *partial, uint32_t *mask_count, float *loss, uint32_t *flags) {
    const int nb = loss_partials(total_pix);
    if (gaze) {
        k_fill_u32<<<1, 64, 0, s>>>(mask_count, 1, 0u);
        k_loss_count<<<nb, kLossBlock, 0, s>>>(gaze, radius_frac, views, nviews, total_pix, mask_count);
    } else {
        k_fill_u32<<<1, 64, 0, s>>>(mask_count, 1, (uint32_t)(3 * total_pix));
    }
    k_loss_l1<<<nb, kLossBlock, 0, s>>>(rgba, target, gaze, radius_frac, views, nviews, total_pix,
                                        mask_count, dl, partial);
    k_loss_final<<<1, 1024, 0, s>>>(partial, nb, mask_count, loss, flags);
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
