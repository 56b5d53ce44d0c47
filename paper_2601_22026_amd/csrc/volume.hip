// volume.hip - the steps around the fit that read the CT volume on the device:
// seeding Gaussians from it and ray-marching target images through it
// (Method, "Volumetric Path Tracing" renders the views the peripheral model is
// fitted to; "Periphery Model Training" builds that model from Gaussians
// seeded on the volume's structures).
//
// Seeding: one Gaussian per voxel whose value exceeds the threshold, in raster
// order (vol[ix][iy][iz], flat index (ix n + iy) n + iz); when there are more
// than cap candidates the cap with the smallest priority are kept, still in
// raster order.  Priority of voxel idx: the SplitMix64 output idx + 1 from
// state seed with its low b bits replaced by idx (b = bits of n^3 - 1), so
// priorities are distinct and the kept set is a uniform random subset.  The
// cap-th smallest priority is found by an MSB-first radix select (eight 8-bit
// digit histograms), then the kept voxels are written in raster order.  Mean =
// voxel centre, isotropic log-scale, identity rotation, the given opacity and
// the transfer-function colour as degree-0 SH, in double precision rounded
// once to float.
//
// Ray march: one thread per pixel, emission-absorption through the box
// [-1, 1]^3 in float32 - segments of the step length from the box entry (the
// last shortened to the exit), the trilinear sample (zero outside the grid) at
// each segment's midpoint, density t = clamp((v - thr) / range, 0, 1), colour
// lerp(lo, hi, t), alpha = 1 - exp(-extinction t length), stop once T < t_stop;
// RGB = C + T bg, A = 1 - T.
#include <cmath>
#include <vector>

#include "gs_internal.h"

namespace gsf {
namespace {

constexpr int kVolBlock = 256;
constexpr int kVolIpt = 8;                       // voxels per thread per block
constexpr int kVolTile = kVolBlock * kVolIpt;

__device__ __forceinline__ uint64_t splitmix64(uint64_t state, uint64_t k) {
    uint64_t z = state + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t priority(uint64_t seed, uint64_t idx, int ibits) {
    return ((splitmix64(seed, idx + 1ull) >> ibits) << ibits) | idx;
}

// Digit histogram of the candidates whose priority agrees with `prefix` on the
// bits above `shift + 8`; 256 bins accumulated per workgroup in LDS.
__global__ __launch_bounds__(kVolBlock) void k_seed_hist(const uint16_t *__restrict__ vol, int64_t nvox,
                                                         float thr, uint64_t seed, int ibits,
                                                         uint64_t prefix, int shift,
                                                         unsigned long long *__restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t hi_mask = shift + 8 >= 64 ? 0ull : ~0ull << (shift + 8);
    for (int64_t i = (int64_t)blockIdx.x * kVolBlock + threadIdx.x; i < nvox;
         i += (int64_t)gridDim.x * kVolBlock) {
        if (!((float)vol[i] > thr)) continue;
        const uint64_t key = priority(seed, (uint64_t)i, ibits);
        if ((key & hi_mask) != (prefix & hi_mask)) continue;
        atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__device__ __forceinline__ bool kept(const uint16_t *__restrict__ vol, int64_t i, float thr,
                                     uint64_t seed, int ibits, uint64_t kstar) {
    return (float)vol[i] > thr && priority(seed, (uint64_t)i, ibits) <= kstar;
}

// Kept voxels per block of kVolTile voxels.
__global__ __launch_bounds__(kVolBlock) void k_seed_count(const uint16_t *__restrict__ vol, int64_t nvox,
                                                          float thr, uint64_t seed, int ibits,
                                                          uint64_t kstar, uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kVolTile + (int64_t)threadIdx.x * kVolIpt;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kVolIpt; k++)
        if (base + k < nvox && kept(vol, base + k, thr, seed, ibits, kstar)) c++;
    if (c) atomicAdd(&s_cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_cnt;
}

struct SeedConst {
    double inv_n2;          // 2 / n
    double thr, range;
    double lo[3], hi[3];
    double sh_dc;           // value of the constant SH basis function
    float log_scale, logit_opacity;
};

// Writes the kept voxels of its block at offsets[block] + (rank in the block),
// planar [14][m].
__global__ __launch_bounds__(kVolBlock) void k_seed_emit(const uint16_t *__restrict__ vol, int64_t nvox,
                                                         int n, float thr, uint64_t seed, int ibits,
                                                         uint64_t kstar, const uint32_t *__restrict__ offsets,
                                                         SeedConst sc, int64_t m, float *__restrict__ P) {
    __shared__ uint32_t s_wave[kVolBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kVolTile + (int64_t)threadIdx.x * kVolIpt;
    bool keep[kVolIpt];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kVolIpt; k++) {
        keep[k] = base + k < nvox && kept(vol, base + k, thr, seed, ibits, kstar);
        c += keep[k] ? 1u : 0u;
    }
    // exclusive scan of c over the block (threads in raster order)
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t pos = offsets[blockIdx.x] + inc - c;
    for (int k = 0; k < w; k++) pos += s_wave[k];
#pragma unroll
    for (int k = 0; k < kVolIpt; k++) {
        if (!keep[k]) continue;
        const int64_t i = base + k;
        const int64_t ix = i / ((int64_t)n * n), iy = (i / n) % n, iz = i % n;
        const double t0 = ((double)vol[i] - sc.thr) / sc.range;
        const double t = t0 < 0.0 ? 0.0 : (t0 > 1.0 ? 1.0 : t0);
        float *p = P + pos;
        p[0 * m] = (float)(((double)ix + 0.5) * sc.inv_n2 - 1.0);
        p[1 * m] = (float)(((double)iy + 0.5) * sc.inv_n2 - 1.0);
        p[2 * m] = (float)(((double)iz + 0.5) * sc.inv_n2 - 1.0);
        p[3 * m] = p[4 * m] = p[5 * m] = sc.log_scale;
        p[6 * m] = 1.f;
        p[7 * m] = p[8 * m] = p[9 * m] = 0.f;
        p[10 * m] = sc.logit_opacity;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            const double col = sc.lo[ch] * (1.0 - t) + sc.hi[ch] * t;
            p[(11 + ch) * m] = (float)((col - 0.5) / sc.sh_dc);
        }
        pos++;
    }
}

// ---- ray march ---------------------------------------------------------------------

struct MarchConst {
    int n;
    float step, extinction, t_stop, thr, inv_range;
    float lo[3], hi[3];
};

__device__ __forceinline__ float vol_at(const uint16_t *__restrict__ vol, int n, int i, int j, int k) {
    return (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) ? 0.f
                                                                       : (float)vol[((int64_t)i * n + j) * n + k];
}

__device__ __forceinline__ float trilinear(const uint16_t *__restrict__ vol, int n, float x, float y, float z) {
    const float h = 0.5f * (float)n;
    const float ux = (x + 1.f) * h - 0.5f, uy = (y + 1.f) * h - 0.5f, uz = (z + 1.f) * h - 0.5f;
    const float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
    const int i = (int)fx0, j = (int)fy0, k = (int)fz0;
    const float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    const float c00 = vol_at(vol, n, i, j, k) * (1.f - fz) + vol_at(vol, n, i, j, k + 1) * fz;
    const float c01 = vol_at(vol, n, i, j + 1, k) * (1.f - fz) + vol_at(vol, n, i, j + 1, k + 1) * fz;
    const float c10 = vol_at(vol, n, i + 1, j, k) * (1.f - fz) + vol_at(vol, n, i + 1, j, k + 1) * fz;
    const float c11 = vol_at(vol, n, i + 1, j + 1, k) * (1.f - fz) + vol_at(vol, n, i + 1, j + 1, k + 1) * fz;
    const float c0 = c00 * (1.f - fy) + c01 * fy, c1 = c10 * (1.f - fy) + c11 * fy;
    return c0 * (1.f - fx) + c1 * fx;
}

__global__ __launch_bounds__(256) void k_raymarch(const uint16_t *__restrict__ vol, const gsf_camera *__restrict__ cam,
                                                  MarchConst mc, float *__restrict__ out) {
    const int W = cam->width, H = cam->height;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)W * H) return;
    const int j = (int)(q / W), i = (int)(q - (int64_t)j * W);
    const float *Rm = cam->viewmat;   // rows of [R | t]
    const float dc0 = ((float)i + 0.5f - cam->cx) / cam->fx, dc1 = ((float)j + 0.5f - cam->cy) / cam->fy;
    float d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = Rm[a] * dc0 + Rm[4 + a] * dc1 + Rm[8 + a];
    const float inn = 1.f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float o[3] = {cam->campos[0], cam->campos[1], cam->campos[2]};
    float t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        d[a] *= inn;
        const float inv = 1.f / d[a];
        float ta = (-1.f - o[a]) * inv, tb = (1.f - o[a]) * inv;
        if (ta > tb) { const float tmp = ta; ta = tb; tb = tmp; }
        t0 = fmaxf(t0, ta);
        t1 = fminf(t1, tb);
    }
    t0 = fmaxf(t0, 0.f);
    float C[3] = {0.f, 0.f, 0.f}, T = 1.f;
    if (t1 > t0) {
        for (int k = 0;; k++) {
            const float s0 = t0 + (float)k * mc.step;
            const float s1 = fminf(s0 + mc.step, t1);
            if (!(s1 > s0)) break;
            const float mid = 0.5f * (s0 + s1);
            const float v = trilinear(vol, mc.n, o[0] + d[0] * mid, o[1] + d[1] * mid, o[2] + d[2] * mid);
            const float t = fminf(fmaxf((v - mc.thr) * mc.inv_range, 0.f), 1.f);
            if (t > 0.f) {
                const float alpha = 1.f - expf(-mc.extinction * t * (s1 - s0));
#pragma unroll
                for (int c = 0; c < 3; c++) C[c] += (mc.lo[c] * (1.f - t) + mc.hi[c] * t) * alpha * T;
                T *= 1.f - alpha;
                if (T < mc.t_stop) break;
            }
        }
    }
    const int64_t plane = (int64_t)W * H;
#pragma unroll
    for (int c = 0; c < 3; c++) out[c * plane + q] = C[c] + T * cam->bg[c];
    out[3 * plane + q] = 1.f - T;
}

// ---- first-hit point cloud ----------------------------------------------------------
// The paper seeds its initial cloud from the first significant hit of rays
// cast at the volume from viewpoints around it, each point coloured by the
// path tracer (Method, "Volumetric Path Tracing").  Here a ray's hit is the
// midpoint of the first march segment after which the accumulated opacity
// reaches hit_alpha, and its colour the emission-absorption colour of that
// segment and the next color_steps - 1, divided by their opacity.

struct HitConst {
    int n, color_steps;
    float step, extinction, thr, inv_range, hit_alpha;
    float lo[3], hi[3];
};

struct RayViews {
    int64_t off[kMaxViews + 1];   // first ray of each view (rays in view, row, column order)
    int nviews;
};

__global__ __launch_bounds__(256) void k_first_hit(const uint16_t *__restrict__ vol,
                                                   const gsf_camera *__restrict__ cams, RayViews rv,
                                                   HitConst hc, uint8_t *__restrict__ hit,
                                                   float4 *__restrict__ pos, float4 *__restrict__ col) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rv.off[rv.nviews]) return;
    int v = 0;
    while (v + 1 < rv.nviews && r >= rv.off[v + 1]) v++;
    const gsf_camera *cam = cams + v;
    const int64_t q = r - rv.off[v];
    const int W = cam->width;
    const int j = (int)(q / W), i = (int)(q - (int64_t)j * W);
    const float *Rm = cam->viewmat;   // rows of [R | t]
    const float dc0 = ((float)i + 0.5f - cam->cx) / cam->fx, dc1 = ((float)j + 0.5f - cam->cy) / cam->fy;
    float d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = Rm[a] * dc0 + Rm[4 + a] * dc1 + Rm[8 + a];
    const float inn = 1.f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float o[3] = {cam->campos[0], cam->campos[1], cam->campos[2]};
    float t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        d[a] *= inn;
        const float inv = 1.f / d[a];
        float ta = (-1.f - o[a]) * inv, tb = (1.f - o[a]) * inv;
        if (ta > tb) { const float tmp = ta; ta = tb; tb = tmp; }
        t0 = fmaxf(t0, ta);
        t1 = fminf(t1, tb);
    }
    t0 = fmaxf(t0, 0.f);
    hit[r] = 0;
    if (!(t1 > t0)) return;
    float T = 1.f;
    int khit = -1;
    float mid_hit = 0.f;
    for (int k = 0;; k++) {
        const float s0 = t0 + (float)k * hc.step;
        const float s1 = fminf(s0 + hc.step, t1);
        if (!(s1 > s0)) break;
        const float mid = 0.5f * (s0 + s1);
        const float val = trilinear(vol, hc.n, o[0] + d[0] * mid, o[1] + d[1] * mid, o[2] + d[2] * mid);
        const float t = fminf(fmaxf((val - hc.thr) * hc.inv_range, 0.f), 1.f);
        T *= expf(-hc.extinction * t * (s1 - s0));
        if (1.f - T >= hc.hit_alpha) {
            khit = k;
            mid_hit = mid;
            break;
        }
    }
    if (khit < 0) return;
    float C[3] = {0.f, 0.f, 0.f}, Ts = 1.f;
    for (int k = khit; k < khit + hc.color_steps; k++) {
        const float s0 = t0 + (float)k * hc.step;
        const float s1 = fminf(s0 + hc.step, t1);
        if (!(s1 > s0)) break;
        const float mid = 0.5f * (s0 + s1);
        const float val = trilinear(vol, hc.n, o[0] + d[0] * mid, o[1] + d[1] * mid, o[2] + d[2] * mid);
        const float t = fminf(fmaxf((val - hc.thr) * hc.inv_range, 0.f), 1.f);
        const float alpha = 1.f - expf(-hc.extinction * t * (s1 - s0));
#pragma unroll
        for (int c = 0; c < 3; c++) C[c] += (hc.lo[c] * (1.f - t) + hc.hi[c] * t) * alpha * Ts;
        Ts *= 1.f - alpha;
    }
    const float ia = 1.f / (1.f - Ts);
    hit[r] = 1;
    pos[r] = make_float4(o[0] + d[0] * mid_hit, o[1] + d[1] * mid_hit, o[2] + d[2] * mid_hit, 0.f);
    col[r] = make_float4(C[0] * ia, C[1] * ia, C[2] * ia, 0.f);
}

// Digit histogram of the hit rays whose priority agrees with `prefix` above `shift`.
__global__ __launch_bounds__(kVolBlock) void k_hit_hist(const uint8_t *__restrict__ hit, int64_t nrays,
                                                        uint64_t seed, int ibits, uint64_t prefix,
                                                        int shift, unsigned long long *__restrict__ hist) {
    __shared__ unsigned long long h[256];
    for (int d = threadIdx.x; d < 256; d += kVolBlock) h[d] = 0ull;
    __syncthreads();
    const uint64_t above = shift >= 56 ? 0ull : (~0ull << (shift + 8));
    for (int64_t i = (int64_t)blockIdx.x * kVolBlock + threadIdx.x; i < nrays;
         i += (int64_t)gridDim.x * kVolBlock) {
        if (!hit[i]) continue;
        const uint64_t key = priority(seed, (uint64_t)i, ibits);
        if ((key & above) != (prefix & above)) continue;
        atomicAdd(&h[(key >> shift) & 0xFFu], 1ull);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kVolBlock)
        if (h[d]) atomicAdd(&hist[d], h[d]);
}

__device__ __forceinline__ bool hit_kept(const uint8_t *hit, int64_t i, uint64_t seed, int ibits,
                                         uint64_t kstar) {
    return hit[i] && priority(seed, (uint64_t)i, ibits) <= kstar;
}

// Kept rays per block of kVolTile rays.
__global__ __launch_bounds__(kVolBlock) void k_hit_count(const uint8_t *__restrict__ hit, int64_t nrays,
                                                         uint64_t seed, int ibits, uint64_t kstar,
                                                         uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_c;
    if (threadIdx.x == 0) s_c = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kVolTile + (int64_t)threadIdx.x * kVolIpt;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kVolIpt; k++) c += base + k < nrays && hit_kept(hit, base + k, seed, ibits, kstar) ? 1u : 0u;
    if (c) atomicAdd(&s_c, c);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_c;
}

struct HitEmit {
    float log_scale, logit_opacity, inv_sh_dc;
};

// Gaussians of the kept rays, in ray order, planar [14][m]; ray_ids nullable.
__global__ __launch_bounds__(kVolBlock) void k_hit_emit(const uint8_t *__restrict__ hit, int64_t nrays,
                                                        uint64_t seed, int ibits, uint64_t kstar,
                                                        const uint32_t *__restrict__ offsets,
                                                        const float4 *__restrict__ pos,
                                                        const float4 *__restrict__ col, HitEmit he,
                                                        int64_t m, float *__restrict__ P,
                                                        int32_t *__restrict__ ray_ids) {
    __shared__ uint32_t s_wave[kVolBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kVolTile + (int64_t)threadIdx.x * kVolIpt;
    bool keep[kVolIpt];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kVolIpt; k++) {
        keep[k] = base + k < nrays && hit_kept(hit, base + k, seed, ibits, kstar);
        c += keep[k] ? 1u : 0u;
    }
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t at = offsets[blockIdx.x] + inc - c;
    for (int k = 0; k < w; k++) at += s_wave[k];
#pragma unroll
    for (int k = 0; k < kVolIpt; k++) {
        if (!keep[k]) continue;
        const int64_t i = base + k;
        const float4 p4 = pos[i], c4 = col[i];
        float *p = P + at;
        p[0 * m] = p4.x;
        p[1 * m] = p4.y;
        p[2 * m] = p4.z;
        p[3 * m] = p[4 * m] = p[5 * m] = he.log_scale;
        p[6 * m] = 1.f;
        p[7 * m] = p[8 * m] = p[9 * m] = 0.f;
        p[10 * m] = he.logit_opacity;
        p[11 * m] = (c4.x - 0.5f) * he.inv_sh_dc;
        p[12 * m] = (c4.y - 0.5f) * he.inv_sh_dc;
        p[13 * m] = (c4.z - 0.5f) * he.inv_sh_dc;
        if (ray_ids) ray_ids[at] = (int32_t)i;
        at++;
    }
}

}  // namespace

int seed_blocks(int64_t nvox) { return (int)((nvox + kVolTile - 1) / kVolTile); }

// Host side of the seeding (synchronises the stream several times).
hipError_t run_seed(hipStream_t s, const uint16_t *vol, int n, double thr, double range,
                    const double *lo, const double *hi, double opacity, int64_t cap, uint64_t seed,
                    float *params, int64_t *count, void *scratch) {
    const int64_t nvox = (int64_t)n * n * n;
    int ibits = 0;
    while ((int64_t(1) << ibits) < nvox) ibits++;
    if (ibits < 1) ibits = 1;
    unsigned long long *hist = (unsigned long long *)scratch;                 // 256
    uint32_t *counts = (uint32_t *)((char *)scratch + 256 * sizeof(unsigned long long));
    const int nb = seed_blocks(nvox);
    std::vector<unsigned long long> h(256);
    std::vector<uint32_t> cnt(nb);
    int grid = nb < 1024 ? nb : 1024;
    // MSB-first radix select of the cap-th smallest priority among the candidates
    uint64_t prefix = 0;
    int64_t rank = cap;          // 1-based rank still to find within the prefix
    int64_t total = -1;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipError_t e = hipMemsetAsync(hist, 0, 256 * sizeof(unsigned long long), s);
        if (e != hipSuccess) return e;
        k_seed_hist<<<grid, kVolBlock, 0, s>>>(vol, nvox, (float)thr, seed, ibits, prefix, shift, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h.data(), hist, 256 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (total < 0) {
            total = 0;
            for (int d = 0; d < 256; d++) total += (int64_t)h[d];
            if (total <= cap) {     // every candidate is kept
                prefix = ~0ull;
                rank = 0;
                break;
            }
        }
        int d = 0;
        while (d < 255 && (int64_t)h[d] < rank) rank -= (int64_t)h[d++];
        prefix |= (uint64_t)d << shift;
    }
    const uint64_t kstar = prefix;   // priorities are distinct: exactly min(total, cap) are <= kstar
    k_seed_count<<<nb, kVolBlock, 0, s>>>(vol, nvox, (float)thr, seed, ibits, kstar, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(cnt.data(), counts, nb * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t m = 0;
    for (int b = 0; b < nb; b++) {
        const uint32_t c = cnt[b];
        cnt[b] = (uint32_t)m;
        m += c;
    }
    if ((e = hipMemcpyAsync(counts, cnt.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    SeedConst sc;
    sc.inv_n2 = 2.0 / n;
    sc.thr = thr;
    sc.range = range;
    for (int c = 0; c < 3; c++) {
        sc.lo[c] = lo[c];
        sc.hi[c] = hi[c];
    }
    sc.sh_dc = 0.5 / std::sqrt(std::acos(-1.0));
    sc.log_scale = (float)std::log(2.0 / n);
    sc.logit_opacity = (float)std::log(opacity / (1.0 - opacity));
    k_seed_emit<<<nb, kVolBlock, 0, s>>>(vol, nvox, n, (float)thr, seed, ibits, kstar, counts, sc, m, params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *count = m;
    return hipSuccess;
}

size_t seed_scratch_bytes(int64_t nvox) { return 256 * sizeof(unsigned long long) + (size_t)seed_blocks(nvox) * 4; }

namespace {
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t first_hit_scratch_bytes(int64_t nrays) {
    return round256((size_t)nrays) + 2 * round256((size_t)nrays * 16) +
           256 * sizeof(unsigned long long) + (size_t)seed_blocks(nrays) * 4;
}

hipError_t run_first_hits(hipStream_t s, const uint16_t *vol, int n, const gsf_camera *cams,
                          int nviews, const int32_t *widths, const int32_t *heights, float step,
                          float extinction, float thr, float range, const float *lo, const float *hi,
                          float hit_alpha, int color_steps, double opacity, int64_t cap,
                          uint64_t seed, float *params, int64_t *count, int32_t *ray_ids,
                          void *scratch) {
    RayViews rv;
    rv.nviews = nviews;
    rv.off[0] = 0;
    for (int v = 0; v < nviews; v++) rv.off[v + 1] = rv.off[v] + (int64_t)widths[v] * heights[v];
    const int64_t nrays = rv.off[nviews];
    char *sp = (char *)scratch;
    uint8_t *hit = (uint8_t *)sp;
    sp += round256((size_t)nrays);
    float4 *pos = (float4 *)sp;
    sp += round256((size_t)nrays * 16);
    float4 *col = (float4 *)sp;
    sp += round256((size_t)nrays * 16);
    unsigned long long *hist = (unsigned long long *)sp;
    uint32_t *counts = (uint32_t *)(sp + 256 * sizeof(unsigned long long));
    HitConst hc;
    hc.n = n;
    hc.color_steps = color_steps;
    hc.step = step;
    hc.extinction = extinction;
    hc.thr = thr;
    hc.inv_range = 1.f / range;
    hc.hit_alpha = hit_alpha;
    for (int c = 0; c < 3; c++) {
        hc.lo[c] = lo[c];
        hc.hi[c] = hi[c];
    }
    k_first_hit<<<(unsigned)((nrays + 255) / 256), 256, 0, s>>>(vol, cams, rv, hc, hit, pos, col);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ibits = 0;
    while ((int64_t(1) << ibits) < nrays) ibits++;
    if (ibits < 1) ibits = 1;
    const int nb = seed_blocks(nrays);
    std::vector<unsigned long long> h(256);
    std::vector<uint32_t> cnt(nb);
    const int grid = nb < 1024 ? nb : 1024;
    // MSB-first radix select of the cap-th smallest priority among the hit rays
    uint64_t prefix = 0;
    int64_t rank = cap;
    int64_t total = -1;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if ((e = hipMemsetAsync(hist, 0, 256 * sizeof(unsigned long long), s)) != hipSuccess) return e;
        k_hit_hist<<<grid, kVolBlock, 0, s>>>(hit, nrays, seed, ibits, prefix, shift, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h.data(), hist, 256 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (total < 0) {
            total = 0;
            for (int d = 0; d < 256; d++) total += (int64_t)h[d];
            if (total <= cap) {     // every hit is kept
                prefix = ~0ull;
                break;
            }
        }
        int d = 0;
        while (d < 255 && (int64_t)h[d] < rank) rank -= (int64_t)h[d++];
        prefix |= (uint64_t)d << shift;
    }
    const uint64_t kstar = prefix;   // priorities are distinct: min(total, cap) are <= kstar
    k_hit_count<<<nb, kVolBlock, 0, s>>>(hit, nrays, seed, ibits, kstar, counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(cnt.data(), counts, nb * sizeof(uint32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t m = 0;
    for (int b = 0; b < nb; b++) {
        const uint32_t c = cnt[b];
        cnt[b] = (uint32_t)m;
        m += c;
    }
    if ((e = hipMemcpyAsync(counts, cnt.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    HitEmit he;
    he.log_scale = (float)std::log(2.0 / n);
    he.logit_opacity = (float)std::log(opacity / (1.0 - opacity));
    he.inv_sh_dc = (float)(1.0 / (0.5 / std::sqrt(std::acos(-1.0))));
    k_hit_emit<<<nb, kVolBlock, 0, s>>>(hit, nrays, seed, ibits, kstar, counts, pos, col, he, m,
                                       params, ray_ids);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *count = m;
    return hipSuccess;
}

hipError_t run_raymarch(hipStream_t s, const uint16_t *vol, int n, const gsf_camera *cams, int nviews,
                        const int32_t *widths, const int32_t *heights, float step, float extinction,
                        float t_stop, float thr, float range, const float *lo, const float *hi,
                        float *out) {
    MarchConst mc;
    mc.n = n;
    mc.step = step;
    mc.extinction = extinction;
    mc.t_stop = t_stop;
    mc.thr = thr;
    mc.inv_range = 1.f / range;
    for (int c = 0; c < 3; c++) {
        mc.lo[c] = lo[c];
        mc.hi[c] = hi[c];
    }
    int64_t off = 0;
    for (int v = 0; v < nviews; v++) {
        const int64_t npix = (int64_t)widths[v] * heights[v];
        k_raymarch<<<(unsigned)((npix + 255) / 256), 256, 0, s>>>(vol, cams + v, mc, out + 4 * off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        off += npix;
    }
    return hipSuccess;
}

}  // namespace gsf
