// adam.hip - bias-corrected Adam over one flat float32 buffer with a learning
// rate per segment (the parameter planes), and the device-side step counter.
//
// The paper's continual refinement restarts optimisation with reloaded
// Gaussians and discarded optimiser state (Method, "Periphery Model
// Training"); zeroing m, v and the step counter is that restart.  The step
// counter lives in device memory so a captured step graph can be replayed.
// In the fused step the loss reduction advances it; a standalone call
// advances it with a one-thread kernel first.
#include "gs_internal.h"

namespace gsf {
namespace {

__global__ void k_step_inc(int32_t *step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) step[0] = step[0] + 1;
}

__device__ __forceinline__ float seg_lr(const SegTable &seg, int64_t e) {
    float lr = seg.lr[0];
    for (int s = 1; s < seg.n; s++)
        if (e >= seg.off[s]) lr = seg.lr[s];
    return lr;
}

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr, float b1,
                                         float b2, float ibc1, float ibc2, float eps) {
    m = fmaf(b1, m, (1.f - b1) * g);
    v = fmaf(b2, v, (1.f - b2) * (g * g));
    const float mh = m * ibc1;
    const float vh = v * ibc2;
    p -= lr * mh / (sqrtf(vh) + eps);
}

// 4 elements per thread; segment boundaries may fall anywhere.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t n,
                                              SegTable seg, float b1, float b2, float eps,
                                              const int32_t *__restrict__ step,
                                              const uint32_t *__restrict__ skip) {
    if (skip && (*skip & GSF_FLAG_CAPACITY)) return;   // the step's keys overflowed
    const float t = (float)step[0];
    const float ibc1 = 1.f / (1.f - powf(b1, t));
    const float ibc2 = 1.f / (1.f - powf(b2, t));
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
        float4 pp = reinterpret_cast<float4 *>(p)[q];
        const float4 gg = reinterpret_cast<const float4 *>(g)[q];
        float4 mm = reinterpret_cast<float4 *>(m)[q];
        float4 vv = reinterpret_cast<float4 *>(v)[q];
        const int64_t e = 4 * q;
        adam_one(pp.x, gg.x, mm.x, vv.x, seg_lr(seg, e), b1, b2, ibc1, ibc2, eps);
        adam_one(pp.y, gg.y, mm.y, vv.y, seg_lr(seg, e + 1), b1, b2, ibc1, ibc2, eps);
        adam_one(pp.z, gg.z, mm.z, vv.z, seg_lr(seg, e + 2), b1, b2, ibc1, ibc2, eps);
        adam_one(pp.w, gg.w, mm.w, vv.w, seg_lr(seg, e + 3), b1, b2, ibc1, ibc2, eps);
        reinterpret_cast<float4 *>(p)[q] = pp;
        reinterpret_cast<float4 *>(m)[q] = mm;
        reinterpret_cast<float4 *>(v)[q] = vv;
    }
    // tail elements
    const int64_t e = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        float pe = p[e], me = m[e], ve = v[e];
        adam_one(pe, g[e], me, ve, seg_lr(seg, e), b1, b2, ibc1, ibc2, eps);
        p[e] = pe;
        m[e] = me;
        v[e] = ve;
    }
}

// Visibility of each Gaussian for the masked update: 1 when any of its V
// records (r = v * n + i) touched at least one tile, else 0.
__global__ __launch_bounds__(256) void k_visible(const uint32_t *__restrict__ count, int n,
                                                 int nviews, uint8_t *__restrict__ vis) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t any = 0;
    for (int v = 0; v < nviews; v++) any |= count[(size_t)v * n + i];
    vis[i] = any != 0 ? 1 : 0;
}

// Visibility-masked Adam over planar [planes][n] state: one thread per
// (plane = blockIdx.y, Gaussian); a hidden Gaussian's p, m and v are neither
// read nor written.  Bias correction uses the shared step number.
__global__ __launch_bounds__(256) void k_adam_masked(float *__restrict__ p,
                                                     const float *__restrict__ g,
                                                     float *__restrict__ m, float *__restrict__ v,
                                                     int64_t n, PlaneLr lr,
                                                     const uint8_t *__restrict__ vis, float b1,
                                                     float b2, float eps,
                                                     const int32_t *__restrict__ step,
                                                     const uint32_t *__restrict__ skip) {
    if (skip && (*skip & GSF_FLAG_CAPACITY)) return;   // the step's keys overflowed
    const float t = (float)step[0];
    const float ibc1 = 1.f / (1.f - powf(b1, t));
    const float ibc2 = 1.f / (1.f - powf(b2, t));
    const int plane = blockIdx.y;
    const float rate = lr.lr[plane];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!vis[i]) continue;
        const int64_t e = plane * n + i;
        float pe = p[e], me = m[e], ve = v[e];
        adam_one(pe, g[e], me, ve, rate, b1, b2, ibc1, ibc2, eps);
        p[e] = pe;
        m[e] = me;
        v[e] = ve;
    }
}

// Optimiser restart: m = v = 0 and step = 0 (a kernel rather than memsets, so
// the reset can sit inside a captured graph).
__global__ __launch_bounds__(256) void k_adam_reset(float *__restrict__ m, float *__restrict__ v,
                                                    int64_t n, int32_t *__restrict__ step) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0) step[0] = 0;
    const int64_t n4 = n / 4;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t q = t0; q < n4; q += stride) {
        reinterpret_cast<float4 *>(m)[q] = z;
        reinterpret_cast<float4 *>(v)[q] = z;
    }
    for (int64_t e = 4 * n4 + t0; e < n; e += stride) {
        m[e] = 0.f;
        v[e] = 0.f;
    }
}

}  // namespace

void launch_visible(hipStream_t s, const uint32_t *count, int n, int nviews, uint8_t *vis) {
    k_visible<<<(n + 255) / 256, 256, 0, s>>>(count, n, nviews, vis);
}

void launch_adam_masked(hipStream_t s, float *p, const float *g, float *m, float *v, int64_t n,
                        int planes, const PlaneLr &lr, const uint8_t *vis, float b1, float b2,
                        float eps, int32_t *step, bool advance, const uint32_t *skip) {
    if (advance) k_step_inc<<<1, 64, 0, s>>>(step);
    int64_t bx = (n + 255) / 256;
    if (bx > 4096) bx = 4096;
    k_adam_masked<<<dim3((unsigned)bx, (unsigned)planes), 256, 0, s>>>(p, g, m, v, n, lr, vis, b1,
                                                                        b2, eps, step, skip);
}

void launch_adam_reset(hipStream_t s, float *m, float *v, int64_t n, int32_t *step) {
    int64_t blocks = (n / 4 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    k_adam_reset<<<(int)blocks, 256, 0, s>>>(m, v, n, step);
}

void launch_adam(hipStream_t s, float *p, const float *g, float *m, float *v, int64_t n,
                 const SegTable &seg, float b1, float b2, float eps, int32_t *step, bool advance,
                 const uint32_t *skip) {
    if (advance) k_step_inc<<<1, 64, 0, s>>>(step);
    int64_t blocks = (n / 4 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    k_adam<<<(int)blocks, 256, 0, s>>>(p, g, m, v, n, seg, b1, b2, eps, step, skip);
}

}  // namespace gsf
