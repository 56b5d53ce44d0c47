// reproject.hip - depth-guided reprojection of the foveal image (viewer side).
//
// The viewer moves the latest foveal image to the current head pose (Method,
// "Real-time Viewer", Eqs. (2)-(4)): pixel (i, j) with texture coordinate
// uv = ((i + 0.5) / W, (j + 0.5) / H) and first-hit distance d is lifted to
// p_world = pos_old + d (p_far - pos_old) / |p_far - pos_old|, p_far being the
// point (P_old V_old)^-1 maps (2 uv - 1, 1, 1) to after the divide by w, and
// projected by P_new V_new.  One thread per pixel; HBM-bound (a 4-byte depth
// in, 16 bytes of clip coordinates out).  The warp moves each pixel's colour to
// the output pixel its point lands in, nearest point first: a 64-bit atomicMin
// on (float bits of the new clip w, source index), then one resolve pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "gs_internal.h"

// The z-buffer of the no-allocation warp (gsf_reproject_warp_noalloc): one per
// GPU, kWarpScratchPixels 64-bit entries (36 MiB), held until the process
// ends.  Host code reaches it only through the device address found by
// warp_scratch_address (the array's name is a host-side stand-in there).
static __device__ __align__(256) unsigned long long scratch[gsf::kWarpScratchPixels];

namespace gsf {
namespace {

std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

}  // namespace

// Once per device, with that device current: the device address of `scratch`.
hipError_t warp_scratch_address(int device, unsigned long long **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        g_scratch_err[device] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? (unsigned long long *)ptr : nullptr;
        g_scratch_done[device] = true;
    }
    *out = g_scratch_ptr[device];
    return g_scratch_err[device];
}

namespace {

struct ReprojConst {
    float inv_old[16];   // (P_old V_old)^-1, row-major, column-vector convention
    float pv_new[16];    // P_new V_new
    float pos[3];        // pos_old
    int width, height;
};

// Eqs. (2)-(4) for pixel (i, j); false when the depth is not finite and positive.
__device__ __forceinline__ bool reproject_px(const ReprojConst &c, int i, int j, float d,
                                             float4 &clip) {
    if (!(d > 0.f) || !(d < __builtin_inff())) return false;
    const float nx = 2.f * (((float)i + 0.5f) / (float)c.width) - 1.f;
    const float ny = 2.f * (((float)j + 0.5f) / (float)c.height) - 1.f;
    const float *M = c.inv_old;
    float h[4];
#pragma unroll
    for (int r = 0; r < 4; r++) h[r] = M[4 * r] * nx + M[4 * r + 1] * ny + M[4 * r + 2] + M[4 * r + 3];
    const float rx = h[0] / h[3] - c.pos[0];
    const float ry = h[1] / h[3] - c.pos[1];
    const float rz = h[2] / h[3] - c.pos[2];
    const float s = d / sqrtf(rx * rx + ry * ry + rz * rz);
    const float p[3] = {c.pos[0] + rx * s, c.pos[1] + ry * s, c.pos[2] + rz * s};
    const float *N = c.pv_new;
    float o[4];
#pragma unroll
    for (int r = 0; r < 4; r++) o[r] = N[4 * r] * p[0] + N[4 * r + 1] * p[1] + N[4 * r + 2] * p[2] + N[4 * r + 3];
    clip = make_float4(o[0], o[1], o[2], o[3]);
    return true;
}

__global__ __launch_bounds__(256) void k_reproject(ReprojConst c, const float *__restrict__ depth,
                                                   float *__restrict__ clip) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= c.width) return;
    const size_t q = (size_t)j * c.width + i, plane = (size_t)c.width * c.height;
    float4 v;
    if (!reproject_px(c, i, j, depth[q], v)) v = make_float4(NAN, NAN, NAN, NAN);
    clip[q] = v.x;
    clip[plane + q] = v.y;
    clip[2 * plane + q] = v.z;
    clip[3 * plane + q] = v.w;
}

__global__ __launch_bounds__(256) void k_warp_clear(unsigned long long *__restrict__ zbuf, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        zbuf[t] = ~0ull;
}

__global__ __launch_bounds__(256) void k_warp_splat(ReprojConst c, const float *__restrict__ depth,
                                                    int out_w, int out_h,
                                                    unsigned long long *__restrict__ zbuf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= c.width) return;
    const size_t q = (size_t)j * c.width + i;
    float4 v;
    if (!reproject_px(c, i, j, depth[q], v)) return;
    if (!(v.w > 0.f)) return;
    const float zn = v.z / v.w;
    const float x = (v.x / v.w + 1.f) * 0.5f * (float)out_w;
    const float y = (v.y / v.w + 1.f) * 0.5f * (float)out_h;
    if (!(zn >= -1.f && zn <= 1.f && x >= 0.f && x < (float)out_w && y >= 0.f && y < (float)out_h))
        return;
    const int tx = min((int)x, out_w - 1), ty = min((int)y, out_h - 1);
    const unsigned long long key = ((unsigned long long)__float_as_uint(v.w) << 32) | (uint32_t)q;
    atomicMin(&zbuf[(size_t)ty * out_w + tx], key);
}

__global__ __launch_bounds__(256) void k_warp_resolve(const unsigned long long *__restrict__ zbuf,
                                                      int64_t n_out, const float *__restrict__ rgba,
                                                      int64_t n_src, float *__restrict__ out,
                                                      int32_t *__restrict__ src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_out) return;
    const unsigned long long key = zbuf[t];
    if (key == ~0ull) {
        out[t] = out[n_out + t] = out[2 * n_out + t] = out[3 * n_out + t] = 0.f;
        src[t] = -1;
        return;
    }
    const int64_t s = (int64_t)(key & 0xFFFFFFFFull);
#pragma unroll
    for (int ch = 0; ch < 4; ch++) out[ch * n_out + t] = rgba[ch * n_src + s];
    src[t] = (int32_t)s;
}

// C = A B for row-major 4x4 matrices.
void mat4_mul(const double *A, const double *B, double *C) {
    for (int r = 0; r < 4; r++)
        for (int k = 0; k < 4; k++) {
            double s = 0.0;
            for (int m = 0; m < 4; m++) s += A[4 * r + m] * B[4 * m + k];
            C[4 * r + k] = s;
        }
}

// Inverse by Gauss-Jordan elimination with partial pivoting; false if singular.
bool mat4_inv(const double *A, double *out) {
    double a[4][8];
    for (int r = 0; r < 4; r++)
        for (int k = 0; k < 8; k++) a[r][k] = k < 4 ? A[4 * r + k] : (k - 4 == r ? 1.0 : 0.0);
    for (int col = 0; col < 4; col++) {
        int piv = col;
        for (int r = col + 1; r < 4; r++)
            if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
        if (!(std::fabs(a[piv][col]) > 1e-300)) return false;
        if (piv != col)
            for (int k = 0; k < 8; k++) std::swap(a[piv][k], a[col][k]);
        const double inv = 1.0 / a[col][col];
        for (int k = 0; k < 8; k++) a[col][k] *= inv;
        for (int r = 0; r < 4; r++) {
            if (r == col) continue;
            const double f = a[r][col];
            for (int k = 0; k < 8; k++) a[r][k] -= f * a[col][k];
        }
    }
    for (int r = 0; r < 4; r++)
        for (int k = 0; k < 4; k++) out[4 * r + k] = a[r][4 + k];
    for (int e = 0; e < 16; e++)
        if (!std::isfinite(out[e])) return false;
    return true;
}

}  // namespace

bool make_reproj(const float *p_old, const float *v_old, const float *pos_old, const float *p_new,
                 const float *v_new, int width, int height, ReprojConstOpaque *out) {
    double P0[16], V0[16], P1[16], V1[16], A[16], Ainv[16], B[16];
    for (int e = 0; e < 16; e++) {
        P0[e] = p_old[e];
        V0[e] = v_old[e];
        P1[e] = p_new[e];
        V1[e] = v_new[e];
    }
    mat4_mul(P0, V0, A);
    if (!mat4_inv(A, Ainv)) return false;
    mat4_mul(P1, V1, B);
    ReprojConst c;
    for (int e = 0; e < 16; e++) {
        c.inv_old[e] = (float)Ainv[e];
        c.pv_new[e] = (float)B[e];
        if (!std::isfinite(c.pv_new[e]) || !std::isfinite(c.inv_old[e])) return false;
    }
    for (int k = 0; k < 3; k++) {
        c.pos[k] = pos_old[k];
        if (!std::isfinite(c.pos[k])) return false;
    }
    c.width = width;
    c.height = height;
    static_assert(sizeof(ReprojConst) <= sizeof(ReprojConstOpaque), "opaque size");
    std::memcpy(out->bytes, &c, sizeof c);
    return true;
}

void launch_reproject(hipStream_t s, const ReprojConstOpaque &k, const float *depth, float *clip) {
    ReprojConst c;
    std::memcpy(&c, k.bytes, sizeof c);
    const dim3 grid((c.width + 255) / 256, c.height);
    k_reproject<<<grid, 256, 0, s>>>(c, depth, clip);
}

void launch_reproject_warp(hipStream_t s, const ReprojConstOpaque &k, const float *rgba,
                           const float *depth, int out_w, int out_h, unsigned long long *zbuf,
                           float *out_rgba, int32_t *src) {
    ReprojConst c;
    std::memcpy(&c, k.bytes, sizeof c);
    const int64_t n_out = (int64_t)out_w * out_h, n_src = (int64_t)c.width * c.height;
    int64_t blocks = (n_out + 255) / 256;
    k_warp_clear<<<(int)std::min<int64_t>(blocks, 65535), 256, 0, s>>>(zbuf, n_out);
    k_warp_splat<<<dim3((c.width + 255) / 256, c.height), 256, 0, s>>>(c, depth, out_w, out_h, zbuf);
    k_warp_resolve<<<(int)blocks, 256, 0, s>>>(zbuf, n_out, rgba, n_src, out_rgba, src);
}

}  // namespace gsf
