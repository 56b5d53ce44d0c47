// project.hip - projection of 3D Gaussians to screen-space splats and its adjoint.
//
// Forward model (3D Gaussian Splatting, which the paper's peripheral model is
// fitted with; Related Work "Novel View Synthesis", Method "Periphery Model
// Training"): scale = exp(log-scale), rotation from the normalised quaternion,
// Sigma = R diag(s^2) R^T; camera point t = W mu + t_v; 2D covariance through the
// local affine approximation of the pinhole map, Sigma' = J W Sigma W^T J^T +
// 0.3 I with the Jacobian J evaluated at x/z, y/z clamped to 1.3 tan(fov/2);
// conic = inverse(Sigma'); opacity = sigmoid(logit); colour = max(0, SH . Y(d)
// + 0.5) with d the unit direction from the camera centre.
//
// Forward pass: one thread per record (view v, Gaussian i), or, with several
// views and SH degree 0-1, one thread per Gaussian looping over the views (its
// parameters read once); backward pass: one thread per Gaussian looping over
// views (no atomics).  Parameter planes are read coalesced across i.
#include <climits>
#include "gs_internal.h"

namespace gsf {
namespace {

// Real spherical-harmonic basis, orthonormal, Condon-Shortley phase,
// k = l*l + l + m.  Constants are closed-form normalisers.
constexpr float kSH0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float kSH2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kSH20 = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kSH22 = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float kSH33 = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float kSH32 = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float kSH31 = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float kSH30 = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float kSH32b = 1.4453057213202769f;  // sqrt(105 / pi) / 4

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = kSH0;
    if (DEG >= 1) {
        Y[1] = -kSH1 * y;
        Y[2] = kSH1 * z;
        Y[3] = -kSH1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * (x * y);
        Y[5] = -kSH2a * (y * z);
        Y[6] = kSH20 * (2.f * zz - xx - yy);
        Y[7] = -kSH2a * (x * z);
        Y[8] = kSH22 * (xx - yy);
    }
    if (DEG >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[9] = -kSH33 * y * (3.f * xx - yy);
        Y[10] = kSH32 * (x * y) * z;
        Y[11] = -kSH31 * y * (4.f * zz - xx - yy);
        Y[12] = kSH30 * z * (2.f * zz - 3.f * xx - 3.f * yy);
        Y[13] = -kSH31 * x * (4.f * zz - xx - yy);
        Y[14] = kSH32b * z * (xx - yy);
        Y[15] = -kSH33 * x * (xx - 3.f * yy);
    }
}

// d = d(loss)/d(direction) accumulated from dY_k weights w_k (= sum_c g_c sh_kc).
template <int DEG>
__device__ __forceinline__ void sh_basis_vjp(float x, float y, float z, const float *w,
                                             float &gx, float &gy, float &gz) {
    gx = gy = gz = 0.f;
    if (DEG >= 1) {
        gy += -kSH1 * w[1];
        gz += kSH1 * w[2];
        gx += -kSH1 * w[3];
    }
    if (DEG >= 2) {
        gx += kSH2a * y * w[4];
        gy += kSH2a * x * w[4];
        gy += -kSH2a * z * w[5];
        gz += -kSH2a * y * w[5];
        gx += -2.f * kSH20 * x * w[6];
        gy += -2.f * kSH20 * y * w[6];
        gz += 4.f * kSH20 * z * w[6];
        gx += -kSH2a * z * w[7];
        gz += -kSH2a * x * w[7];
        gx += 2.f * kSH22 * x * w[8];
        gy += -2.f * kSH22 * y * w[8];
    }
    if (DEG >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += -6.f * kSH33 * x * y * w[9];
        gy += -kSH33 * (3.f * xx - 3.f * yy) * w[9];
        gx += kSH32 * y * z * w[10];
        gy += kSH32 * x * z * w[10];
        gz += kSH32 * x * y * w[10];
        gx += 2.f * kSH31 * x * y * w[11];
        gy += -kSH31 * (4.f * zz - xx - 3.f * yy) * w[11];
        gz += -8.f * kSH31 * y * z * w[11];
        gx += -6.f * kSH30 * x * z * w[12];
        gy += -6.f * kSH30 * y * z * w[12];
        gz += kSH30 * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        gx += -kSH31 * (4.f * zz - 3.f * xx - yy) * w[13];
        gy += 2.f * kSH31 * x * y * w[13];
        gz += -8.f * kSH31 * x * z * w[13];
        gx += 2.f * kSH32b * x * z * w[14];
        gy += -2.f * kSH32b * y * z * w[14];
        gz += kSH32b * (xx - yy) * w[14];
        gx += -kSH33 * (3.f * xx - 3.f * yy) * w[15];
        gy += 6.f * kSH33 * x * y * w[15];
    }
}

// World-space state of one Gaussian (view independent).
struct Gauss {
    float mu[3], s[3], qn[4], qinv, R[9], Sig[6], o;   // Sig: xx xy xz yy yz zz
};

__device__ __forceinline__ void load_gauss(const float *__restrict__ P, int n, int i, Gauss &g) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        g.mu[a] = P[(size_t)a * n + i];
        g.s[a] = expf(P[(size_t)(3 + a) * n + i]);
    }
    float q[4], qq = 0.f;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        q[a] = P[(size_t)(6 + a) * n + i];
        qq = fmaf(q[a], q[a], qq);
    }
    const float qnorm = sqrtf(qq);
    g.qinv = 1.f / qnorm;
#pragma unroll
    for (int a = 0; a < 4; a++) g.qn[a] = q[a] * g.qinv;
    const float w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
    g.R[0] = 1.f - 2.f * (y * y + z * z);
    g.R[1] = 2.f * (x * y - w * z);
    g.R[2] = 2.f * (x * z + w * y);
    g.R[3] = 2.f * (x * y + w * z);
    g.R[4] = 1.f - 2.f * (x * x + z * z);
    g.R[5] = 2.f * (y * z - w * x);
    g.R[6] = 2.f * (x * z - w * y);
    g.R[7] = 2.f * (y * z + w * x);
    g.R[8] = 1.f - 2.f * (x * x + y * y);
    float s2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) s2[a] = g.s[a] * g.s[a];
    // Sigma_ab = sum_k R_ak s_k^2 R_bk
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const float *ra = g.R + 3 * ia[e], *rb = g.R + 3 * ib[e];
        g.Sig[e] = fmaf(ra[0] * s2[0], rb[0], fmaf(ra[1] * s2[1], rb[1], ra[2] * s2[2] * rb[2]));
    }
    g.o = 1.f / (1.f + expf(-P[(size_t)10 * n + i]));
}

__device__ __forceinline__ float sig_at(const float *S, int a, int b) {
    // symmetric 3x3 from its upper triangle (xx xy xz yy yz zz)
    const int idx = a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : (b == 0 ? a : (b == 1 ? 2 + a : 5));
    return S[idx];
}

// View-dependent projection of one Gaussian.
struct Proj {
    float t[3], rx, ry;
    int clx, cly;          // Jacobian clamp sign per axis
    float J00, J02, J11, J12;
    float M[6];            // M = J W (2 x 3)
    float a, b, c, det;    // Sigma' entries (low-pass included)
    float A, B, C;         // conic
    float mx, my;
};

__device__ __forceinline__ bool project(const Gauss &g, const gsf_camera &cam, Proj &p) {
    const float *W = cam.viewmat;
#pragma unroll
    for (int r = 0; r < 3; r++)
        p.t[r] = fmaf(W[4 * r], g.mu[0], fmaf(W[4 * r + 1], g.mu[1], fmaf(W[4 * r + 2], g.mu[2], W[4 * r + 3])));
    const float tz = p.t[2];
    if (!(tz > cam.znear)) return false;
    const float limx = kJClamp * cam.tan_half_fov_x, limy = kJClamp * cam.tan_half_fov_y;
    p.rx = p.t[0] / tz;
    p.ry = p.t[1] / tz;
    p.clx = p.rx > limx ? 1 : (p.rx < -limx ? -1 : 0);
    p.cly = p.ry > limy ? 1 : (p.ry < -limy ? -1 : 0);
    const float rxc = fminf(limx, fmaxf(-limx, p.rx)), ryc = fminf(limy, fmaxf(-limy, p.ry));
    const float iz = 1.f / tz;
    p.J00 = cam.fx * iz;
    p.J11 = cam.fy * iz;
    p.J02 = -cam.fx * rxc * iz;
    p.J12 = -cam.fy * ryc * iz;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        p.M[k] = fmaf(p.J00, W[k], p.J02 * W[8 + k]);
        p.M[3 + k] = fmaf(p.J11, W[4 + k], p.J12 * W[8 + k]);
    }
    // Sigma' = M Sigma M^T
    float MS[6];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int l = 0; l < 3; l++)
            MS[3 * r + l] = fmaf(p.M[3 * r], sig_at(g.Sig, 0, l),
                                 fmaf(p.M[3 * r + 1], sig_at(g.Sig, 1, l), p.M[3 * r + 2] * sig_at(g.Sig, 2, l)));
    p.a = fmaf(MS[0], p.M[0], fmaf(MS[1], p.M[1], MS[2] * p.M[2])) + kLowPass;
    p.b = fmaf(MS[0], p.M[3], fmaf(MS[1], p.M[4], MS[2] * p.M[5]));
    p.c = fmaf(MS[3], p.M[3], fmaf(MS[4], p.M[4], MS[5] * p.M[5])) + kLowPass;
    p.det = p.a * p.c - p.b * p.b;
    if (!(p.det > 0.f)) return false;
    const float idet = 1.f / p.det;
    p.A = p.c * idet;
    p.B = -p.b * idet;
    p.C = p.a * idet;
    p.mx = fmaf(cam.fx, p.rx, cam.cx);
    p.my = fmaf(cam.fy, p.ry, cam.cy);
    return true;
}

template <int DEG>
__device__ __forceinline__ void view_dir(const Gauss &g, const gsf_camera &cam, float d[3],
                                         float &inv_norm) {
    const float u0 = g.mu[0] - cam.campos[0], u1 = g.mu[1] - cam.campos[1], u2 = g.mu[2] - cam.campos[2];
    const float nn = sqrtf(fmaf(u0, u0, fmaf(u1, u1, u2 * u2)));
    inv_norm = 1.f / nn;
    d[0] = u0 * inv_norm;
    d[1] = u1 * inv_norm;
    d[2] = u2 * inv_norm;
}

// Record r = v n + i's projection of Gaussian g; returns its key count (0 when
// culled).  shc: its SH coefficients [K][3] in registers, or null to read them
// from P.
template <int DEG>
__device__ __forceinline__ uint32_t project_gauss(const Gauss &g, const float *shc,
                                                    const float *__restrict__ P, int n, int v, int i,
                                                    const gsf_camera *__restrict__ cams,
                                                    const ViewDesc *__restrict__ views, int tile,
                                                    SplatPtrs sp, uint32_t *__restrict__ depth_key,
                                                    uint2 *__restrict__ rect,
                                                    uint32_t *__restrict__ count,
                                                    uint2 *__restrict__ rspan,
                                                    const float *__restrict__ cull_gaze,
                                                    float cull_radius, const FoveaRows &fr) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int r = v * n + i;
    const gsf_camera &cam = cams[v];
    Proj p;
    bool ok = project(g, cam, p) && (g.o >= kAlphaMin);
    if (ok) ok = isfinite(p.mx) && isfinite(p.my) && isfinite(p.A) && isfinite(p.B) && isfinite(p.C);
    if (!ok) {
        depth_key[r] = 0xFFFFFFFFu;
        rect[r] = make_uint2(0u, 0u);
        rspan[r] = make_uint2(0u, 0u);   // every record: whole 64-byte chunks are written
        count[r] = 0u;
        return 0u;
    }
    // pixel mean in double precision (camera transform included), stored as an
    // integer pixel plus the offset of the mean from that pixel's centre
    double td[3];
#pragma unroll
    for (int q = 0; q < 3; q++)
        td[q] = fma((double)cam.viewmat[4 * q], (double)g.mu[0],
                    fma((double)cam.viewmat[4 * q + 1], (double)g.mu[1],
                        fma((double)cam.viewmat[4 * q + 2], (double)g.mu[2], (double)cam.viewmat[4 * q + 3])));
    const double mxd = fma((double)cam.fx, td[0] / td[2], (double)cam.cx);
    const double myd = fma((double)cam.fy, td[1] / td[2], (double)cam.cy);
    const double ixd = floor(mxd), iyd = floor(myd);
    // support box: AABB of the ellipse where o e^power >= 1/255, padded
    const float k2 = 2.f * logf(255.f * g.o);
    const float hx = fmaf(sqrtf(k2 * p.a), 1.f + kBoxRel, kBoxAbs);
    const float hy = fmaf(sqrtf(k2 * p.c), 1.f + kBoxRel, kBoxAbs);
    const ViewDesc vd = views[v];
    const float x0 = fmaxf(ceilf((float)(mxd - hx - 0.5)), 0.f);
    const float x1 = fminf(floorf((float)(mxd + hx - 0.5)), (float)(vd.width - 1));
    const float y0 = fmaxf(ceilf((float)(myd - hy - 0.5)), 0.f);
    const float y1 = fminf(floorf((float)(myd + hy - 0.5)), (float)(vd.height - 1));
    const bool empty = !(x0 <= x1) || !(y0 <= y1);
    uint32_t tx0 = 0u, tx1 = 0u, ty0 = 0u, ty1 = 0u;
    FoveaTiles f{0, -1, 0, -1};
    bool away = false;   // fovea culling: the box meets no tile of the fovea
    if (!empty) {
        tx0 = (uint32_t)x0 / tile;
        tx1 = (uint32_t)x1 / tile;
        ty0 = (uint32_t)y0 / tile;
        ty1 = (uint32_t)y1 / tile;
        if (cull_gaze) {
            f = fovea_tiles(cull_gaze, v, cull_radius, vd.width, vd.height, tile);
            away = f.tx0 > f.tx1 || (int)tx1 < f.tx0 || (int)tx0 > f.tx1 || (int)ty1 < f.ty0 ||
                   (int)ty0 > f.ty1;
        }
    }
    depth_key[r] = __float_as_uint(p.t[2]);
    if (away) {   // never read: no colour, no splat record
        rect[r] = make_uint2(0u, 0u);
        rspan[r] = make_uint2(0u, 0u);   // every record: whole 64-byte chunks are written
        count[r] = 0u;
        return 0u;
    }
    float d[3], inv_norm;
    view_dir<DEG>(g, cam, d, inv_norm);
    float Y[16];
    sh_basis<DEG>(d[0], d[1], d[2], Y);
    float col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < K; k++)
            acc = fmaf(shc ? shc[3 * k + ch] : P[(size_t)(11 + 3 * k + ch) * n + i], Y[k], acc);
        col[ch] = fmaxf(acc + 0.5f, 0.f);
    }
    // conic pre-scaled for a base-2 exponent, and the alpha threshold of the
    // same exponent: o 2^power2 >= 1/255 where power2 >= tau = -log2(255 o)
    *sp.at(r, kRecA) = make_float4((float)(ixd + 0.5 - mxd), (float)(iyd + 0.5 - myd),
                                   (-0.5f * kLog2e) * p.A, -kLog2e * p.B);
    *sp.at(r, kRecB) = make_float4((-0.5f * kLog2e) * p.C, g.o, col[0], col[1]);
    *sp.at(r, kRecC) = make_float4(col[2], -log2f(255.f * g.o), (float)ixd, (float)iyd);
    if (empty) {
        rect[r] = make_uint2(0u, 0u);
        rspan[r] = make_uint2(0u, 0u);   // every record: whole 64-byte chunks are written
        count[r] = 0u;
        return 0u;
    }
    if (cull_gaze) {   // only the tiles that meet the fovea are composited (rows clipped below)
        tx0 = max(tx0, (uint32_t)f.tx0);
        tx1 = min(tx1, (uint32_t)f.tx1);
        ty0 = max(ty0, (uint32_t)f.ty0);
        ty1 = min(ty1, (uint32_t)f.ty1);
    }
    rect[r] = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
    // the tiles of each box row that the support ellipse reaches
    const float Kp = k2 * ((1.f + kBoxRel) * (1.f + kBoxRel));
    float ey;
    const float4 ep = ellipse_pack(p.a, p.b, p.c, Kp, ey);
    *sp.at(r, kRecEll) = ep;
    uint32_t cnt = 0, listed_rows = 0;
    const Ellipse e{ep.x, ep.y, ep.z, ep.w, sqrtf(ep.y / ep.z), (float)(ixd + 0.5 - mxd),
                    (float)(iyd + 0.5 - myd), (int)ixd, (int)iyd};
    const int tl = 31 - __clz(tile);
    const bool pack = ty1 - ty0 + 1 <= (uint32_t)kPackRows && tx1 - tx0 + 1 <= (uint32_t)kPackCols;
    uint32_t packed[2] = {0u, 0u};
    for (uint32_t ty = ty0; ty <= ty1; ty++) {
        int c0, c1;
        if (row_span(e, (int)ty, tl, vd.width, vd.height, (int)tx0, (int)tx1, c0, c1) &&
            fovea_rows_clip(fr, v, (int)ty, c0, c1)) {
            const uint32_t w = (uint32_t)(c1 - c0 + 1);
            cnt += w;
            listed_rows++;
            if (pack) {
                const uint32_t k = ty - ty0;
                packed[k >> 1] |= (((uint32_t)c0 - tx0) | (w << 8)) << (16 * (k & 1));
            }
        }
    }
    // packed spans, or the number of row-table entries the duplicate pass writes
    rspan[r] = pack ? make_uint2(packed[0], packed[1]) : make_uint2(listed_rows, 0u);
    count[r] = cnt;
    return cnt;
}

// Record r's projection (its Gaussian's parameters read from P).
template <int DEG>
__device__ __forceinline__ uint32_t project_record(const float *__restrict__ P, int n, int r,
                                                     const gsf_camera *__restrict__ cams,
                                                     const ViewDesc *__restrict__ views, int tile,
                                                     SplatPtrs sp, uint32_t *__restrict__ depth_key,
                                                     uint2 *__restrict__ rect,
                                                     uint32_t *__restrict__ count,
                                                     uint2 *__restrict__ rspan,
                                                     const float *__restrict__ cull_gaze,
                                                     float cull_radius, const FoveaRows &fr) {
    const int v = r / n;
    const int i = r - v * n;
    Gauss g;
    load_gauss(P, n, i, g);
    return project_gauss<DEG>(g, nullptr, P, n, v, i, cams, views, tile, sp, depth_key, rect, count,
                              rspan, cull_gaze, cull_radius, fr);
}

// Several views, SH degrees 0-1: one thread per Gaussian projects it into every
// view, its parameters read once instead of once per view (records of one
// view stay consecutive across the threads, so the stores coalesce).  The
// per-block count totals come from k_block_totals.
template <int DEG>
__global__ __launch_bounds__(256) void k_project_fwd_views(const float *__restrict__ P, int n,
                                                           int nviews,
                                                           const gsf_camera *__restrict__ cams,
                                                           const ViewDesc *__restrict__ views,
                                                           int tile, SplatPtrs sp,
                                                           uint32_t *__restrict__ depth_key,
                                                           uint2 *__restrict__ rect,
                                                           uint32_t *__restrict__ count,
                                                           uint2 *__restrict__ rspan,
                                                           const float *__restrict__ cull_gaze,
                                                           float cull_radius, FoveaRows fr) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= n) return;
    Gauss g;
    load_gauss(P, n, i, g);
    float shc[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; k++) shc[k] = P[(size_t)(11 + k) * n + i];
    for (int v = 0; v < nviews; v++)
        project_gauss<DEG>(g, shc, P, n, v, i, cams, views, tile, sp, depth_key, rect, count, rspan,
                           cull_gaze, cull_radius, fr);
}

// block_sums[b] / block_act[b]: the total count / the records with a nonzero
// count among records 256 b .. 256 b + 255.  One wave per 256 records, four
// per lane in one 16-byte load (the count array is 256-byte aligned).
__global__ __launch_bounds__(256) void k_block_totals(const uint32_t *__restrict__ count, int nrec,
                                                      uint32_t *__restrict__ block_sums,
                                                      uint32_t *__restrict__ block_act) {
    const int bb = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (bb * 256 >= nrec) return;
    const int lane = (int)(threadIdx.x & 63), r0 = bb * 256 + lane * 4;
    uint4 q = make_uint4(0u, 0u, 0u, 0u);
    if (r0 + 3 < nrec) {
        q = *reinterpret_cast<const uint4 *>(count + r0);
    } else {
        if (r0 < nrec) q.x = count[r0];
        if (r0 + 1 < nrec) q.y = count[r0 + 1];
        if (r0 + 2 < nrec) q.z = count[r0 + 2];
    }
    uint32_t c = q.x + q.y + q.z + q.w;
    uint32_t a = (q.x != 0u) + (q.y != 0u) + (q.z != 0u) + (q.w != 0u);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        a += __shfl_xor(a, o, 64);
    }
    if (lane == 0) {
        block_sums[bb] = c;
        block_act[bb] = a;
    }
}

// One thread per record, 256 records per block; block b also writes the key
// count of its records to block_sums[b], the first level of the scan that
// places the keys.
template <int DEG>
__global__ __launch_bounds__(256) void k_project_fwd(const float *__restrict__ P, int n, int nrec,
                                                     const gsf_camera *__restrict__ cams,
                                                     const ViewDesc *__restrict__ views, int tile,
                                                     SplatPtrs sp, uint32_t *__restrict__ depth_key,
                                                     uint2 *__restrict__ rect,
                                                     uint32_t *__restrict__ count,
                                                     uint2 *__restrict__ rspan,
                                                     const float *__restrict__ cull_gaze,
                                                     float cull_radius, FoveaRows fr,
                                                     uint32_t *__restrict__ block_sums,
                                                     uint32_t *__restrict__ block_act) {
    __shared__ uint32_t s_w[4], s_a[4];
    const int r = blockIdx.x * 256 + (int)threadIdx.x;
    uint32_t c = r < nrec ? project_record<DEG>(P, n, r, cams, views, tile, sp, depth_key, rect, count,
                                                rspan, cull_gaze, cull_radius, fr)
                          : 0u;
    const uint32_t a = (uint32_t)__popcll(__ballot(c != 0u));   // records that list a tile
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) {
        s_w[threadIdx.x >> 6] = c;
        s_a[threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        block_act[blockIdx.x] = s_a[0] + s_a[1] + s_a[2] + s_a[3];
    }
}

// d(quaternion)/... from d(R) for the rotation of a unit quaternion (w, x, y, z).
__device__ __forceinline__ void quat_vjp(const float *q, const float *dR, float *dq) {
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                   w * dR[7] - 2.f * x * dR[8]);
    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                   z * dR[7] - 2.f * y * dR[8]);
    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                   y * dR[5] + x * dR[6] + y * dR[7]);
}

// FUSED: the per-record screen-space gradient is summed here from the
// compositing adjoint's per-key terms (wave_key_sum); otherwise it is read
// from g2d [9][V*n], which a separate pass wrote.
template <int DEG, bool FUSED>
__global__ __launch_bounds__(128) void k_project_bwd(const float *__restrict__ P, int n, int nviews,
                                                     const gsf_camera *__restrict__ cams, KeyPlace kp,
                                                     const float *__restrict__ g2d,
                                                     float *__restrict__ grads, bool accumulate) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;   // every lane takes part in the per-view key sums
    Gauss g;
    load_gauss(P, n, valid ? i : 0, g);
    float dmu[3] = {0.f, 0.f, 0.f};
    float dS[9];
#pragma unroll
    for (int e = 0; e < 9; e++) dS[e] = 0.f;
    float dop = 0.f;
    float dsh[K][3];
#pragma unroll
    for (int k = 0; k < K; k++) dsh[k][0] = dsh[k][1] = dsh[k][2] = 0.f;

    for (int v = 0; v < nviews; v++) {
        // this view's screen-space gradient: the sum of the record's per-key terms
        float gg[9];
        const uint32_t r = (uint32_t)v * (uint32_t)n + (uint32_t)i;
        if (FUSED) {
            wave_key_sum(kp, r, valid, gg);
        } else {
            const size_t nrec = (size_t)nviews * n;
#pragma unroll
            for (int f = 0; f < 9; f++) gg[f] = valid ? g2d[f * nrec + r] : 0.f;
        }
        bool any = false;
#pragma unroll
        for (int f = 0; f < 9; f++) any |= gg[f] != 0.f;
        if (!valid || !any) continue;
        const gsf_camera &cam = cams[v];
        Proj p;
        if (!project(g, cam, p)) continue;
        const float *W = cam.viewmat;
        const float tz = p.t[2], iz = 1.f / tz, iz2 = iz * iz;
        // conic = inverse(Sigma'): dSigma' = -Q dQ Q, dQ = [[gA, gB/2], [gB/2, gC]]
        const float gA = gg[2], hB = 0.5f * gg[3], gC = gg[4];
        const float X00 = p.A * gA + p.B * hB, X01 = p.A * hB + p.B * gC;
        const float X10 = p.B * gA + p.C * hB, X11 = p.B * hB + p.C * gC;
        const float da = -(X00 * p.A + X01 * p.B);
        const float db = -(X00 * p.B + X01 * p.C);
        const float dc = -(X10 * p.B + X11 * p.C);
        // dSigma += M^T dSigma' M
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
            for (int l = 0; l < 3; l++) {
                const float m0k = p.M[k], m1k = p.M[3 + k], m0l = p.M[l], m1l = p.M[3 + l];
                dS[3 * k + l] += da * m0k * m0l + db * (m0k * m1l + m1k * m0l) + dc * m1k * m1l;
            }
        // dM = 2 dSigma' M Sigma
        float MS[6];
#pragma unroll
        for (int rr = 0; rr < 2; rr++)
#pragma unroll
            for (int l = 0; l < 3; l++)
                MS[3 * rr + l] = p.M[3 * rr] * sig_at(g.Sig, 0, l) + p.M[3 * rr + 1] * sig_at(g.Sig, 1, l) +
                                 p.M[3 * rr + 2] * sig_at(g.Sig, 2, l);
        float dM[6];
#pragma unroll
        for (int l = 0; l < 3; l++) {
            dM[l] = 2.f * (da * MS[l] + db * MS[3 + l]);
            dM[3 + l] = 2.f * (db * MS[l] + dc * MS[3 + l]);
        }
        // dJ = dM W^T (only the four non-zero Jacobian entries)
        const float dJ00 = dM[0] * W[0] + dM[1] * W[1] + dM[2] * W[2];
        const float dJ02 = dM[0] * W[8] + dM[1] * W[9] + dM[2] * W[10];
        const float dJ11 = dM[3] * W[4] + dM[4] * W[5] + dM[5] * W[6];
        const float dJ12 = dM[3] * W[8] + dM[4] * W[9] + dM[5] * W[10];
        float dtx = 0.f, dty = 0.f, dtz = 0.f;
        dtz -= cam.fx * iz2 * dJ00 + cam.fy * iz2 * dJ11;
        const float limx = kJClamp * cam.tan_half_fov_x, limy = kJClamp * cam.tan_half_fov_y;
        if (p.clx == 0) {
            dtx -= cam.fx * iz2 * dJ02;
            dtz += 2.f * cam.fx * p.t[0] * iz2 * iz * dJ02;
        } else {
            dtz += cam.fx * ((float)p.clx * limx) * iz2 * dJ02;
        }
        if (p.cly == 0) {
            dty -= cam.fy * iz2 * dJ12;
            dtz += 2.f * cam.fy * p.t[1] * iz2 * iz * dJ12;
        } else {
            dtz += cam.fy * ((float)p.cly * limy) * iz2 * dJ12;
        }
        // pixel mean: mx = fx tx / tz + cx
        dtx += cam.fx * iz * gg[0];
        dtz -= cam.fx * p.t[0] * iz2 * gg[0];
        dty += cam.fy * iz * gg[1];
        dtz -= cam.fy * p.t[1] * iz2 * gg[1];
#pragma unroll
        for (int k = 0; k < 3; k++) dmu[k] += W[k] * dtx + W[4 + k] * dty + W[8 + k] * dtz;
        dop += gg[5];
        // colour
        float d[3], inv_norm;
        view_dir<DEG>(g, cam, d, inv_norm);
        float Y[16];
        sh_basis<DEG>(d[0], d[1], d[2], Y);
        float wY[16];
#pragma unroll
        for (int k = 0; k < K; k++) wY[k] = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < K; k++) acc = fmaf(P[(size_t)(11 + 3 * k + ch) * n + i], Y[k], acc);
            if (!(acc + 0.5f > 0.f)) continue;
            const float gc = gg[6 + ch];
#pragma unroll
            for (int k = 0; k < K; k++) {
                dsh[k][ch] += Y[k] * gc;
                if (DEG > 0) wY[k] += gc * P[(size_t)(11 + 3 * k + ch) * n + i];
            }
        }
        if (DEG > 0) {
            float gx, gy, gz;
            sh_basis_vjp<DEG>(d[0], d[1], d[2], wY, gx, gy, gz);
            const float dot = gx * d[0] + gy * d[1] + gz * d[2];
            dmu[0] += (gx - d[0] * dot) * inv_norm;
            dmu[1] += (gy - d[1] * dot) * inv_norm;
            dmu[2] += (gz - d[2] * dot) * inv_norm;
        }
    }
    // Sigma = M3 M3^T with M3 = R diag(s): dM3 = 2 dSigma M3 (dSigma symmetric)
    float dR[9], ds[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int rr = 0; rr < 3; rr++)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++) acc += dS[3 * rr + k] * g.R[3 * k + cc] * g.s[cc];
            const float dm3 = 2.f * acc;
            ds[cc] += dm3 * g.R[3 * rr + cc];
            dR[3 * rr + cc] = dm3 * g.s[cc];
        }
    if (!valid) return;
    float dqn[4];
    quat_vjp(g.qn, dR, dqn);
    const float qdot = dqn[0] * g.qn[0] + dqn[1] * g.qn[1] + dqn[2] * g.qn[2] + dqn[3] * g.qn[3];
    // plane c of Gaussian i: written, or added to what is there (accumulate)
    auto put = [&](int c, float val) {
        float *q = grads + (size_t)c * n + i;
        *q = accumulate ? *q + val : val;
    };
#pragma unroll
    for (int a = 0; a < 3; a++) {
        put(a, dmu[a]);
        put(3 + a, ds[a] * g.s[a]);
    }
#pragma unroll
    for (int a = 0; a < 4; a++) put(6 + a, (dqn[a] - g.qn[a] * qdot) * g.qinv);
    put(10, g.o * (1.f - g.o) * dop);
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) put(11 + 3 * k + ch, dsh[k][ch]);
}

// The row table of fovea culling: per view and tile row, the columns of the
// tiles that can hold a pixel of the disk (fovea_tile_live, one interval per
// row: its first and last), or none (lo > hi).  One wave per row, a lane per
// column.
__global__ __launch_bounds__(256) void k_fovea_rows(const float *__restrict__ gaze, float radius_frac,
                                                    const ViewDesc *__restrict__ views, int nviews,
                                                    int tile, int per_view, uint2 *__restrict__ rows) {
    const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    if (i >= nviews * per_view) return;
    const int v = i / per_view, ty = i - v * per_view;
    const ViewDesc vd = views[v];
    int lo = INT_MAX, hi = -1;
    if (ty < vd.tiles_y) {
        for (int t0 = 0; t0 < vd.tiles_x; t0 += 64) {
            const int tx = t0 + lane;
            const bool live = tx < vd.tiles_x &&
                              fovea_tile_live(gaze, v, radius_frac, vd.width, vd.height, tile, tx, ty);
            const uint64_t m = __ballot(live);
            if (m) {
                lo = min(lo, t0 + __builtin_ctzll(m));
                hi = t0 + 63 - __builtin_clzll(m);
            }
        }
    }
    if (lane == 0) rows[i] = hi >= 0 ? make_uint2((uint32_t)lo, (uint32_t)hi) : make_uint2(1u, 0u);
}

}  // namespace

void launch_project_fwd(hipStream_t s, const float *P, int n, int nviews, int deg,
                        const gsf_camera *cams, const ViewDesc *views, int tile, SplatPtrs sp,
                        uint32_t *depth_key, uint2 *rect, uint32_t *count, uint2 *rspan,
                        const float *cull_gaze, float cull_radius, const FoveaRows &fr,
                        uint32_t *block_sums,
                        uint32_t *block_act) {
    const int nrec = n * nviews;
    const dim3 grid((nrec + 255) / 256), block(256);
    if (deg <= 1 && nviews > 1) {   // one thread per Gaussian for all views, then the block totals
        const dim3 ggrid((n + 255) / 256);
        if (deg == 0)
            k_project_fwd_views<0><<<ggrid, block, 0, s>>>(P, n, nviews, cams, views, tile, sp, depth_key,
                                                            rect, count, rspan, cull_gaze, cull_radius, fr);
        else
            k_project_fwd_views<1><<<ggrid, block, 0, s>>>(P, n, nviews, cams, views, tile, sp, depth_key,
                                                            rect, count, rspan, cull_gaze, cull_radius, fr);
        k_block_totals<<<(nrec + 1023) / 1024, block, 0, s>>>(count, nrec, block_sums, block_act);
        return;
    }
    switch (deg) {
    case 0: k_project_fwd<0><<<grid, block, 0, s>>>(P, n, nrec, cams, views, tile, sp, depth_key, rect, count, rspan, cull_gaze, cull_radius, fr, block_sums, block_act); break;
    case 1: k_project_fwd<1><<<grid, block, 0, s>>>(P, n, nrec, cams, views, tile, sp, depth_key, rect, count, rspan, cull_gaze, cull_radius, fr, block_sums, block_act); break;
    case 2: k_project_fwd<2><<<grid, block, 0, s>>>(P, n, nrec, cams, views, tile, sp, depth_key, rect, count, rspan, cull_gaze, cull_radius, fr, block_sums, block_act); break;
    default: k_project_fwd<3><<<grid, block, 0, s>>>(P, n, nrec, cams, views, tile, sp, depth_key, rect, count, rspan, cull_gaze, cull_radius, fr, block_sums, block_act); break;
    }
}

void launch_fovea_rows(hipStream_t s, const float *gaze, float radius_frac, const ViewDesc *views,
                       int nviews, int tile, const FoveaRows &fr) {
    const int total = nviews * fr.per_view;   // one wave per row, four per workgroup
    k_fovea_rows<<<(total + 3) / 4, 256, 0, s>>>(gaze, radius_frac, views, nviews, tile, fr.per_view,
                                                  const_cast<uint2 *>(fr.rows));
}

bool project_bwd_sums_keys(int deg) { return deg <= 1; }

void launch_project_bwd(hipStream_t s, const float *P, int n, int nviews, int deg,
                        const gsf_camera *cams, const KeyPlace &kp, const float *g2d, float *grads,
                        bool accumulate) {
    const dim3 grid((n + 127) / 128), block(128);
    switch (deg) {
    case 0: k_project_bwd<0, true><<<grid, block, 0, s>>>(P, n, nviews, cams, kp, g2d, grads, accumulate); break;
    case 1: k_project_bwd<1, true><<<grid, block, 0, s>>>(P, n, nviews, cams, kp, g2d, grads, accumulate); break;
    case 2: k_project_bwd<2, false><<<grid, block, 0, s>>>(P, n, nviews, cams, kp, g2d, grads, accumulate); break;
    default: k_project_bwd<3, false><<<grid, block, 0, s>>>(P, n, nviews, cams, kp, g2d, grads, accumulate); break;
    }
}

}  // namespace gsf
