/*
 * raymarch.c - emission-absorption ray march of a uint16 volume (input
 * generator for target images; same definition as synth.raymarch with the
 * trilinear transfer-function sampler, written in C for large images).
 *
 * Volume vol[ix][iy][iz] (C order) spans [-1, 1]^3 with voxel centres at
 * (idx + 1/2) * 2/n - 1; samples are trilinear in the raw values with zero
 * outside the grid.  Density t = clamp((v - thr) / range, 0, 1); colour =
 * lo (1 - t) + hi t; alpha = 1 - exp(-extinction * t * length) per segment of
 * length `step` from the box entry (the last one shortened to the exit),
 * sampled at segment midpoints; the march stops once T < t_stop.
 * cam: R[9] (world -> camera, row-major), campos[3], fx, fy, cx, cy, bg[3], w, h.
 * out: float [4][nrows][w] = RGB + bg T, A = 1 - T.
 */
#include <math.h>
#include <stdint.h>

static double sample(const uint16_t *vol, int n, double x, double y, double z) {
    const double ux = (x + 1.0) * (n / 2.0) - 0.5, uy = (y + 1.0) * (n / 2.0) - 0.5,
                 uz = (z + 1.0) * (n / 2.0) - 0.5;
    const double fx0 = floor(ux), fy0 = floor(uy), fz0 = floor(uz);
    const int64_t i0 = (int64_t)fx0, j0 = (int64_t)fy0, k0 = (int64_t)fz0;
    const double fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    double acc = 0.0;
    for (int dx = 0; dx < 2; dx++)
        for (int dy = 0; dy < 2; dy++)
            for (int dz = 0; dz < 2; dz++) {
                const int64_t i = i0 + dx, j = j0 + dy, k = k0 + dz;
                if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) continue;
                const double w = (dx ? fx : 1 - fx) * (dy ? fy : 1 - fy) * (dz ? fz : 1 - fz);
                acc += w * (double)vol[(i * n + j) * n + k];
            }
    return acc;
}

void syn_raymarch(const uint16_t *vol, int n, const double *cam, const int64_t *rows, int64_t nrows,
                  double step, double extinction, double t_stop, const double *lo, const double *hi,
                  double thr, double range, float *out) {
    const double *R = cam, *o = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    const double *bg = cam + 16;
    const int64_t W = (int64_t)cam[19];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t rr = 0; rr < nrows; rr++) {
        const int64_t j = rows[rr];
        for (int64_t i = 0; i < W; i++) {
            const double dc[3] = {((double)i + 0.5 - cx) / fx, ((double)j + 0.5 - cy) / fy, 1.0};
            double d[3];
            for (int a = 0; a < 3; a++) d[a] = R[a] * dc[0] + R[3 + a] * dc[1] + R[6 + a] * dc[2];
            const double nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int a = 0; a < 3; a++) d[a] /= nn;
            double t0 = -INFINITY, t1 = INFINITY;
            for (int a = 0; a < 3; a++) {
                const double inv = 1.0 / d[a];
                double ta = (-1.0 - o[a]) * inv, tb = (1.0 - o[a]) * inv;
                if (ta > tb) { const double tmp = ta; ta = tb; tb = tmp; }
                if (ta > t0) t0 = ta;
                if (tb < t1) t1 = tb;
            }
            if (t0 < 0) t0 = 0;
            double C[3] = {0, 0, 0}, T = 1.0;
            if (t1 > t0) {
                for (int64_t k = 0;; k++) {
                    const double s0 = t0 + (double)k * step;
                    double s1 = s0 + step;
                    if (s1 > t1) s1 = t1;
                    if (!(s1 > s0)) break;
                    const double mid = 0.5 * (s0 + s1);
                    const double v = sample(vol, n, o[0] + d[0] * mid, o[1] + d[1] * mid, o[2] + d[2] * mid);
                    double t = (v - thr) / range;
                    t = t < 0 ? 0 : (t > 1 ? 1 : t);
                    if (t > 0) {
                        const double alpha = 1.0 - exp(-extinction * t * (s1 - s0));
                        for (int c = 0; c < 3; c++) C[c] += (lo[c] * (1 - t) + hi[c] * t) * alpha * T;
                        T *= 1.0 - alpha;
                        if (T < t_stop) break;
                    }
                }
            }
            const int64_t q = rr * W + i, plane = nrows * W;
            for (int c = 0; c < 3; c++) out[c * plane + q] = (float)(C[c] + T * bg[c]);
            out[3 * plane + q] = (float)(1.0 - T);
        }
    }
}
