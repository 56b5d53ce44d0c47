/*
 * gsfit.h - C ABI of the MI355X (gfx950) differentiable Gaussian-splatting fit path.
 *
 * The paper (arXiv 2601.22026, Method section, "Periphery Model Training")
 * fits its peripheral model of anatomy by optimising 3D Gaussians against posed
 * renderings with a 3D Gaussian Splatting rasterizer and Adam; its continual
 * refinement restarts the optimiser with reloaded Gaussians and discarded
 * optimiser state.  This library implements that fit step on one GPU:
 *
 *   gsf_forward   Gaussians + cameras -> RGBA images        (projection, key
 *                 duplication, (tile, depth) sort, per-tile front-to-back
 *                 alpha compositing)
 *   gsf_loss_l1   images + targets -> mean L1 loss, dL/dRGBA (optional circular
 *                 fovea mask per view)
 *   gsf_backward  dL/dRGBA -> dL/d(parameters)              (adjoint of the above)
 *   gsf_adam      bias-corrected Adam with per-segment learning rates
 *   gsf_step_*    the four calls above as one captured HIP graph
 *   continual refinement: gsf_view_select (Eq. (1), host), gsf_adam_reset
 *                 (restart with discarded optimiser state), gsf_adam_masked
 *                 and gsf_step_args.masked_adam (visibility-masked update)
 *   seeding: gsf_seed_volume (Gaussians from a CT volume's voxels),
 *                 gsf_seed_first_hits (Gaussians at the first significant hits
 *                 of rays from several viewpoints), gsf_raymarch
 *                 (emission-absorption target images)
 *   viewer: gsf_reproject, gsf_reproject_warp (depth-guided reprojection of
 *                 the foveal image)
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every pointer is DEVICE memory unless its comment says (host).  The caller
 *   owns all device buffers (parameters, gradients, optimiser state, images,
 *   targets, cameras, workspace).  The library owns only the opaque host-side
 *   context and plan objects and the graphs it instantiates.
 * - Every call is asynchronous on the context's stream, except gsf_poll,
 *   gsf_debug_copy, gsf_seed_volume, gsf_seed_first_hits and (for plans
 *   created with host_sized = 1) gsf_forward, which synchronise that stream, and
 *   gsf_view_select, which runs on the host only.
 * - Errors: every call returns a gsf_status; no exception crosses the ABI.
 *   Argument errors are detected on the host before anything is enqueued.
 *   Conditions detected on the device (key overflow, non-finite loss) set sticky
 *   flags read by gsf_poll.  gsf_last_error() returns a context-owned message
 *   valid until the next call on that context.
 * - Parameters: planar float32 [C][n], C = 11 + 3K, K = (sh_degree + 1)^2:
 *     planes 0..2 mean xyz, 3..5 log-scale xyz, 6..9 rotation quaternion
 *     (w, x, y, z; normalised inside), 10 opacity logit, 11 + 3k + c SH
 *     coefficient k (k = l*l + l + m) of colour channel c.
 *   Gradients use the same layout.
 * - Images: per view planar float32 [4][H][W] (R, G, B, A), views concatenated
 *   in plan order.  Targets: per view [3][H][W], concatenated likewise.
 * - Cameras: a device array of gsf_camera, one per view, in plan order.  They
 *   live in device memory so captured graphs see updated poses.
 * - Pixel (i, j) has its centre at (i + 0.5, j + 0.5); camera axes are x right,
 *   y down, z forward.
 */
#ifndef GSFIT_H
#define GSFIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSF_OK = 0,
    GSF_E_INVALID = 1,     /* bad argument (null pointer, size out of range, bad option) */
    GSF_E_CAPACITY = 2,    /* key count exceeded the plan's key capacity */
    GSF_E_HIP = 3,         /* a HIP runtime call failed; see gsf_last_error */
    GSF_E_STATE = 4,       /* call out of order (no workspace, no forward, no graph) */
    GSF_E_NONFINITE = 5,   /* non-finite loss detected */
    GSF_E_UNSUPPORTED = 6  /* option the library does not support */
} gsf_status;

/* sticky device flags reported by gsf_poll */
#define GSF_FLAG_CAPACITY 1u
#define GSF_FLAG_NONFINITE 2u

typedef struct gsf_ctx gsf_ctx;
typedef struct gsf_plan gsf_plan;

/* One pinhole camera (128 bytes). */
typedef struct gsf_camera {
    float viewmat[12];          /* world -> camera [R | t], row-major 3x4 */
    float campos[3];            /* camera centre in world (SH view direction) */
    float fx, fy, cx, cy;       /* focal lengths and principal point, pixels */
    float tan_half_fov_x;       /* half-FOV tangents: the projection Jacobian is */
    float tan_half_fov_y;       /*   evaluated at x/z clamped to +-1.3 of these  */
    float znear;                /* Gaussians with camera depth <= znear are culled */
    float bg[3];                /* background colour composited behind the Gaussians */
    int32_t width, height;      /* image size, pixels (1 .. 8192) */
    int32_t reserved[5];        /* must be zero */
} gsf_camera;

/* Plan description: everything that fixes workspace sizes and launch shapes. */
typedef struct gsf_plan_desc {
    int64_t n_max;              /* maximum Gaussian count per call (>= 1) */
    int32_t sh_degree;          /* 0 .. 3 */
    int32_t n_views;            /* 1 .. 64 */
    const int32_t *widths;      /* (host) [n_views] */
    const int32_t *heights;     /* (host) [n_views] */
    int32_t tile;               /* tile edge in pixels: 8, 16 or 32 */
    int32_t lds_batch;          /* Gaussians staged in LDS per batch: 64, 128 or 256 */
    int32_t t_mode;             /* transmittance in the adjoint:
                                   0 recomputed back to front from the final
                                     transmittance (8 B/pixel saved; one workgroup
                                     per tile);
                                   1 checkpointed: the forward also stores (T, colour)
                                     per pixel at every LDS-batch boundary
                                     (16 B/pixel/boundary) and the adjoint runs one
                                     workgroup per (tile, batch);
                                   2 stored: the forward stores T in front of every
                                     included (Gaussian, pixel) pair, key capacity x
                                     tile^2 x 4 B; one workgroup per tile */
    int32_t host_sized;         /* 1: gsf_forward reads the key count back to the host
                                   and sizes the sort from it (plain path);
                                   0: the count stays on the device (capturable) */
    int64_t key_capacity;       /* maximum (tile, Gaussian) keys; 0 = 32 per record + 2^20 */
} gsf_plan_desc;

/* ---- context ---------------------------------------------------------------- */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns GSF_E_HIP if the device
 * cannot be selected. */
gsf_status gsf_ctx_create(int device, void *hip_stream, gsf_ctx **out);
gsf_status gsf_ctx_destroy(gsf_ctx *ctx);
/* Change the stream later calls enqueue on. */
gsf_status gsf_ctx_set_stream(gsf_ctx *ctx, void *hip_stream);
/* Last error message of this context (context-owned, never NULL). */
const char *gsf_last_error(const gsf_ctx *ctx);

/* ---- plans --------------------------------------------------------------------- */

/* Validate `desc` and create a plan.  Widths/heights are copied. */
gsf_status gsf_plan_create(gsf_ctx *ctx, const gsf_plan_desc *desc, gsf_plan **out);
/* Bytes of device workspace the plan needs (written to *bytes, host). */
gsf_status gsf_plan_workspace_bytes(const gsf_plan *plan, size_t *bytes);
/* Bind caller-owned device workspace of at least gsf_plan_workspace_bytes bytes,
 * 256-byte aligned.  The state saved by gsf_forward for gsf_backward lives here
 * and stays valid until the next gsf_forward on the same plan. */
gsf_status gsf_plan_bind_workspace(gsf_plan *plan, void *dev, size_t bytes);
/* Totals of the plan (host): tiles over all views, pixels over all views. */
gsf_status gsf_plan_info(const gsf_plan *plan, int64_t *total_tiles, int64_t *total_pixels);
gsf_status gsf_plan_destroy(gsf_plan *plan);

/* ---- the fit step --------------------------------------------------------------- */

/* Render all views of the plan: the 3D Gaussian Splatting image formation the
 * paper's fit adopts (Related Work, "Novel View Synthesis"; Method, "Periphery
 * Model Training": Mini-Splatting2 with the rasterization of Taming 3DGS) -
 * each Gaussian projected to a screen-space conic (EWA splatting: local affine
 * approximation of the perspective map, 0.3 px^2 low-pass), listed in the
 * tiles its opacity-aware support ellipse reaches, sorted by (tile, depth), and
 * composited front to back per pixel (alpha = min(0.99, o e^power), skipped
 * below 1/255, stopping before transmittance falls under 1e-4; RGB = C + T bg,
 * A = 1 - T).  params: [C][n] (1 <= n <= n_max); cams: [n_views]; out_rgba:
 * concatenated per-view [4][H][W] (caller-owned).  cull_gaze_px: nullable device
 * [n_views][2]; when given (with cull_radius_frac in [0, 4]), only the pixels of
 * each view's fovea disk (centre within cull_radius_frac * width of the gaze
 * point, the loss's FP32 mask test) are composited: the other pixels of the
 * tiles composited are written as background with alpha 0, and the tiles that
 * cannot hold a pixel of the disk (outside the fovea box, or in its corners
 * when the box's tiles are fewer than the plan's) may be left as they were; a
 * later gsf_loss_l1 with the same gaze and radius reads only the disk.  With host_sized = 1 this synchronises the
 * stream once and returns GSF_E_CAPACITY if the key count exceeded the capacity
 * (the image is then background only).  GSF_E_INVALID for null pointers, n out
 * of range or a bad radius; GSF_E_STATE without a workspace. */
gsf_status gsf_forward(gsf_plan *plan, const float *params, int64_t n, const gsf_camera *cams,
                       const float *cull_gaze_px, float cull_radius_frac, float *out_rgba);

/* The fit's image loss (Method, "Periphery Model Training": the model is
 * optimised against the rendered training views; L1 on colour, the 3DGS
 * photometric term; the fovea mask restricts a foveated view to the region it
 * renders): the mean absolute error over the masked (view, pixel, RGB channel)
 * entries of `rgba` against `target_rgb` (concatenated per-view [3][H][W]).
 * gaze_px: nullable device [n_views][2] pixel coordinates; when given, only
 * pixels whose centre lies within mask_radius_frac * width of the gaze point
 * count.  norm_count: 0 = divide by this plan's own masked entry count; > 0 =
 * divide by it instead (the entry count over every plan of a loss split across
 * plans, e.g. one plan per view; see gsf_loss_count).  accumulate: 0 = loss[0]
 * = this plan's mean, 1 = loss[0] += it.  Writes the loss to loss[0] (device)
 * and dL/dRGBA (sign / count; alpha plane zero) to dl_drgba (concatenated
 * per-view [4][H][W]); after a fovea-culled gsf_forward on this plan (same gaze
 * and radius), only the masked-in pixels of dl_drgba are written (gsf_backward
 * reads no other).  A non-finite loss sets GSF_FLAG_NONFINITE.
 * GSF_E_INVALID for null pointers, a bad radius, norm_count outside
 * [0, 2^32 - 1] or accumulate not 0/1. */
gsf_status gsf_loss_l1(gsf_plan *plan, const float *rgba, const float *target_rgb,
                       const float *gaze_px, float mask_radius_frac, int64_t norm_count,
                       int32_t accumulate, float *loss, float *dl_drgba);

/* Number of entries gsf_loss_l1 averages over on this plan (host *count): 3 x
 * pixels without a gaze, else 3 x the pixels inside the fovea masks.
 * Synchronises the context stream. */
gsf_status gsf_loss_count(gsf_plan *plan, const float *gaze_px, float mask_radius_frac,
                          int64_t *count);

/* Gradient of the loss w.r.t. the parameters (the adjoint of gsf_forward, which
 * the fit's gradient-based optimisation needs; Method, "Periphery Model
 * Training") given dL/dRGBA of the last gsf_forward on this plan (same params,
 * n and cams): back to front through the compositing, then through the conic
 * projection to mean, log-scale, rotation, opacity logit and SH colour, summed
 * over the plan's views.  grads: [C][n]; accumulate = 0 overwrites it, 1 adds
 * to it (a gradient summed over several plans).  GSF_E_STATE before a forward;
 * GSF_E_INVALID for null pointers, n differing from the forward's or
 * accumulate not 0/1. */
gsf_status gsf_backward(gsf_plan *plan, const float *params, int64_t n, const gsf_camera *cams,
                        const float *dl_drgba, int32_t accumulate, float *grads);

/* The fit's optimiser (Method, "Periphery Model Training": the Mini-Splatting2
 * / 3DGS optimisation, Adam; per-group learning rates, which the paper raises
 * by about 50 % for scale, opacity and colour).
 * One Adam step on n_elems float32 elements: m <- b1 m + (1-b1) g,
 * v <- b2 v + (1-b2) g^2, p <- p - lr m_hat / (sqrt(v_hat) + eps), with bias
 * correction by the step number held in step_dev[0] (device int32), which this
 * call increments first.  Element e uses seg_lr[s] for seg_off[s] <= e <
 * seg_off[s+1] (host arrays, n_seg in 1..16, seg_off[0] = 0,
 * seg_off[n_seg] = n_elems).  Resetting m, v and step_dev to zero restarts the
 * optimiser (continual refinement by restart). */
gsf_status gsf_adam(gsf_ctx *ctx, float *p, const float *g, float *m, float *v, int64_t n_elems,
                    const int64_t *seg_off, const float *seg_lr, int32_t n_seg, float beta1,
                    float beta2, float eps, int32_t *step_dev);

/* Visibility-masked Adam on planar [planes][n] float32 state (p, g, m, v device
 * arrays, planes in 1..64): for every Gaussian i with visible[i] != 0 (device
 * uint8 [n]) each plane c takes the Adam step of gsf_adam at plane_lr[c] (host
 * [planes]); Gaussians with visible[i] == 0 keep p, m and v unchanged (they are
 * not read or written).  step_dev[0] is incremented first and its new value is
 * the step number of the bias correction for every Gaussian.  This is the sparse
 * Adam of Taming 3DGS, which the paper's optimiser adopts (Method, "Periphery
 * Model Training").  GSF_E_INVALID for null pointers, n < 1, planes out of
 * range or a non-finite learning rate. */
gsf_status gsf_adam_masked(gsf_ctx *ctx, float *p, const float *g, float *m, float *v, int64_t n,
                           int32_t planes, const float *plane_lr, const uint8_t *visible,
                           float beta1, float beta2, float eps, int32_t *step_dev);

/* Optimiser restart of the continual refinement (Method, "Periphery Model
 * Training": optimisation restarts from the current Gaussians with the
 * optimiser state discarded): m[0..n_elems) = v[0..n_elems) = 0 and
 * step_dev[0] = 0, written by a kernel on the context stream (no memset, so a
 * captured graph may hold it).  m and v: device, 16-byte aligned. */
gsf_status gsf_adam_reset(gsf_ctx *ctx, float *m, float *v, int64_t n_elems, int32_t *step_dev);

/* Training-view selection of the continual refinement (Method, "Periphery Model
 * Training", Eq. (1)).  The candidates are offered in order; candidate j is kept
 * (keep[j] = 1, else 0) when for every view of the set - the n_set views of
 * `set`, then the candidates kept before j - the camera centres (campos) lie
 * more than delta_pos apart or the unit viewing directions d satisfy
 * d_j . d_i < cos(theta_view_deg).  d is the camera's +z axis in world
 * coordinates: the third row of viewmat's rotation, normalised.  An empty set
 * keeps the first candidate.  The paper sets delta_pos = 0.05 (scene units) and
 * theta_view = 5 degrees.  All arrays are host memory (set may be NULL when
 * n_set = 0); evaluated on the host in double precision; no context, no device
 * work.  *n_kept: the number of kept candidates.  GSF_E_INVALID for null
 * pointers, negative counts, delta_pos < 0 or non-finite, theta outside
 * [0, 180], or a camera with a zero or non-finite direction or centre (then
 * nothing is written to keep). */
gsf_status gsf_view_select(const gsf_camera *set, int32_t n_set, const gsf_camera *cand,
                           int32_t n_cand, float delta_pos, float theta_view_deg, int32_t *keep,
                           int32_t *n_kept);

/* Depth-guided reprojection of a foveal image (Method, "Real-time Viewer",
 * Eqs. (2)-(4)).  Pixel (i, j) of a width x height image has texture
 * coordinate uv = ((i + 0.5) / width, (j + 0.5) / height) and first-hit
 * distance depth[j * width + i] (device float32, world units).  Its far-plane
 * point is p_far = (h.x, h.y, h.z) / h.w with h = (P_old V_old)^-1 (2u - 1,
 * 2v - 1, 1, 1); its world point is pos_old + depth (p_far - pos_old) /
 * |p_far - pos_old|; clip = P_new V_new (p_world, 1).  Matrices: host float32
 * [16], row-major, for column vectors (clip = M x); pos_old: host float32 [3].
 * P V products and the inverse are formed on the host in double, the per-pixel
 * work on the device in float32.  clip: device float32 [4][height][width]
 * (x, y, z, w planes), NaN where the depth is not finite and positive.
 * GSF_E_INVALID for null pointers, sizes outside 1..16384, a singular
 * P_old V_old or a non-finite matrix entry. */
gsf_status gsf_reproject(gsf_ctx *ctx, const float *depth, int32_t width, int32_t height,
                         const float *p_old, const float *v_old, const float *pos_old,
                         const float *p_new, const float *v_new, float *clip);

/* The foveal image moved to the new view by its reprojected points (the
 * viewer's depth-deformed image, Method "Real-time Viewer", drawn as points):
 * every pixel with a depth lands on the output pixel (floor(x), floor(y)) with
 * x = (ndc_x + 1) / 2 * out_width, y = (ndc_y + 1) / 2 * out_height, if clip
 * w > 0, ndc_z in [-1, 1] and (x, y) inside; where several land the smallest
 * clip w wins, ties to the lower source index j * width + i.  rgba: device
 * [4][height][width]; zbuf: device scratch of out_width * out_height uint64
 * (8-byte aligned, overwritten); out_rgba: device [4][out_height][out_width],
 * the winner's four values, zero where nothing lands; out_src: device int32
 * [out_height][out_width], the winner's source index or -1.  The gaps are the
 * disocclusions the peripheral model fills.  Errors as gsf_reproject. */
gsf_status gsf_reproject_warp(gsf_ctx *ctx, const float *rgba, const float *depth, int32_t width,
                              int32_t height, const float *p_old, const float *v_old,
                              const float *pos_old, const float *p_new, const float *v_new,
                              int32_t out_width, int32_t out_height, uint64_t *zbuf,
                              float *out_rgba, int32_t *out_src);

/* gsf_reproject_warp without the zbuf argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, a viewer's per-frame
 * loop, harnesses that forbid allocation).  The z-buffer is a device-resident
 * array inside the library, one per GPU, of 2048 x 2304 64-bit entries
 * (36 MiB, held until the process ends): out_width * out_height may not exceed
 * 4,718,592 (GSF_E_INVALID otherwise; use gsf_reproject_warp then).  Its
 * address is looked up once per device when a context is created.  This call
 * allocates nothing; it clears the z-buffer itself each time, writes the same
 * outputs as gsf_reproject_warp and has the same errors, plus GSF_E_HIP if the
 * z-buffer's address could not be found.  Every call on one GPU shares that
 * z-buffer: calls that overlap on one GPU (different streams, or contexts on
 * different streams) race and must be ordered by the caller. */
gsf_status gsf_reproject_warp_noalloc(gsf_ctx *ctx, const float *rgba, const float *depth,
                                      int32_t width, int32_t height, const float *p_old,
                                      const float *v_old, const float *pos_old, const float *p_new,
                                      const float *v_new, int32_t out_width, int32_t out_height,
                                      float *out_rgba, int32_t *out_src);

/* Arguments of one full step: forward, loss, backward, Adam on the parameters. */
typedef struct gsf_step_args {
    float *params;              /* [C][n]; updated in place by Adam */
    int64_t n;
    const gsf_camera *cams;
    const float *target_rgb;
    const float *gaze_px;       /* nullable */
    float mask_radius_frac;
    float *loss;                /* [1] */
    float *rgba;                /* image buffer */
    float *dl_drgba;            /* image-sized gradient buffer */
    float *grads;               /* [C][n] */
    float *adam_m, *adam_v;     /* [C][n] each */
    int32_t *step_dev;          /* [1] */
    const float *seg_lr;        /* (host) [11 + 3K]: learning rate per parameter plane */
    float beta1, beta2, eps;
    int32_t fovea_cull;         /* 1: with gaze_px, composite and back-propagate only the
                                   pixels of each view's fovea disk (the loss's mask), over
                                   the tiles of its fovea box that can hold one; loss and
                                   gradients are those of the full frame (other pixels
                                   carry no loss); rgba outside the disk is background or
                                   left as it was, as gsf_forward says; dl_drgba outside
                                   the disk is left as it was.  0: full frames. */
    int32_t alpha_loss;         /* 1: target_rgb is RGBA per view ([4][H][W], colour
                                   premultiplied) and the L1 also covers alpha (alpha
                                   training, Method "Periphery Model Training") */
    int32_t random_bg;          /* 1 (needs alpha_loss): every step draws one background
                                   colour per view (SplitMix64 from bg_seed, output
                                   1 + (step * 64 + v) * 4 + c, top 24 bits scaled to
                                   [0, 1), step = *step_dev before the step) and renders,
                                   differentiates and compares over it; the target is
                                   composited over it as rgb + (1 - alpha) bg.  The
                                   cameras' bg is not used then.  0: the cameras' bg. */
    uint64_t bg_seed;
    int32_t masked_adam;        /* 1: visibility-masked Adam (the sparse Adam of Taming
                                   3DGS, on which the paper's optimiser builds): only the
                                   Gaussians that touched at least one tile in some view
                                   of this step (with fovea_cull: a tile of the fovea
                                   boxes) take the Adam update; the others keep their
                                   parameters, m and v.  Bias correction still uses the
                                   shared step counter.  0: every Gaussian is updated. */
} gsf_step_args;

/* L1 of an RGBA prediction against RGBA targets (alpha training): the target
 * colour is premultiplied and composited over bg (device [n_views][3], NULL =
 * black) as rgb + (1 - alpha) bg; the mean runs over R, G, B and, with
 * alpha != 0, A of every masked pixel (mask as in gsf_loss_l1).  rgba as
 * produced by gsf_forward with the same bg in the cameras; dl_drgba receives
 * the sign gradient of all four planes.  Same ownership and errors as
 * gsf_loss_l1. */
gsf_status gsf_loss_l1_rgba(gsf_plan *plan, const float *rgba, const float *target_rgba,
                            const float *bg, int32_t alpha, const float *gaze_px,
                            float mask_radius_frac, float *loss, float *dl_drgba);

/* ---- tile size and LDS batch by measurement ----------------------------------------- */

/* The candidates of gsf_autotune.  80 bytes. */
typedef struct gsf_tune_space {
    int32_t n_tiles;            /* 1 .. 3 */
    int32_t tiles[3];           /* each 8, 16 or 32 */
    int64_t key_capacity[3];    /* key capacity of the plans of tiles[k] (0: the plan default) */
    int32_t n_batches;          /* 1 .. 3 */
    int32_t batches[3];         /* each 64, 128 or 256 */
    int32_t n_t_modes;          /* 1 .. 3 */
    int32_t t_modes[3];         /* each 0, 1 or 2 (gsf_plan_desc.t_mode) */
    int32_t warmup;             /* untimed replays per candidate (>= 0) */
    int32_t reps;               /* timed replays per candidate (>= 1) */
} gsf_tune_space;

/* 120 bytes. */
typedef struct gsf_tune_result {
    int32_t tile, lds_batch, t_mode;   /* the fastest candidate */
    float ms[27];                      /* ms per step of candidate (tiles[k], batches[j],
                                          t_modes[m]) at [9 k + 3 j + m]; -1 outside the
                                          space; +inf when its keys overflowed */
} gsf_tune_result;

/* Device workspace (bytes, host) gsf_autotune needs: the largest candidate
 * plan plus 256 bytes. */
gsf_status gsf_autotune_workspace_bytes(gsf_ctx *ctx, const gsf_plan_desc *base,
                                        const gsf_tune_space *space, size_t *bytes);
/* Pick the tile size, LDS batch and adjoint transmittance mode that make the
 * captured fused step fastest on this input (the fused, captured form of the
 * fit step: one launch per stage over every view).  For every candidate a plan
 * is made from `base` (n_max, SH degree, views) with that tile, batch, mode and
 * the tile's key capacity, device-sized, bound to `workspace` (caller-owned,
 * 256-byte aligned, gsf_autotune_workspace_bytes long); the forward, loss and
 * backward of `args` (with its options: fovea culling, alpha loss, random
 * backgrounds) are captured in a HIP graph, replayed `warmup` times, then timed
 * with HIP events over `reps` replays on the context stream.  Adam is left
 * out, its time does not depend on the candidate, so params, adam_m, adam_v
 * and *step_dev are not touched (a private step counter drives the loss and
 * the backgrounds); rgba, dl_drgba, grads and loss are overwritten.  A
 * candidate whose keys overflow its capacity is timed +inf.  Writes *out
 * (host).  Synchronises the stream.  GSF_E_INVALID for a bad space, null
 * pointers or a short workspace; GSF_E_STATE on the null stream (graphs cannot
 * be captured there); GSF_E_CAPACITY when every candidate overflowed. */
gsf_status gsf_autotune(gsf_ctx *ctx, const gsf_plan_desc *base, const gsf_tune_space *space,
                        const gsf_step_args *args, void *workspace, size_t bytes,
                        gsf_tune_result *out);

/* Enqueue one step eagerly.  With host_sized = 0 the key count stays on the
 * device: if it exceeds the plan's capacity the step sets GSF_FLAG_CAPACITY
 * and leaves parameters, m, v and *step_dev untouched (its image, loss and
 * gradients are undefined); every later step does the same until gsf_poll
 * clears the flag, so after a re-plan with more capacity the same step can be
 * run again. */
gsf_status gsf_step(gsf_plan *plan, const gsf_step_args *args);
/* Capture one step into a HIP graph owned by the plan (replaces any previous
 * one).  Needs host_sized = 0.  Nothing runs during capture. */
gsf_status gsf_step_capture(gsf_plan *plan, const gsf_step_args *args);
/* Launch the captured graph once on the context stream. */
gsf_status gsf_step_replay(gsf_plan *plan);

/* ---- the CT volume on the device --------------------------------------------------- */

/* Seeding (Method, "Periphery Model Training": the model starts from Gaussians
 * placed on the volume's structures).  vol: device uint16 [n][n][n] (C order,
 * spanning [-1, 1]^3, voxel centres at (idx + 1/2) 2/n - 1).  One Gaussian per
 * voxel with value > threshold, in raster order; above cap candidates, the cap
 * with the smallest priority are kept (priority of flat index idx: SplitMix64
 * output idx + 1 from state seed with its low b bits replaced by idx, b = bits
 * of n^3 - 1), still in raster order.  Each: mean = voxel centre, log-scale
 * ln(2/n) on all axes, rotation (1, 0, 0, 0), opacity logit ln(o / (1 - o)),
 * degree-0 SH (col - 1/2) / Y00 with col = lo (1 - t) + hi t, t = clamp((v -
 * threshold) / range, 0, 1); computed in double, rounded once to float.
 * params: device float with room for 14 * cap values, written planar [14][m];
 * *count (host) = m = min(candidates, cap).  scratch: device memory of
 * gsf_seed_scratch_bytes(n) bytes.  Synchronises the context stream. */
gsf_status gsf_seed_scratch_bytes(int32_t n, size_t *bytes);

/* First-hit point cloud (Method, "Volumetric Path Tracing": rays cast at the
 * volume from viewpoints around it; the first significant hit of each ray
 * becomes a point, coloured by marching on from it).  Every pixel-centre ray of
 * the n_views cameras (device gsf_camera array; widths, heights: host, must
 * equal the cameras' sizes; rays numbered in view, row, column order) is
 * marched through [-1, 1]^3 as gsf_raymarch does (segments of `step` from the
 * box entry, midpoint samples, t = clamp((v - threshold) / range, 0, 1),
 * segment opacity 1 - exp(-extinction t length)).  The hit is the midpoint of
 * the first segment after which the accumulated opacity reaches hit_alpha
 * (in (0, 1)); its colour is the emission-absorption colour lo (1 - t) + hi t
 * (lo, hi: host [3]) of that segment and the next color_steps - 1 (or up to the
 * exit) composited from zero opacity, divided by their accumulated opacity.
 * Above cap hits, the cap rays with the smallest priority are kept (ray r:
 * SplitMix64 output r + 1 from state seed with its low b bits replaced by r,
 * b = bits of (rays - 1)), in ray order.  Each point becomes a Gaussian: mean at
 * the hit, log-scale ln(2/n), rotation (1, 0, 0, 0), opacity logit
 * ln(o / (1 - o)), degree-0 SH (colour - 1/2) / Y00; the march runs in float.
 * params: device float with room for 14 * cap values, written planar [14][m];
 * ray_ids: nullable device int32 [cap], the ray of each Gaussian; *count (host)
 * = m.  scratch: device memory of gsf_first_hit_scratch_bytes(rays) bytes,
 * 256-byte aligned.  Synchronises the context stream.  GSF_E_INVALID for null
 * pointers, sizes or parameters out of range or a short scratch. */
gsf_status gsf_first_hit_scratch_bytes(int64_t n_rays, size_t *bytes);
gsf_status gsf_seed_first_hits(gsf_ctx *ctx, const uint16_t *vol, int32_t n, const gsf_camera *cams,
                               int32_t n_views, const int32_t *widths, const int32_t *heights,
                               float step, float extinction, float threshold, float range,
                               const float *lo, const float *hi, float hit_alpha,
                               int32_t color_steps, double opacity, int64_t cap, uint64_t seed,
                               float *params, int32_t *ray_ids, int64_t *count, void *scratch,
                               size_t scratch_bytes);
gsf_status gsf_seed_volume(gsf_ctx *ctx, const uint16_t *vol, int32_t n, double threshold,
                           double range, const double *lo, const double *hi, double opacity,
                           int64_t cap, uint64_t seed, float *params, int64_t *count,
                           void *scratch, size_t scratch_bytes);

/* Emission-absorption ray march of the volume for n_views cameras (Method,
 * "Volumetric Path Tracing"; the fit's target images): float32, segments of
 * `step` world units from the entry into [-1, 1]^3 (the last shortened), the
 * trilinear sample (zero outside the grid) at each midpoint, density t as in
 * gsf_seed_volume, colour lo (1 - t) + hi t (host float[3]), alpha = 1 -
 * exp(-extinction t length), stopping once T < t_stop.  out: device RGBA per
 * view [4][H][W] (views concatenated) = C + T bg, 1 - T.  widths/heights
 * (host) must match the cameras.  Asynchronous on the context stream. */
gsf_status gsf_raymarch(gsf_ctx *ctx, const uint16_t *vol, int32_t n, const gsf_camera *cams,
                        int32_t n_views, const int32_t *widths, const int32_t *heights, float step,
                        float extinction, float t_stop, float threshold, float range,
                        const float *lo, const float *hi, float *out_rgba);

/* ---- diagnostics ---------------------------------------------------------------- */

/* Per-stage GPU timing of eager calls on a plan (hipEvents recorded around each
 * stage on the context stream; not available while capturing).  Enabling
 * resets the accumulators.  Stages holding exactly one kernel: PROJECT,
 * RENDER, RENDER_BWD, PROJECT_BWD. */
enum {
    GSF_STAGE_PROJECT = 0,     /* projection + support boxes (one kernel) */
    GSF_STAGE_DUPLICATE = 1,   /* record-order scan of the listed-tile counts (gradient slots,
                                  key total, the records with keys compacted) */
    GSF_STAGE_TILE_SORT = 2,   /* stable radix sort of the keys by tile */
    GSF_STAGE_RANGES = 3,      /* per-tile ranges from the key boundaries + compositing order */
    GSF_STAGE_DEPTH_SORT = 4,  /* stable radix sort of the records with keys by depth, then
                                  their keys emitted in that order */
    GSF_STAGE_RENDER = 5,      /* forward compositing (one kernel) */
    GSF_STAGE_LOSS = 6,        /* masked L1 loss */
    GSF_STAGE_RENDER_BWD = 7,  /* compositing adjoint (one kernel) */
    GSF_STAGE_PROJECT_BWD = 8, /* projection adjoint (one kernel) */
    GSF_STAGE_ADAM = 9,        /* step counter + Adam (inside gsf_step only) */
    GSF_STAGE_GRAD_SUM = 10,   /* per-record sum of the per-key screen-space gradients (one
                                  kernel; SH degrees 2-3 only: for 0-1 it runs inside
                                  PROJECT_BWD) */
    GSF_STAGE_COUNT = 11
};
gsf_status gsf_plan_set_timing(gsf_plan *plan, int enable);
/* Work accounting of the last gsf_forward (synchronises): out[0] = (pixel,
 * splat) pairs the forward compositing visits (up to and including the splat
 * that stops a pixel, else the whole tile list), out[1] = pairs included in
 * the image, out[2] = pairs the adjoint visits (up to each pixel's last
 * included splat), over the pixels that forward composited (after a
 * fovea-culled forward: those of the fovea disk; its gaze buffer must still
 * be valid).  Runs an extra counting kernel; not part of the fit step. */
gsf_status gsf_count_pairs(gsf_plan *plan, int64_t *out /* (host) [3] */);
/* Synchronise and return the accumulated milliseconds and call counts per
 * stage (host arrays of GSF_STAGE_COUNT entries; either may be NULL). */
gsf_status gsf_plan_stage_times(gsf_plan *plan, double *total_ms, int64_t *calls);

/* Synchronise the stream, return and clear the sticky flags (host *flags), and
 * report the key count of the last forward (host *m_keys, may be NULL). */
gsf_status gsf_poll(gsf_plan *plan, uint32_t *flags, int64_t *m_keys);

enum {
    GSF_DBG_RECT = 0,      /* uint32[2] per record (v*n + i): tile x0 | y0 << 16, x1 | y1 << 16 */
    GSF_DBG_COUNT = 1,     /* uint32 per record: tiles touched (0 = culled or empty) */
    GSF_DBG_DEPTH = 2,     /* float per record: camera-space depth */
    GSF_DBG_KEYS = 3,      /* uint32 per key: global tile id, sorted */
    GSF_DBG_VALS = 4,      /* uint32 per key: record id, in sorted key order */
    GSF_DBG_RANGES = 5,    /* uint32[2] per global tile: [start, end) */
    GSF_DBG_TFINAL = 6,    /* float per pixel (all views concatenated) */
    GSF_DBG_NCONTRIB = 7,  /* uint32 per pixel: list entries up to the last included */
    GSF_DBG_G2D = 8,       /* float [9][n_views * n]: per-record screen-space gradient of the
                              last gsf_backward (summed from its per-key terms on request) */
    GSF_DBG_PROJ = 9,      /* float [11] per record: mean x, mean y, conic A, B, C, opacity,
                              red, green, blue, camera depth, valid (1 or 0) */
    GSF_DBG_ORDER = 10,    /* uint32 per global tile: compositing order of the tiles (a
                              permutation; tiles with more keys first); after a
                              fovea-culled forward, the global ids of its launch
                              tiles (those of the fovea boxes), in that order */
    GSF_DBG_BG = 11,       /* float [n_views][3]: backgrounds drawn by the last random_bg step */
    GSF_DBG_VIS = 12       /* uint8 [n]: Gaussian visibility of the last masked_adam step */
};
/* Synchronise and copy an internal buffer of the last forward/backward to host
 * memory (at most cap bytes; bytes copied in *written). */
gsf_status gsf_debug_copy(gsf_plan *plan, int which, void *host_dst, size_t cap, size_t *written);

#ifdef __cplusplus
}
#endif
#endif /* GSFIT_H */
