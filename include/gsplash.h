/*
 * gsplash.h -- C ABI of the MI355X (gfx950) underwater Gaussian rasterizer.
 *
 * The library renders N anisotropic 3D Gaussians (Preliminaries, "3D Gaussian
 * Splatting": mean, covariance factored as rotation x scale, SH colour,
 * opacity) into one or more pinhole views with the underwater image formation
 * model of eq. (3dgs_uw) -- the alpha composite of eq. (3dgs_orig) attenuated
 * by exp(-B_d z) plus backscatter B_inf (1 - exp(-B_b z)), per RGB channel --
 * evaluated at the alpha-weighted depth z of eq. (Depth), and computes the
 * exact adjoint of that forward (appendix "Partial Derivatives", with the
 * factor z in dL/dB_d, dL/dB_b and the dependence of z on alpha included).
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers unless the parameter name starts
 *     with host_.  Floating point is FP32.  Gaussian parameters are
 *     structure-of-arrays planes: plane k of an [K][n] array starts at k * n.
 *   - The caller owns every buffer, including the workspace and the `saved`
 *     forward context; the library allocates and frees no device memory and
 *     keeps no global mutable state, apart from the fixed scratch array of
 *     gs_l1_dssim_loss_noalloc.
 *   - Every compute call only enqueues work on `stream` (a hipStream_t) and
 *     never synchronises the host, so a forward/backward sequence can be
 *     captured into a HIP graph.  Only gs_read_status and the queries that
 *     say so (key export, statistics, gs_phases_needed) synchronise.
 *   - Synchronous errors are returned as GS_ERR_*; nothing is enqueued when an
 *     error is returned.  Asynchronous conditions (pair-capacity overflow, a
 *     forward cut short by opts.phase_limit, non-finite inputs) are recorded
 *     in a status word inside `saved`.
 *   - Views are packed in order: view v's pixels start at pixel offset
 *     P_v = sum_{u<v} width_u * height_u.  Per-view images are planar CHW:
 *     out_rgb[3 * P_v + c * (W*H) + y * W + x]; depth and alpha are
 *     [P_v + y * W + x].
 */
#ifndef GSPLASH_H
#define GSPLASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_OK                        0
#define GS_ERR_INVALID_ARGUMENT     -1   /* null pointer, bad size or option value */
#define GS_ERR_UNSUPPORTED          -2   /* valid but not implemented (e.g. tile shape) */
#define GS_ERR_WORKSPACE_TOO_SMALL  -3   /* a caller buffer is smaller than gs_workspace_query says */
#define GS_ERR_HIP                  -4   /* a HIP runtime call failed */

#define GS_STATUS_PAIR_OVERFLOW      1u  /* more (Gaussian, tile) pairs than opts.max_pairs */
#define GS_STATUS_NONFINITE_INPUT    2u  /* a Gaussian had a non-finite parameter (it was culled) */
#define GS_STATUS_INCOMPLETE         4u  /* opts.phase_limit ended the forward while a tile still had a pixel
                                            above t_min and Gaussians were left unbinned */
/* A forward reporting either of these rendered a truncated image: the backward
 * entry points then produce no gradient and the Adam entry points skip the step. */
#define GS_STATUS_TRUNCATED (GS_STATUS_PAIR_OVERFLOW | GS_STATUS_INCOMPLETE)

#define GS_MAX_VIEWS                64
#define GS_MAX_PAIRS         2147483647LL /* pair indices are 31-bit */
#define GS_MAX_PHASES                8

typedef void* gs_stream_t;               /* hipStream_t; NULL = the default stream */

/* Pinhole camera (Preliminaries: "given the camera pose ... a pixel defines a
 * ray").  World -> camera: x_c = R x_w + t, R row-major.  The camera looks
 * down +z with image y pointing down; pixel (u, v) is sampled at its centre
 * (u + 1/2, v + 1/2); projection m = (fx x_c/z_c + cx, fy y_c/z_c + cy).
 * Gaussians whose camera-space depth is <= near_z are culled. */
typedef struct gs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float near_z;
} gs_camera;

/* Medium coefficients of eq. (3dgs_uw), one set per view, per RGB channel:
 * direct attenuation B_d, backscatter attenuation B_b, veiling light B_inf. */
typedef struct gs_medium {
    float Bd[3], Bb[3], Binf[3];
} gs_medium;

/* Gaussian parameters (Preliminaries, theta_i).  Activated values: scales > 0
 * (the covariance is R(q) diag(s)^2 R(q)^T), opacity in (0, 1) (the sigmoid of
 * eq. (opacity_impact) already applied, see gs_activate).  quats are (w,x,y,z),
 * any non-zero length (normalised inside).  sh holds (sh_degree+1)^2 * 3 planes,
 * plane index coef * 3 + channel; colour = max(0, 1/2 + sum_lm Y_lm(dir) k_lm)
 * with real orthonormal SH (Condon-Shortley phase) of the unit direction from
 * the camera centre to the mean. */
typedef struct gs_gaussians {
    int64_t n;
    int32_t sh_degree;                   /* 0..3 */
    int32_t reserved;
    const float* means;                  /* [3][n] */
    const float* scales;                 /* [3][n] */
    const float* quats;                  /* [4][n] */
    const float* opacity;                /* [n]    */
    const float* sh;                     /* [(sh_degree+1)^2 * 3][n] */
} gs_gaussians;

/* Gradients w.r.t. the gs_gaussians fields, same layouts.  OVERWRITTEN (not
 * accumulated) by gs_render_backward; every pointer must be non-NULL. */
typedef struct gs_gaussian_grads {
    float* means;
    float* scales;
    float* quats;
    float* opacity;
    float* sh;
} gs_gaussian_grads;

/* Rasterizer options.  gs_default_options fills the defaults noted here. */
/* gs_options.record_fetch */
#define GS_FETCH_DEFAULT 0
#define GS_FETCH_LDS 1
#define GS_FETCH_SCALAR 2

typedef struct gs_options {
    int32_t tile_w, tile_h;              /* 16x16 (default) or 8x8 pixels per tile */
    int32_t lds_batch;                   /* records staged in LDS per batch: 64 (default), 128 or 256 */
    int32_t persistent;                  /* 0: one workgroup per tile; 1: persistent workgroups pull tiles from a
                                            queue in tile order; 2: the same queue ordered longest list first
                                            (power-of-two buckets of each tile's list length, by a stable radix
                                            sort before each pass).  Images are identical for every value. */
    int32_t pixels_per_lane;             /* 16x16 tiles: pixels each lane blends, 1 (four waves per tile, 8x8
                                            each), 2 (two waves, 16x8 each) or 4 (one wave); 8x8 tiles: 1;
                                            0 = per-pass default (forward 2, backward 4).  Images are
                                            identical for every value. */
    int32_t record_fetch;                /* GS_FETCH_LDS: the workgroup stages batches of records in LDS;
                                            GS_FETCH_SCALAR: each wave loads records through the scalar cache
                                            (lds_batch is then unused); GS_FETCH_DEFAULT (0) = per-pass
                                            default (forward LDS, backward scalar) */
    float alpha_min;                     /* 1/255: a Gaussian with alpha < alpha_min is skipped at that pixel */
    float alpha_max;                     /* 0.99: alpha = min(alpha_max, o exp(-q/2)) */
    float t_min;                         /* 1e-4: stop before blending a Gaussian that would leave T < t_min */
    float dilation;                      /* 0.3: added to the diagonal of the 2D covariance (EWA low-pass) */
    float kappa;                         /* 11.1: tile rectangle = bounding box of q <= kappa (> 2 ln 255) */
    int32_t depth_mode;                  /* z the medium term uses: 0 = alpha-weighted depth zhat;
                                            1 = 2/(1+exp(-0.1 zhat)) - 1 (Implementation section) */
    int32_t tile_cull;                   /* 1 (default): drop a (Gaussian, tile) pair of the rectangle when no
                                            pixel centre of the tile can reach alpha >= alpha_min (a bound
                                            with a rounding margin; images are identical); 0: every tile of
                                            the rectangle, as in the method's binning */
    int32_t phases;                      /* depth-progressive binning: 1 = bin every (Gaussian, tile) pair at
                                            once; 2..8 = bin the depth-sorted Gaussians in that many rank
                                            ranges (e.g. nearest 1/128 | rest for 2 and shift 7) and, after
                                            each range, only for tiles that still have a pixel above t_min,
                                            walking only the alive columns of each tile row; 0 (default) =
                                            automatic: 2 for one view, 4 for several (gs_schedule).  Images
                                            are identical for every value. */
    int32_t phase0_shift;                /* the first range is the nearest 1/2^shift of the visible
                                            Gaussians, each later one (but the last) 4x wider: 1..20;
                                            0 (default) = automatic: for one view log2 of the Gaussians
                                            per tile, rounded and clamped to 2..12 (about one Gaussian
                                            per tile first); 6 for several.  Images are identical for
                                            every value. */
    int32_t depth_output;                /* depth image: 0 (default) = the z of depth_mode; 1 = the logistic
                                            map 2/(1+exp(-0.1 zhat)) - 1 of the Implementation section, for
                                            visualisation, whatever depth_mode the medium uses */
    int32_t phase_growth;                /* log2 of the growth of the depth phases' rank ranges: phase p
                                            (but the last) ends at the nearest 1/2^(shift - growth p) of
                                            the visible Gaussians: 1 (2x), 2 (4x), 3 (8x) or 4 (16x);
                                            0 (default) = 2.  Images are identical for every value. */
    int64_t max_pairs;                   /* capacity of the stored (Gaussian, tile) pair list, <= GS_MAX_PAIRS */
    void* timer;                         /* optional gs_timer* receiving per-kernel HIP events; NULL = none */
    /* Loss terms on the parameters that the backward entry points add to the
     * gradients they produce (0 / NULL = none; gs_default_options sets none): */
    const float* medium_prior;           /* DEVICE [n_views][6] (B_inf_hat[3], B_b_hat[3]) from
                                            gs_estimate_backscatter: the medium gradient gets
                                            prior_lambda sign(B - B_hat) on its B_inf and B_b entries
                                            (lambda_est L_best of eq. (OurFinalLoss)) */
    float prior_lambda;
    float reg_opacity;                   /* lambda_o: the loss gets lambda_o mean_i(opacity_i), so each
                                            Gaussian's opacity gradient gets lambda_o / n */
    float reg_scale;                     /* lambda_s: the loss gets lambda_s mean over the 3 n activated
                                            scale entries, so each gets lambda_s / (3 n) (the regularisers
                                            of the MCMC densification the paper adopts, Sec. Implementation) */
    int32_t phase_limit;                 /* 0 (default): run every depth phase of the schedule; 1..8: run only
                                            the first phase_limit of them.  If a tile still has a pixel above
                                            t_min after the last phase run while Gaussians are left unbinned,
                                            the forward reports GS_STATUS_INCOMPLETE (its image is then
                                            truncated); otherwise the image equals the full schedule's bit
                                            for bit, since the phases left out would blend nothing.  For a
                                            caller that replays a fixed scene: gs_phases_needed gives the
                                            limit a full forward of it needed. */
} gs_options;

/* Fill `opts` with the defaults above (phases and phase0_shift automatic, max_pairs = 1 << 24). */
void gs_default_options(gs_options* opts);

/* Library version string (static storage). */
const char* gs_version(void);

/* Device bytes that gs_render_forward/backward need for these options, scene
 * size and views (host_cams is a HOST array of n_views cameras).  `saved` is
 * the forward context that must be kept unchanged until gs_render_backward;
 * `workspace` is scratch for either call.  Touches no device; callable without
 * a GPU.  Returns GS_ERR_INVALID_ARGUMENT for bad options or sizes. */
int gs_workspace_query(const gs_options* opts, int64_t n, int32_t n_views, const gs_camera* host_cams,
                       size_t* workspace_bytes, size_t* saved_bytes);

/* Forward render (eq. 3dgs_orig, opacity_impact, 3dgs_uw, Depth) of all views.
 *   host_cams  : HOST copy of the cameras; fixes the image sizes (and so the
 *                launch shapes).
 *   dev_cams   : DEVICE copy of the same cameras; the kernels read poses and
 *                intrinsics from here (so a captured graph can be replayed
 *                after the poses are updated in place; sizes must not change).
 *   dev_medium : DEVICE [n_views] medium coefficients.
 *   out_rgb    : [sum 3 W H] attenuated colour C_uw (CHW per view);
 *   out_depth  : [sum W H] the depth image (opts.depth_output: the z of the
 *                medium term, or its logistic map for visualisation); 0 where no
 *                Gaussian contributes (such pixels are treated as at infinite
 *                range: C_uw = B_inf where B_b > 0);
 *   out_alpha  : [sum W H] accumulated opacity sum_i alpha_i T_i;
 *   out_restored : [sum 3 W H] or NULL: the clean image J of
 *                eq. (scattering_approx), i.e. the in-air composite
 *                C_air = sum_i c_i alpha_i T_i before the medium's attenuation
 *                and backscatter (0 where no Gaussian contributes), CHW per view.
 *   saved      : forward context (>= saved_bytes) used by gs_render_backward,
 *                gs_read_status and gs_export_keys.
 * Returns GS_OK or a GS_ERR_* code; capacity overflow and a forward cut short
 * by opts.phase_limit are reported asynchronously through gs_read_status
 * (GS_STATUS_TRUNCATED: the outputs are then not valid). */
int gs_render_forward(const gs_options* opts, const gs_gaussians* g, int32_t n_views,
                      const gs_camera* host_cams, const gs_camera* dev_cams, const gs_medium* dev_medium,
                      float* out_rgb, float* out_depth, float* out_alpha, float* out_restored,
                      void* saved, size_t saved_bytes, void* workspace, size_t workspace_bytes,
                      gs_stream_t stream);

/* Adjoint of gs_render_forward for L with upstream gradients grad_rgb (same
 * layout as out_rgb), grad_depth (same layout as out_depth, may be NULL) and
 * grad_restored (same layout as out_restored, may be NULL).
 * Transmittance is recomputed from the saved final transmittance rather than
 * storing per-pixel Gaussian lists.  Writes gradients w.r.t. every Gaussian
 * parameter (activated scales and opacity) into `grads` (overwritten) and
 * grad_medium [n_views][9] = (dB_d[3], dB_b[3], dB_inf[3]) (overwritten).
 * opts, g, n_views, cameras and medium must equal those of the forward call
 * that produced `saved`.  If that forward's image was truncated
 * (GS_STATUS_TRUNCATED: pair capacity overflow, or cut short by
 * opts.phase_limit), the adjoint kernels do nothing and every gradient
 * written is zero. */
int gs_render_backward(const gs_options* opts, const gs_gaussians* g, int32_t n_views,
                       const gs_camera* host_cams, const gs_camera* dev_cams, const gs_medium* dev_medium,
                       const float* grad_rgb, const float* grad_depth, const float* grad_restored,
                       const void* saved, size_t saved_bytes, gs_gaussian_grads* grads, float* grad_medium,
                       void* workspace, size_t workspace_bytes, gs_stream_t stream);

/* Synchronise `stream` and read the status word of a forward context:
 * status_bits = OR of GS_STATUS_*, pairs_needed = pair count the last forward
 * produced (compare with opts.max_pairs).  Either output may be NULL. */
int gs_read_status(const void* saved, uint32_t* status_bits, int64_t* pairs_needed, gs_stream_t stream);

/* Synchronise `stream` and report in *phases (HOST) how many leading depth
 * phases the forward that produced `saved` needed: the first phase after which
 * no tile had a pixel above t_min, or no Gaussian was left unbinned, or else
 * every phase of the schedule.  opts, n, n_views and host_cams must equal the
 * forward's.  When that forward was itself cut short (GS_STATUS_INCOMPLETE),
 * the value is one more than the phases it ran: a lower bound. */
int gs_phases_needed(const gs_options* opts, int64_t n, int32_t n_views, const gs_camera* host_cams,
                     const void* saved, size_t saved_bytes, int32_t* phases, gs_stream_t stream);

/* Write the (tile, depth) key list of the last forward into caller buffers:
 * keys[k] = (global tile id << 32) | FP32 bits of the view depth, values[k] =
 * view * n + Gaussian index (tiles numbered row-major within a view, views in
 * order).  The list is stored phase by phase: within phase p it is sorted by
 * key (ties in Gaussian index order), and tile_ranges[(p * tiles + t) * 2 ..]
 * = [start, end) of tile t in phase p (tile_ranges holds GS_MAX_PHASES *
 * gs_tile_count pairs of u32).  With opts.phases = 1 the whole list is one
 * sorted run of every pair.  Buffers hold `capacity` pairs; *pair_count (HOST)
 * receives the number stored.  Synchronises `stream`.
 * (Preliminaries, "Tiles"; depth order of eq. 3dgs_orig.) */
int gs_export_keys(const gs_options* opts, int64_t n, int32_t n_views, const gs_camera* host_cams,
                   const void* saved, size_t saved_bytes, uint64_t* keys, uint32_t* values,
                   uint32_t* tile_ranges, int64_t capacity, int64_t* pair_count, gs_stream_t stream);

/* Workload statistics of the last forward (synchronises `stream`):
 *   stats[0] = K, the number of (Gaussian, tile) pairs in the tile lists (all
 *              phases, culled pairs excluded);
 *   stats[1] = E, the number of tile-list entries the pixels evaluated in total
 *              (each pixel walks its tile's depth-ordered list up to and including
 *              the entry that terminated it);
 *   stats[2] = the number of list entries the compositing actually reached
 *              (per tile, the furthest point any of its pixels reached);
 *   stats[3] = the number of tiles with a non-empty list;
 *   stats[4] = the number of those evaluations that blended (alpha >= alpha_min).
 * `stats` is a HOST array of 5 entries.  Re-evaluates every walked entry: a
 * diagnostic, slower than the forward itself. */
int gs_forward_stats(const gs_options* opts, int64_t n, int32_t n_views, const gs_camera* host_cams,
                     const void* saved, size_t saved_bytes, int64_t* stats, gs_stream_t stream);

/* The depth-phase schedule these options give for n Gaussians and n_views views (host only):
 * the number of phases and the first phase's shift, with the automatic values (0) resolved.
 * `phases` and `phase0_shift` may be NULL.  Returns GS_OK or GS_ERR_INVALID_ARGUMENT as
 * gs_workspace_query would. */
int gs_schedule(const gs_options* opts, int64_t n, int32_t n_views, const gs_camera* host_cams, int32_t* phases,
                int32_t* phase0_shift);

/* Total number of tiles over the views for these options (host only). */
int64_t gs_tile_count(const gs_options* opts, int32_t n_views, const gs_camera* host_cams);

/* Parameter activation (eq. opacity_impact's sigmoid; exp scales):
 * scales[i] = exp(log_scales[i]) for i < 3n, opacity[i] = 1/(1+exp(-logits[i])). */
int gs_activate(int64_t n, const float* log_scales, const float* logits, float* scales, float* opacity,
                gs_stream_t stream);

/* Activation of one parameter group (the A0 step for a gs_adam_group):
 * y[i] = x[i] (activation 0), exp(x[i]) (1) or 1/(1+exp(-x[i])) (2), i < count. */
int gs_activation(int64_t count, int32_t activation, const float* x, float* y, gs_stream_t stream);

/* Chain gradients through gs_activate: g_log_scales = g_scales * scales,
 * g_logits = g_opacity * opacity * (1 - opacity) (scales/opacity activated). */
int gs_activate_backward(int64_t n, const float* scales, const float* opacity, const float* g_scales,
                         const float* g_opacity, float* g_log_scales, float* g_logits, gs_stream_t stream);

/* L1 term of eq. (3DGSoriginalLoss): loss[0] = mean |pred - target| over
 * `count` elements (loss may be NULL), grad[i] = sign(pred - target) / count
 * (grad may be NULL). */
int gs_l1_loss(int64_t count, const float* pred, const float* target, float* loss, float* grad,
               gs_stream_t stream);

/* Image loss of eq. (3DGSoriginalLoss) / (OurFinalLoss) for packed views (the
 * layout of out_rgb; host_cams fixes the view sizes):
 *     L = sum_v [ (1 - lambda) L1_v + lambda (1 - SSIM_v) ],
 * L1_v = mean |pred - target| over the view's 3 W H values, SSIM_v = mean of the
 * SSIM map over them (Wang et al., cited for D-SSIM; per colour channel, an
 * 11 x 11 Gaussian window of standard deviation 1.5, zero padding outside the
 * image, C1 = 0.01^2, C2 = 0.03^2 for values in [0, 1]).  The paper sets
 * lambda = 0.3 (appendix "Experimental Setup").
 *   loss : DEVICE [n_views + 1] or NULL: each view's L_v, then L.
 *   grad : DEVICE, layout of pred, or NULL: dL/dpred (overwritten).
 *   workspace : DEVICE scratch of gs_loss_workspace_query bytes (per-tile
 *              partial sums; the loss is their fixed-order sum, deterministic).
 * One pass reads pred and target and writes grad; no intermediate map reaches
 * memory.  Returns GS_ERR_INVALID_ARGUMENT (bad sizes, lambda outside [0, 1],
 * both outputs NULL) or GS_ERR_WORKSPACE_TOO_SMALL before any device work. */
int gs_loss_workspace_query(int32_t n_views, const gs_camera* host_cams, size_t* workspace_bytes);
int gs_l1_dssim_loss(int32_t n_views, const gs_camera* host_cams, const float* pred, const float* target,
                     float lambda, float* loss, float* grad, void* workspace, size_t workspace_bytes,
                     gs_stream_t stream);

/* gs_l1_dssim_loss without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, outputs and kernels; the
 * per-tile partial sums go to a library-owned device array of 8 MiB (2^20
 * workgroups: up to 64 views of 1920 x 1080), of which each GPU the library
 * runs on holds its own copy until the process ends.  The array's address is
 * looked up once per device, on the first call with that device current;
 * `stream` must belong to the current device.  Calls no allocating routine.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (two streams, or two host threads) race and may return wrong losses; the
 * gradient does not use the array.  Returns GS_ERR_WORKSPACE_TOO_SMALL (nothing
 * enqueued) when the views need more than 2^20 workgroups (32 x 16 pixels of
 * one channel each), GS_ERR_HIP if the array's address cannot be found, and
 * otherwise what gs_l1_dssim_loss returns. */
int gs_l1_dssim_loss_noalloc(int32_t n_views, const gs_camera* host_cams, const float* pred, const float* target,
                             float lambda, float* loss, float* grad, gs_stream_t stream);

/* Backscatter estimation (Sec. Optimization; appendix "Backscatter Estimation",
 * Alg. 1 and Alg. 2): per view, rough estimates of the veiling light B_inf and
 * the backscatter attenuation B_b from an observed image and the rendered
 * depth z of eq. (Depth), which the L_best term of eq. (OurFinalLoss) then pulls
 * the learned medium towards (re-estimated every 500 iterations in the paper).
 * Steps per view:
 *   1. image and depth resized bilinearly to resize_height rows (width
 *      floor(W rows / H + 1/2); 0 or H = no resize; half-pixel centres, edges
 *      clamped), negative values set to 0;
 *   2. the pixels with a depth (z > 0) cut into edges - 1 evenly spaced depth
 *      clusters between their smallest and largest depth; in a cluster of n
 *      pixels the ceil(p_dark n) pixels of smallest r^2 + g^2 + b^2 (ties: lower
 *      pixel index) are its dark pixels;
 *   3. the dark pixels' depth range cut into intervals - 1 evenly spaced
 *      intervals ([e_i, e_{i+1}), the last closed); per channel and interval the
 *      smallest dark value (ties: lower pixel index) and its depth form a point;
 *   4. per channel, the bounded least-squares fit of B_inf (1 - exp(-B_b z)) to
 *      the points, B_inf in [0, 1], B_b in [0, 5] (0, 0 without points).
 * Every decision of steps 1-3 is taken in FP32 with a fixed operation order
 * (stated in the source); the fit is FP64. */
typedef struct gs_backscatter_options {
    float p_dark;                        /* 0.01: share of each cluster kept as dark pixels, in (0, 1] */
    int32_t edges;                       /* 10: cluster edges (edges - 1 clusters), 2..33 */
    int32_t intervals;                   /* 25: interval edges of Alg. 1 (intervals - 1 intervals), 2..257 */
    int32_t resize_height;               /* 300: rows after the resize; 0 = full resolution */
} gs_backscatter_options;

void gs_default_backscatter_options(gs_backscatter_options* opts);
/* Host-only: bytes of the workspace gs_estimate_backscatter needs for these views. */
int gs_backscatter_workspace_query(const gs_backscatter_options* opts, int32_t n_views, const gs_camera* host_cams,
                                   size_t* workspace_bytes);
/*   image  : DEVICE, packed like out_rgb (the observed images, CHW per view).
 *   depth  : DEVICE, packed like out_depth (rendered depth, 0 = no depth).
 *   est    : DEVICE [n_views][6] out: B_inf_hat[3], B_b_hat[3] per view.
 *   points : DEVICE [n_views][3][intervals - 1][2] or NULL: (depth, value) of
 *            each interval's point, NaN for an interval without dark pixels.
 *   cost   : DEVICE [n_views][3] or NULL: the fit's residual sum of squares.
 *   workspace : DEVICE scratch of gs_backscatter_workspace_query bytes.
 * Only the camera sizes of host_cams are used.  Images must be finite.
 * Returns GS_ERR_INVALID_ARGUMENT / GS_ERR_WORKSPACE_TOO_SMALL before any
 * device work. */
int gs_estimate_backscatter(const gs_backscatter_options* opts, int32_t n_views, const gs_camera* host_cams,
                            const float* image, const float* depth, float* est, float* points, float* cost,
                            void* workspace, size_t workspace_bytes, gs_stream_t stream);
/* L_best of eq. (OurFinalLoss) times lambda (lambda_est of the paper):
 *   loss = lambda sum_v (|B_inf - B_inf_hat|_1 + |B_b - B_b_hat|_1)
 * medium : DEVICE [n_views][9] (B_d, B_b, B_inf per view, as gs_medium);
 * est    : DEVICE [n_views][6] from gs_estimate_backscatter;
 * loss   : DEVICE [1] or NULL;
 * grad_medium : DEVICE [n_views][9] or NULL: lambda sign(B - B_hat) is ADDED
 *               to the B_b and B_inf entries (B_d untouched). */
int gs_backscatter_prior(int32_t n_views, const float* medium, const float* est, float lambda, float* loss,
                         float* grad_medium, gs_stream_t stream);

/* MCMC densification (Sec. Implementation: the paper replaces the densification
 * of 3DGS with the MCMC approach of the work it cites; appendix "Experimental
 * Setup": every 100 iterations, minimum opacity 0.1).  The cited rules are not
 * in the paper; this library reads them as:
 *   - relocation: every dead Gaussian (opacity <= dead_opacity), in index order,
 *     takes a copy of a live Gaussian drawn with probability proportional to
 *     opacity;
 *   - addition: gs_mcmc_add_count(n, capacity, 1.05) copies of Gaussians drawn
 *     proportionally to opacity over all n are appended;
 *   - a Gaussian drawn c times becomes N = c + 1 identical Gaussians with
 *     opacity o' = 1 - (1 - o)^(1/N) (N stacked copies keep o on a ray) and
 *     scales s o / S(N, o'), S(N, a) = sum_{m=1..N} sum_{k<m} C(m-1, k) (-1)^k
 *     a^(k+1) / sqrt(k+1) (keeps the integral of the stacked opacity profile);
 *     N is capped at 51 and o' kept in [0.005, 1 - 2^-23]; computed in FP64;
 *   - the Adam moments of every rewritten Gaussian restart at 0;
 *   - between densifications the means take Langevin noise (gs_mcmc_noise);
 *   - the opacity and scale regularisers are gs_options.reg_opacity / reg_scale.
 * Random numbers are inputs.  Draw j uses the u32 draws[j]: with integer
 * weights w_i = floor(o_i 2^24) (0 for dead Gaussians in relocation), P their
 * sum and P_i their exclusive prefix sums, it picks the i with
 * P_i <= floor(draws[j] P / 2^32) < P_i + w_i (exact integer arithmetic). */
typedef struct gs_mcmc_state {
    int64_t n;                           /* Gaussians; every plane is [K][n] */
    int32_t sh_degree;                   /* 0..3 */
    int32_t reserved;
    float* param[5];                     /* raw parameters: means [3], log-scales [3], quaternions [4],
                                            opacity logits [1], SH [(sh_degree+1)^2 * 3] planes */
    float* m[5];                         /* first Adam moments, same layouts */
    float* v[5];                         /* second Adam moments, same layouts */
    float* scales;                       /* activated scales [3][n] (exp of the log-scales) */
    float* opacity;                      /* activated opacity [n] (sigmoid of the logits) */
} gs_mcmc_state;

/* max(0, min(capacity, floor(growth n)) - n): the Gaussians one addition appends. */
int64_t gs_mcmc_add_count(int64_t n, int64_t capacity, double growth);
/* Host-only: workspace bytes for a state of n Gaussians and n_draws draws
 * (relocation: n_draws = n; addition: the appended count). */
int gs_mcmc_workspace_query(int64_t n, int64_t n_draws, size_t* workspace_bytes);
/* Relocation, in place.  draws: DEVICE u32 [n] (the j-th dead Gaussian uses
 * draws[j]); sources: DEVICE u32 [n] or NULL, receives each dead Gaussian's
 * source; taken: DEVICE u32 [1] or NULL, receives the number of relocated
 * Gaussians (0 when no Gaussian is live).  dead_opacity in [0, 1). */
int gs_mcmc_relocate(gs_mcmc_state* state, float dead_opacity, const uint32_t* draws, uint32_t* sources,
                     uint32_t* taken, void* workspace, size_t workspace_bytes, gs_stream_t stream);
/* Addition, out of place: dst (dst->n = src->n + k, same sh_degree, buffers
 * disjoint from src's) receives src's Gaussians with the drawn ones split and
 * the k copies appended at n .. n + k - 1 (copy j of the source of draws[j]).
 * sources, taken as in gs_mcmc_relocate; when no Gaussian of src has a
 * non-zero weight, *taken = 0 and dst's appended entries are unspecified (keep
 * src). */
int gs_mcmc_add(const gs_mcmc_state* src, gs_mcmc_state* dst, const uint32_t* draws, uint32_t* sources,
                uint32_t* taken, void* workspace, size_t workspace_bytes, gs_stream_t stream);
/* Langevin noise on the means (in place), for each Gaussian:
 *   mu += lr_means noise_lr sigmoid(100 ((1 - o) - 0.995)) R diag(s^2) R^T eta
 * with R the rotation of the normalised quaternion, s the activated scales, o
 * the activated opacity, eta DEVICE [3][n] standard normal draws (an input);
 * noise_lr = 5e5 in this library's reading.  FP32. */
int gs_mcmc_noise(int64_t n, float* means, const float* quats, const float* scales, const float* opacity,
                  const float* eta, float lr_means, float noise_lr, gs_stream_t stream);

/* One parameter group of the fused Adam step (Sec. Optimization: Adam with
 * the 3DGS learning rates, medium at the colour learning rate). */
typedef struct gs_adam_group {
    float* param;                        /* raw parameter, updated in place */
    const float* grad;                   /* gradient (see activation) */
    float* m;                            /* first moment, updated */
    float* v;                            /* second moment, updated */
    float* activated;                    /* activation != 0: receives act(param) after the update */
    int64_t count;
    float lr;
    int32_t activation;                  /* 0 none; 1 exp; 2 sigmoid.  With an activation, `grad` is the
                                            gradient w.r.t. the ACTIVATED value and `activated` must hold the
                                            activated value of the current param on entry. */
    int32_t reserved;
} gs_adam_group;

/* Device-side training state of the Adam entry points: int32[2], zeroed by the
 * caller before the first step.
 *   state[0] : the Adam step counter t (incremented by each step that runs).
 *   state[1] : sticky skip flag.  A step whose forward context reports a
 *              GS_STATUS_TRUNCATED bit (its render was truncated) is not
 *              applied: the counter, parameters, moments and activated copies
 *              stay unchanged and that bit is OR-ed into state[1].  While
 *              state[1] != 0 every later step is skipped too, so a replayed
 *              graph cannot apply a bad step after a truncated render; only
 *              the caller clears it (after growing the capacity, or lifting
 *              opts.phase_limit). */
#define GS_STATE_STEP 0
#define GS_STATE_SKIP 1

/* Training-step adjoint with the optimizer fused into the projection adjoint
 * (Sec. Optimization): the adjoint of gs_render_backward, but instead of writing
 * the parameter gradients it applies one Adam step -- as gs_adam_step_device,
 * same step counter semantics -- to the raw parameters in registers, so the
 * gradients of the Gaussians never reach memory.  The SH gradient of a
 * Gaussian is, per view, the outer product of the SH basis at its view
 * direction and its colour gradient: the projection adjoint steps the other
 * groups and keeps those factors in the workspace (one view: direction and
 * colour gradient; several views: each view's colour gradient), and a second
 * kernel steps the SH coefficients and the means from them (with several views
 * gs_render_backward runs the same kernel to write those gradients).  For the
 * same 2D gradients -- the compositing adjoint's atomic sums may differ in order
 * from call to call -- results equal gs_render_backward followed by
 * gs_adam_step_device bit for bit.
 *   groups[6] : HOST array, in this order: means (count 3n, activation 0),
 *               log-scales (3n, activation 1, activated = the scales g->scales
 *               points to), quaternions (4n, 0), opacity logits (n, activation 2,
 *               activated = g->opacity), SH ((deg+1)^2 * 3 * n, 0), medium
 *               (9 * n_views, 0, param = dev_medium).  g->means, g->quats, g->sh
 *               must be the groups' params.  Each group's `grad`
 *               is ignored except the medium group's, which receives the medium
 *               gradient [n_views][9].
 *   state      : DEVICE int32[2] training state (see GS_STATE_*): the step
 *                counter is incremented first and the incremented value is t;
 *                a forward whose image was truncated (GS_STATUS_TRUNCATED)
 *                skips the step.
 * Only the m, v, param and activated arrays are written (plus workspace, state
 * and the medium group's grad).
 * Returns GS_ERR_INVALID_ARGUMENT on any mismatch; otherwise as gs_render_backward. */
int gs_render_backward_adam(const gs_options* opts, const gs_gaussians* g, int32_t n_views,
                            const gs_camera* host_cams, const gs_camera* dev_cams, const gs_medium* dev_medium,
                            const float* grad_rgb, const float* grad_depth, const float* grad_restored,
                            const void* saved, size_t saved_bytes, const gs_adam_group* groups, float beta1,
                            float beta2, float eps, int32_t* state, void* workspace, size_t workspace_bytes,
                            gs_stream_t stream);

/* Fused Adam update (beta1, beta2, eps, bias correction at `step` >= 1) over
 * up to 8 groups in one launch. */
int gs_adam_step(const gs_adam_group* host_groups, int32_t n_groups, float beta1, float beta2, float eps,
                 int32_t step, gs_stream_t stream);

/* As gs_adam_step, for replay from a captured graph: the step number lives in
 * device memory.  state (DEVICE int32[2], see GS_STATE_*): state[0] is
 * incremented first and the incremented value is the step used for bias
 * correction (start it at 0).  saved (nullable) is the forward context the
 * gradients came from: when it reports a GS_STATUS_TRUNCATED bit, or state[1]
 * is already set, the step is skipped and the flag is kept in state[1]. */
int gs_adam_step_device(const gs_adam_group* host_groups, int32_t n_groups, float beta1, float beta2, float eps,
                        int32_t* state, const void* saved, gs_stream_t stream);

/* HIP graph capture of any sequence of the enqueue-only calls above (for
 * callers that replay a fixed pipeline, e.g. a training step over fixed views).
 * gs_graph_begin starts capturing `stream` (which must not be the default
 * stream); gs_graph_end stops it and instantiates the graph into *graph;
 * gs_graph_launch replays it on `stream`; gs_graph_destroy frees it.  Buffers
 * referenced by the captured calls must stay allocated while the graph lives. */
int gs_graph_begin(gs_stream_t stream);
int gs_graph_end(gs_stream_t stream, void** graph);
int gs_graph_launch(void* graph, gs_stream_t stream);
int gs_graph_destroy(void* graph);

/* Optional per-kernel timing with HIP events (used by benchmarks).  A timer
 * records a start/stop event pair around each kernel it sees in opts.timer.
 * gs_timer_read synchronises the recorded events and returns, for the kernel
 * named `kernel`, the summed duration (ms) and the number of launches. */
void* gs_timer_create(int32_t capacity);
void gs_timer_destroy(void* timer);
void gs_timer_reset(void* timer);
int gs_timer_read(void* timer, const char* kernel, double* total_ms, int32_t* launches);

/* Enqueues one empty kernel named k_marker (one thread; `id` is its only
 * argument), so that a profiler's kernel trace can tell apart the phases of a
 * run (set-up, warm-up, timed steps) by the markers between them. */
int gs_profile_marker(int32_t id, gs_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GSPLASH_H */
