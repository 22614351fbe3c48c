/*
 * gs4d -- differentiable 4D Gaussian-splatting rasterizer for MI355X (gfx950).
 *
 * C ABI of libgs4d.so.  The method is Instant4D (arXiv 2510.01119): a native
 * 4D Gaussian is sliced at render time t into a conditional 3D Gaussian
 * (Sec. 3.3, Eq. "4dgs"), weighted by the temporal opacity o_t = o N(t; mu_4,
 * Sigma_44) and culled when o_t is negligible (Sec. 3.3, "Motion-Aware
 * Gaussian"), then rendered with the Gaussian-splatting rasterizer the paper
 * inherits from 3D/4D Gaussian splatting (Sec. 3.1): EWA projection, 16x16
 * tile binning, depth sort, front-to-back alpha compositing, and the analytic
 * backward.  Point clouds are reduced by voxel grid pruning (Sec. 3.2).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller, unless marked
 *     "host".  No entry point allocates or frees device memory: scratch
 *     memory is a caller-provided workspace of the size reported by the
 *     matching *_workspace_size() query.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream) and never synchronises the host.
 *   - Arguments are validated on the host before any launch; a rejected call
 *     launches nothing and returns GS4D_ERR_INVALID_ARG.  A failed launch
 *     returns GS4D_ERR_HIP.  gs4d_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Data-dependent overflow (pair capacity, prune capacity) is detected on
 *     the device: the kernels never write past a capacity; they raise a
 *     device status flag and store the size that was needed.
 *   - Parameters are SoA planes: params is float [20][n]
 *        0..3  mean (x, y, z, t)            4..7  log scale (x, y, z, t)
 *        8..11 left quaternion (w, x, y, z)  12..15 right quaternion (w,x,y,z)
 *        16    opacity logit                 17..19 rgb
 *     The 4D rotation maps p = t + x i + y j + z k to q_l p q_r with the
 *     normalised quaternions; Sigma = (R S)(R S)^T with S = diag(exp(log scale)).
 *   - Non-finite parameters, degenerate quaternions, Gaussians behind the
 *     near plane, temporally culled ones (255 o_t < 1) and ones whose exact
 *     alpha >= 1/255 footprint misses the image are culled (zero tiles).
 */
#ifndef GS4D_H
#define GS4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS4D_OK = 0,
    GS4D_ERR_INVALID_ARG = -1,
    GS4D_ERR_CAPACITY = -2,
    GS4D_ERR_HIP = -3,
    GS4D_ERR_UNSUPPORTED = -4
} gs4d_status;

#define GS4D_N_FIELDS 20     /* floats per Gaussian in params / dparams     */
#define GS4D_ISO_FIELDS 13   /* floats per Gaussian, isotropic motion-aware form */
#define GS4D_REC_FLOATS 12   /* floats per (view, Gaussian) projected record */
#define GS4D_GRAD2D_FLOATS 9 /* floats per (view, Gaussian) 2D gradient      */
#define GS4D_TILE 16         /* tile edge in pixels                          */
#define GS4D_MAX_VIEWS 16    /* views per call                               */

/* One camera at one timestamp (host struct, 96 bytes).  All views passed to
 * one call must share width and height. */
typedef struct gs4d_view {
    float Rt[12];       /* world -> camera [R | t], row-major 3x4; camera axes x right, y down, z forward */
    float fx, fy, cx, cy;
    int32_t width, height;
    float t;            /* render timestamp                                  */
    float near_z;       /* near plane (Gaussians with camera z < near_z are culled) */
    float bg[3];        /* background rgb                                    */
    int32_t reserved;   /* must be 0                                         */
} gs4d_view;

/* ---------------------------------------------------------------------------
 * gs4d_preprocess -- slice, cull, project and bin every (view, Gaussian).
 *   Sec. 3.3 Eq. "4dgs" (conditional mean/covariance at t), Sec. 3.3
 *   "Motion-Aware Gaussian" (o_t and its cull), Sec. 3.1 (EWA splatting).
 *   params   float [20][n]
 *   views    host, n_views entries (1 <= n_views <= GS4D_MAX_VIEWS)
 *   rec      out float [n_views][n][12]:
 *              0 mean2D.x 1 mean2D.y 2 conic.a 3 conic.b 4 conic.c 5 o_t
 *              6 camera depth z 7 footprint half-width x 8..10 rgb
 *              11 footprint half-width y   (all zeros if culled); outside
 *              the box mean2D +- half-widths every pixel has alpha < 1/255
 *   rect     out int32 [n_views][n][4]: tile rectangle [x0, y0, x1, y1) of
 *              the exact alpha >= 1/255 footprint (zeros if culled)
 *   touched  out int32 [n_views][n]: tiles covered, (x1-x0)*(y1-y0)
 *   Everything that decides an integer here is computed in FP32 with a fixed
 *   operation order, so results are reproducible bit for bit.
 * ------------------------------------------------------------------------- */
int gs4d_preprocess(const float *params, int64_t n, const gs4d_view *views, int32_t n_views,
                    float *rec, int32_t *rect, int32_t *touched, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_preprocess_iso -- gs4d_preprocess for the paper's isotropic,
 *   motion-aware parameterisation (Sec. 3.3 "Motion-Aware Gaussian" and the
 *   isotropic variant: one spatial scale, a temporal scale and a velocity).
 *   params   float [13][n]: 0-2 mean xyz, 3 mean t, 4 log s, 5 log s_t,
 *            6-8 velocity v (d mean / d t), 9 opacity logit, 10-12 rgb.
 *   The 4D covariance [[s^2 I + s_t^2 v v^T, s_t^2 v], [s_t^2 v^T, s_t^2]]
 *   sliced at the view's t gives mean + v (t - mean_t), covariance s^2 I
 *   and o_t = o exp(-(t - mean_t)^2 / (2 s_t^2)); projection, culls,
 *   record layout, rect and touched are those of gs4d_preprocess, so
 *   gs4d_bin_sort and the renderers take the output unchanged.
 * gs4d_preprocess_iso_bwd -- its chain rule from grad2d [n_views][n][9]
 *   to dparams [13][n] (overwritten, summed over views).
 * ------------------------------------------------------------------------- */
int gs4d_preprocess_iso(const float *params, int64_t n, const gs4d_view *views, int32_t n_views,
                        float *rec, int32_t *rect, int32_t *touched, void *stream);
int gs4d_preprocess_iso_bwd(const float *params, int64_t n, const gs4d_view *views,
                            int32_t n_views, const int32_t *touched, const float *grad2d,
                            float *dparams, void *stream);

/* ---------------------------------------------------------------------------
 * Sphericylindrical-harmonic (SCH) appearance: the view- and time-dependent
 * colour of 4D Gaussian splatting that the paper replaces by one RGB value
 * per Gaussian and ablates (Sec. 3.1, SCH equation; Sec. 4.4, the "w/o RGB"
 * ablation).  Basis Z_{nl}^m(t, d) = cos(2 pi n t / T) Y_l^m(d), n = 0..N,
 * l = 0..L, Y_l^m the real spherical harmonics (orthonormal on the sphere,
 * no Condon-Shortley phase: Y_{1,1} = sqrt(3/4pi) x, Y_{1,-1} = sqrt(3/4pi) y),
 * d the unit direction from the camera centre -R^T t to the Gaussian's
 * conditional mean at the view's t.  Basis index b = n (L+1)^2 + l^2 + l + m;
 * coefficients coef float [3 K][n], K = (N+1)(L+1)^2, row 3 b + channel;
 * colour_c = sum_b coef[3 b + c] Z_b (no offset, no clamp).
 *   gs4d_sch_rows(L, N)  rows of coef, 3 K (-1 if L or N is out of range)
 *   gs4d_preprocess_sch  gs4d_preprocess of rotor-form params [20][n] whose
 *       rows 17-19 are ignored: record slots 8-10 hold the SCH colour;
 *       a (view, Gaussian) whose colour is not finite is culled.
 *   gs4d_preprocess_sch_bwd  chain rule from grad2d [n_views][n][9]: dparams
 *       [20][n] (rows 17-19 zero; the colour's dependence on the direction
 *       joins the conditional mean's gradient) and dcoef [3 K][n], both
 *       overwritten, summed over views.
 *   gs4d_sch_from_rgb  coef with colour rgb [3][rgb_stride] (only the
 *       n = 0, l = 0 row set: rgb / Y_00).
 * ------------------------------------------------------------------------- */
#define GS4D_SCH_MAX_DEGREE 3
#define GS4D_SCH_MAX_FREQ 2
typedef struct gs4d_sch {
    int32_t degree;     /* L, 0..GS4D_SCH_MAX_DEGREE                      */
    int32_t n_freq;     /* N, 0..GS4D_SCH_MAX_FREQ                        */
    float period;       /* T > 0, in the views' time units                */
    int32_t reserved;   /* must be 0                                      */
} gs4d_sch;
int64_t gs4d_sch_rows(int32_t degree, int32_t n_freq);
int gs4d_preprocess_sch(const float *params, const float *coef, int64_t n, const gs4d_sch *sch,
                        const gs4d_view *views, int32_t n_views, float *rec, int32_t *rect,
                        int32_t *touched, void *stream);
int gs4d_preprocess_sch_bwd(const float *params, const float *coef, int64_t n,
                            const gs4d_sch *sch, const gs4d_view *views, int32_t n_views,
                            const int32_t *touched, const float *grad2d, float *dparams,
                            float *dcoef, void *stream);
int gs4d_sch_from_rgb(const float *rgb, int64_t rgb_stride, int64_t n, const gs4d_sch *sch,
                      float *coef, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_bin_sort -- duplicate each visible (view, Gaussian) once per touched
 *   tile and sort the pairs by (tile, depth) (Sec. 3.1, the tile-based
 *   splatting renderer).
 *   key = (global tile << 32) | bits(FP32 depth), value = Gaussian index;
 *   global tile = view * tiles_per_view + ty * tiles_x + tx.  Output is
 *   ascending by (key, value): a total order, hence unique.
 *   keys, vals     out, pair_capacity entries
 *   ranges         out int32 [n_views * tiles_per_view][2]: [start, end) per
 *                  tile in the sorted arrays, (0, 0) for an empty tile
 *   n_pairs        out device int64: number of pairs (also when over capacity)
 *   overflow       out device int32: 1 if n_pairs > pair_capacity (then keys,
 *                  vals and ranges are not valid), else 0
 *   ws, ws_bytes   workspace, >= gs4d_bin_sort_workspace_size(n, n_views, pair_capacity)
 *   pair_capacity must be < 2^31.
 * ------------------------------------------------------------------------- */
size_t gs4d_bin_sort_workspace_size(int64_t n, int32_t n_views, int64_t pair_capacity);
int gs4d_bin_sort(const float *rec, const int32_t *rect, const int32_t *touched, int64_t n,
                  const gs4d_view *views, int32_t n_views, int64_t pair_capacity, uint64_t *keys,
                  uint32_t *vals, int32_t *ranges, int64_t *n_pairs, int32_t *overflow, void *ws,
                  size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_bin_sort_noalloc -- gs4d_bin_sort for callers that cannot allocate
 *   (code under HIP graph capture, serving loops, harnesses that forbid
 *   hipMalloc): the same arguments without the workspace, the same output
 *   bit for bit.  Its scratch memory is a device array of the library of
 *   GS4D_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, so the
 *   call allocates nothing.  A call whose gs4d_bin_sort_workspace_size(n,
 *   n_views, pair_capacity) exceeds that returns GS4D_ERR_INVALID_ARG without
 *   launching anything.  The scratch is per device (the current one, which
 *   must own `stream`): calls that overlap on one GPU race and must be
 *   ordered by the caller (one stream, or events).
 * ------------------------------------------------------------------------- */
#define GS4D_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gs4d_bin_sort_noalloc(const float *rec, const int32_t *rect, const int32_t *touched, int64_t n,
                          const gs4d_view *views, int32_t n_views, int64_t pair_capacity,
                          uint64_t *keys, uint32_t *vals, int32_t *ranges, int64_t *n_pairs,
                          int32_t *overflow, void *stream);

/* Binning strategy of gs4d_bin_sort (process-wide; the output is the same):
 *   GS4D_BIN_PER_TILE  emit pairs in item order, sort on the tile bits, then
 *                      one workgroup per tile sorts its pairs by depth in LDS
 *                      (fewest launches; suits tiles of up to a few thousand
 *                      pairs)
 *   GS4D_BIN_PRESORT   sort the items by depth on the device first, emit in
 *                      that order, then sort on the tile bits (suits tiles of
 *                      tens of thousands of pairs)
 *   GS4D_BIN_COUNT     count the pairs per (tile, block of Gaussians), scan
 *                      the counts, write every pair straight into its tile,
 *                      then the per-tile depth sort (four launches; for up
 *                      to 8192 tiles per view, else as GS4D_BIN_PER_TILE)
 *   GS4D_BIN_AUTO      while pair_capacity <= 4096 * tiles: counting where
 *                      it applies, else per tile; above that presort (the
 *                      default) */
#define GS4D_BIN_AUTO 0
#define GS4D_BIN_PER_TILE 1
#define GS4D_BIN_PRESORT 2
#define GS4D_BIN_COUNT 3
int gs4d_set_bin_strategy(int32_t strategy);

/* Render options.  Zero-initialise and set what is needed. */
#define GS4D_RENDER_GRAD2D_ZEROED 1
typedef struct gs4d_render_opts {
    int32_t batch;          /* Gaussians staged in LDS per round: 64, 128 or 256 (0 -> 256) */
    int32_t persistent;     /* 0: one workgroup per (view, tile); 1: persistent workgroups
                               taking work-list positions from `queue`; 2: persistent with a
                               static assignment (workgroup i takes positions i and
                               2G-1-i of every 2G, G workgroups), no queue            */
    int32_t n_workgroups;   /* persistent launch size (0 -> 4 per CU)                       */
    int32_t flags;          /* GS4D_RENDER_GRAD2D_ZEROED: gs4d_render_bwd_2d's grad2d is
                               already zero (the call then launches the backward kernel
                               only, no clearing fill); other bits must be 0            */
    const float *target;    /* optional [n_views][3][H][W]: fused per-view L1 loss          */
    float l1_weight;        /* weight of the fused L1 term                                  */
    float *loss_per_view;   /* out [n_views], accumulated (caller zeroes), needs target     */
    float *dL_dimage;       /* out [n_views][3][H][W] dL1/dimage * l1_weight, needs target  */
    uint64_t *counters;     /* optional out [3], accumulated: evaluated (pixel, entry)
                               pairs, blends, and evaluated pairs up to each pixel's last
                               blend (the entries its backward re-evaluates)          */
    const int32_t *order;   /* optional [n_views*tiles_per_view] tile processing order (persistent) */
    int32_t *queue;         /* device int32 work counter for persistent mode 1 (caller zeroes) */
} gs4d_render_opts;

/* ---------------------------------------------------------------------------
 * gs4d_render_fwd -- front-to-back alpha compositing per pixel (Sec. 3.1):
 *   power = min(0, -1/2 (a dx^2 + c dy^2) - b dx dy), alpha =
 *   min(0.99, o_t e^power) (skip if < 1/255), T' = T (1 - alpha) (stop
 *   before blending if T' < 1e-4), C += rgb alpha T; output C + T bg.
 *   Pixel centres at (x + 1/2, y + 1/2).  The conic is positive definite,
 *   so the exponent is <= 0 in exact arithmetic: the min with 0 absorbs
 *   rounding only (the backward differentiates the exponent itself).
 *   image    out float [n_views][3][H][W]
 *   T_final  out float [n_views][H][W]
 *   last     out int32 [n_views][H][W]: global pair index of the last blended
 *            entry, -1 if none
 *            T_final and last may both be NULL: forward-only rendering, which
 *            keeps no state for gs4d_render_bwd (the image is the same)
 *   opts     host, may be NULL
 * ------------------------------------------------------------------------- */
int gs4d_render_fwd(const float *rec, int64_t n, const uint32_t *vals, const int32_t *ranges,
                    const gs4d_view *views, int32_t n_views, const gs4d_render_opts *opts,
                    float *image, float *T_final, int32_t *last, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_render_bwd -- analytic backward of gs4d_render_fwd and
 *   gs4d_preprocess down to the 20 raw parameters: the optimisation loop's
 *   backward pass through the splatting renderer (Sec. 3.1; Table B-1,
 *   "Backward") and through the slice of Sec. 3.3 Eq. "4dgs" and its
 *   temporal opacity.  Per pixel the entries are
 *   replayed back to front from `last`; each transmittance is recovered as
 *   T_i = T_{i+1} / (1 - alpha_i) from T_final, never stored.  Gradients are
 *   zero through the 0.99 clamp, skipped entries and clamped guard-band
 *   coordinates.
 *   opts       host, may be NULL: persistent / n_workgroups / order / queue as
 *              for gs4d_render_fwd (a separate queue counter, zeroed); the
 *              other fields are ignored
 *   dL_dimage  float [n_views][3][H][W]
 *   dparams    out float [20][n], overwritten (sum over views)
 *   grad2d     optional out float [n_views][n][9] (d mean2D.xy, d conic.abc,
 *              d o_t, d rgb); NULL -> kept in the workspace
 *   ws         >= gs4d_render_bwd_workspace_size(n, n_views)
 * ------------------------------------------------------------------------- */
size_t gs4d_render_bwd_workspace_size(int64_t n, int32_t n_views);
int gs4d_render_bwd(const float *params, int64_t n, const float *rec, const int32_t *touched,
                    const uint32_t *vals, const int32_t *ranges, const gs4d_view *views,
                    int32_t n_views, const gs4d_render_opts *opts, const float *dL_dimage,
                    const float *T_final, const int32_t *last, float *dparams, float *grad2d,
                    void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_render_bwd_2d -- the per-pixel half of gs4d_render_bwd: zeroes and
 *   fills grad2d [n_views][n][9] = d(mean2D.xy, conic.abc, o_t, rgb) with the
 *   back-to-front replay described above (Sec. 3.1 splatting backward).
 * gs4d_preprocess_bwd -- the per-Gaussian half: chain rule from grad2d
 *   through the EWA projection, the conditional at t (Sec. 3.3 Eq. "4dgs"),
 *   the temporal opacity, the 4D rotor and the activations to dparams
 *   [20][n] (overwritten, summed over views).  touched as produced by
 *   gs4d_preprocess (culled entries contribute nothing).
 * ------------------------------------------------------------------------- */
int gs4d_render_bwd_2d(const float *rec, int64_t n, const uint32_t *vals, const int32_t *ranges,
                       const gs4d_view *views, int32_t n_views, const gs4d_render_opts *opts,
                       const float *dL_dimage, const float *T_final, const int32_t *last,
                       float *grad2d, void *stream);
int gs4d_preprocess_bwd(const float *params, int64_t n, const gs4d_view *views, int32_t n_views,
                        const int32_t *touched, const float *grad2d, float *dparams, void *stream);

/* gs4d_tile_order -- work order for the persistent render launches: the
 *   global tiles by decreasing size class (pairs n >= 1: 1 + 8 floor(log2 n)
 *   + the three bits of n below its leading one, eight classes per octave;
 *   empty tiles last), by tile id within a class, computed on the device from
 *   `ranges` in one workgroup, so that the longest tiles start first and the
 *   short ones fill the tail.  Also zeroes n_queues (<= 64) int32 work
 *   counters (the `queue` fields of gs4d_render_opts).  The order only
 *   schedules work: results do not depend on it.
 *   order  out int32 [n_tiles]; ws >= gs4d_tile_order_workspace_size(n_tiles)
 *   (no workspace is used; the query is kept for a stable interface). */
size_t gs4d_tile_order_workspace_size(int64_t n_tiles);
int gs4d_tile_order(const int32_t *ranges, int64_t n_tiles, int32_t *order, int32_t *queues,
                    int32_t n_queues, void *ws, size_t ws_bytes, void *stream);

/* gs4d_set_bwd_variant -- block shape of the render backward: each lane
 *   handles pixels_per_lane (1, 2 or 4) pixels of its tile, so a workgroup
 *   has 256 / pixels_per_lane threads.  Results are identical up to FP32
 *   summation order; the choice only changes speed (picked by the autotuner).
 *   Process-wide setting; returns GS4D_ERR_INVALID_ARG for other values. */
int gs4d_set_bwd_variant(int32_t pixels_per_lane);

/* ---------------------------------------------------------------------------
 * gs4d_grid_prune -- voxel grid pruning (Sec. 3.2): each point goes to the
 *   voxel floor(fl32(x / S_v)) per axis of its motion class (static: voxel
 *   edge voxel_static; dynamic: voxel_dynamic, the per-class sizes of the
 *   Lite/Full presets, Sec. 4.1); points of one (class, voxel) are replaced
 *   by their centroid and the mean of their attributes (FP64 sums); voxels
 *   with fewer than min_count points are dropped.  A class with edge <= 0
 *   is not pruned (each point is its own cell).
 *   key = class << 63 | unpruned << 62 | (ix+2^19) << 40 | (iy+2^19) << 20 | (iz+2^19)
 *   (unpruned: low 62 bits = point index); output ascending by key.
 *   xyz       float [3][m]          attr  float [k_attr][m] (may be NULL if k_attr = 0)
 *   cls       uint8 [m] (nonzero = dynamic) or NULL (all static)
 *   out_xyz   out float [3][capacity]   out_attr out float [k_attr][capacity]
 *   out_count out int32 [capacity]      out_key  out uint64 [capacity]
 *   n_out     out device int64: number of kept voxels (also when over capacity)
 *   status    out device int32: 0 ok, 1 over capacity, 2 voxel index outside [-2^19, 2^19)
 *   m < 2^31; ws >= gs4d_grid_prune_workspace_size(m, k_attr).
 * ------------------------------------------------------------------------- */
size_t gs4d_grid_prune_workspace_size(int64_t m, int32_t k_attr);
int gs4d_grid_prune(const float *xyz, const float *attr, int32_t k_attr, const uint8_t *cls,
                    int64_t m, float voxel_static, float voxel_dynamic, int32_t min_count,
                    int64_t capacity, float *out_xyz, float *out_attr, int32_t *out_count,
                    uint64_t *out_key, int64_t *n_out, int32_t *status, void *ws, size_t ws_bytes,
                    void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_backproject -- back projection on consistent depth (Sec. 3.2, the
 *   back-projection equation): every pixel (x, y) whose accumulated alpha
 *   cover[y][x] > min_cover becomes the world point
 *     X = R^T (xc - t),  xc = ((x + 1/2 - cx) D / fx, (y + 1/2 - cy) D / fy, D),
 *   D = depth_acc / cover (the alpha-weighted depth), with the view's
 *   world-to-camera [R | t] and intrinsics.  Kept pixels are written in
 *   row-major pixel order.
 *   depth_acc, cover  float [H][W] (H, W from the view)
 *   view      host; min_cover > 0
 *   out_xyz   out float [3][capacity]   out_depth out float [capacity]
 *   out_pixel out int32 [capacity]: y W + x of each kept pixel
 *   n_out     out device int64: number of kept pixels (all of them, also past
 *             capacity; only the first `capacity` are written)
 *   depth_sum optional device double, accumulated (caller zeroes): the sum of
 *             D over the kept pixels (the frame's mean depth for the adaptive
 *             voxel edge S_v = lambda (1/N) sum_i mean(D_i) / f, Sec. 3.2)
 *   ws >= gs4d_backproject_workspace_size(H W); H W < 2^31.
 * ------------------------------------------------------------------------- */
size_t gs4d_backproject_workspace_size(int64_t hw);
int gs4d_backproject(const float *depth_acc, const float *cover, const gs4d_view *view,
                     float min_cover, int64_t capacity, float *out_xyz, float *out_depth,
                     int32_t *out_pixel, int64_t *n_out, double *depth_sum, void *ws,
                     size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_heuristic_init -- the initialisation of Sec. 4.1 for k pruned points
 *   (rotor-form parameters [20][k]):
 *     mean xyz = the voxel centroid, mean t = the mean timestamp, rgb = the
 *     mean colour (as given);
 *     log s_t = ln(2 / frames) for dynamic points (2 / fps with time
 *       normalised to [0, 1]: two frame intervals) and 0 for static ones
 *       (s_t = 1, the whole video);
 *     log s_xyz = ln(voxel edge of the point's class); for a class that is
 *       not pruned (edge <= 0, the Full preset's dynamic points), ln(D / f),
 *       the footprint of one back-projected pixel at its depth D;
 *     identity rotors; opacity 0.1 (logit ln(0.1 / 0.9)).
 *   xyz, rgb  float [3] rows of `stride` floats (the first k used)
 *   t         float [k]         depth float [k] (only read for an unpruned class)
 *   dynamic   uint8 [k] (nonzero = dynamic) or NULL (all static)
 *   focal     > 0 when a class is not pruned;  frames >= 2
 *   params    out float [20][k]
 * ------------------------------------------------------------------------- */
int gs4d_heuristic_init(const float *xyz, const float *rgb, const float *t, const float *depth,
                        const uint8_t *dynamic, int64_t k, int64_t stride, float voxel_static,
                        float voxel_dynamic, float focal, int32_t frames, float *params,
                        void *stream);

/* ------------------------------------------------------------------------- *
 * Optimisation-loop helpers (Sec. 4.1: a single photometric loss with the
 * 3D Gaussian-splatting loss weights and optimiser, position learning rate
 * 1e-5, learning-rate schedule stretched to the iteration budget).
 * ------------------------------------------------------------------------- */

/* Adam (bias-corrected) over rows x n SoA parameters.  Row r uses the
 * learning rate lr0[r]^(1-u) lr1[r]^u with u = min(step / budget, 1).
 * step is a device int32 holding the number of steps already taken; the call
 * uses step + 1 and then increments it (graph-replay friendly). */
typedef struct gs4d_adam_cfg {
    float lr0[GS4D_N_FIELDS];
    float lr1[GS4D_N_FIELDS];
    int32_t budget;
    int32_t rows;           /* <= GS4D_N_FIELDS */
    float beta1, beta2, eps;
} gs4d_adam_cfg;
int gs4d_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                   const gs4d_adam_cfg *cfg, int32_t *step, void *stream);

/* L1 = mean |img - target| over count values.  loss (device float) is
 * accumulated with weight * L1; dL_dimg (if not NULL) is accumulated with
 * weight * sign(img - target) / count. */
int gs4d_loss_l1(const float *img, const float *target, int64_t count, float weight, float *loss,
                 float *dL_dimg, void *stream);

/* SSIM (11x11 Gaussian window, sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, zero
 * padding, mean over images x channels x pixels) of img [b][c][h][w]
 * against target.  ssim_sum (device float) is accumulated with the mean
 * SSIM times `weight`; dL_dimg (if not NULL) is accumulated with
 * weight * dSSIM/dimg.  Calls that can run concurrently must not share a
 * workspace. */
size_t gs4d_ssim_workspace_size(int32_t b, int32_t c, int32_t h, int32_t w);
int gs4d_ssim(const float *img, const float *target, int32_t b, int32_t c, int32_t h, int32_t w,
              float weight, float *ssim_sum, float *dL_dimg, void *ws, size_t ws_bytes,
              void *stream);

/* The photometric loss of the optimisation loop in one call (Sec. 4.1, the
 * single photometric loss; reading: w_l1 L1 + w_ssim (1 - SSIM), with
 * w_l1 = 1, w_ssim = 0.2 at scene scale):
 *   loss (device float, overwritten) = w_l1 mean|img - target|
 *                                      + w_ssim (1 - mean SSIM)
 *   dL_dimg (overwritten) = its gradient.
 * img, target [b][c][h][w]; ws >= gs4d_photometric_loss_workspace_size(). */
size_t gs4d_photometric_loss_workspace_size(int32_t b, int32_t c, int32_t h, int32_t w);
int gs4d_photometric_loss(const float *img, const float *target, int32_t b, int32_t c, int32_t h,
                          int32_t w, float w_l1, float w_ssim, float *loss, float *dL_dimg,
                          void *ws, size_t ws_bytes, void *stream);

/* Sum of squared differences, accumulated into sse (device double). */
int gs4d_sse(const float *img, const float *target, int64_t count, double *sse, void *stream);

/* ------------------------------------------------------------------------- *
 * Learned initialisation (not in the paper; it refines the heuristic
 * initialisation of Sec. 4.1, which fixes every back-projected point's
 * temporal scale from its motion class and gives it no velocity).  Per
 * pruned point: 8 nearest neighbours -> 16 standardised features -> a
 * 16-64-64-64-4 SiLU network with BF16 parameters and FP32 accumulation ->
 * (log s_t, v) -> the rotor-form 4D Gaussian whose slice at any t has
 * covariance s^2 I (s = the initial spatial scale), velocity v (the slope of
 * the conditional mean, Sec. 3.3 Eq. "4dgs") and temporal variance s_t^2.
 * ------------------------------------------------------------------------- */

/* gs4d_knn8 -- for every point of xyz [3][n], the 8 other points of
 *   smallest Euclidean distance (FP32 squared distances, ties by smaller
 *   index; duplicates are other points).  Exact: points are sorted by
 *   cell (edge `cell`), cubes of cells around each point grow until no
 *   unvisited cell can hold a closer point, and a point still unresolved
 *   after 8 rings is answered by a scan of all points.
 *   nbr  out int32 [8][n] (-1 where fewer than 8 other points exist)
 *   d2   out float [8][n] (squared distances, ascending; +inf with -1)
 *   status out device int32: 0, or 1 if some point was non-finite or had
 *          |coordinate / cell| >= 2^20 -- such points are left out of the
 *          neighbour graph and get nbr = -1.
 *   cell > 0; n < 2^31; ws >= gs4d_knn8_workspace_size(n). */
size_t gs4d_knn8_workspace_size(int64_t n);
int gs4d_knn8(const float *xyz, int64_t n, float cell, int32_t *nbr, float *d2, int32_t *status,
              void *ws, size_t ws_bytes, void *stream);

/* gs4d_init_features -- the network's 16 inputs per point, standardised
 *   as (f - shift[i]) * scale[i]:
 *     0-2 xyz, 3 depth, 4 2D optical-flow magnitude, then statistics of the
 *     space-time offsets (x_j - x, t_j - t) to the 8 neighbours (population
 *     moments): 5-7 mean spatial offset, 8-10 per-axis variance, 11-13
 *     covariance of each spatial axis with the time offset, 14 variance of
 *     the time offset; 15 motion class (1 dynamic).  On a trail
 *     x = x0 + v (t - t0), features 11-13 over 14 are v.
 *   attr float [>= 6][n] = (r, g, b, t, depth, flow magnitude, ...), the
 *   per-voxel means of the pruned cloud (colour is not an input);
 *   dyn uint8 [n] or NULL; nbr from gs4d_knn8 (entries -1 are skipped; no
 *   neighbour gives offset mean and variance 0).
 *   shift, scale: host float [16].  feat out float [16][n]. */
int gs4d_init_features(const float *xyz, const float *attr, const uint8_t *dyn,
                       const int32_t *nbr, int64_t n, const float *shift, const float *scale,
                       float *feat, void *stream);

/* The network: flat parameters in the order W1 [64][16], b1 [64],
 * W2 [64][64], b2, W3 [64][64], b3, W4 [4][64], b4 [4] (GS4D_MLP_PARAMS
 * values), held as BF16 (uint16 bit patterns); h_l = silu(W_l h_{l-1} + b_l),
 * y = W4 h3 + b4, silu(z) = z / (1 + e^-z); FP32 accumulation. */
#define GS4D_MLP_PARAMS 9668
/* y out float [4][n] for x float [16][n]. */
int gs4d_mlp_fwd(const uint16_t *w_bf16, const float *x, int64_t n, float *y, void *stream);

/* Backward of the network.  Exactly one of dy, target is non-NULL:
 *   dy     float [4][n]: upstream gradient of y;
 *   target float [4][n]: the loss L = (1/n) sum_p sum_o w_o (y_po - t_po)^2
 *          with w_o = out_weight[o] (host float [4]) is differentiated and,
 *          if loss is not NULL, written to loss (device float).
 *   grad out float [GS4D_MLP_PARAMS]: gradient of the parameters (summed
 *        over points in a fixed order: deterministic), overwritten.
 *   dx   out float [16][n] or NULL: gradient of the inputs.
 *   ws >= gs4d_mlp_bwd_workspace_size(n).  n = 0 zeroes grad (and loss). */
size_t gs4d_mlp_bwd_workspace_size(int64_t n);
int gs4d_mlp_bwd(const uint16_t *w_bf16, const float *x, int64_t n, const float *dy,
                 const float *target, const float *out_weight, float *grad, float *dx,
                 float *loss, void *ws, size_t ws_bytes, void *stream);

/* Adam on the FP32 master copy (count values), then the BF16 working copy
 * w_bf16 = master rounded to nearest (ties to even).  step: device int32,
 * steps taken so far; the call uses step + 1 and increments it. */
int gs4d_mlp_adam(float *master, const float *grad, float *m, float *v, uint16_t *w_bf16,
                  int64_t count, float lr, float beta1, float beta2, float eps, int32_t *step,
                  void *stream);

/* Round count FP32 values to BF16 (nearest, ties to even). */
int gs4d_to_bf16(const float *src, uint16_t *dst, int64_t count, void *stream);

/* gs4d_motion_init -- params [20][n] in/out: rows 4..15 (log scales and the
 *   two quaternions) are replaced by the rotor form of
 *       Sigma = [[s^2 I + s_t^2 v v^T, s_t^2 v], [s_t^2 v^T, s_t^2]]
 *   with s = exp(params[4]) (the isotropic initial spatial scale),
 *   log s_t = pred[0], v = pred[1..3] (pred float [4][n]).  Its slice at
 *   any t has covariance s^2 I, conditional-mean slope v and temporal
 *   variance s_t^2 (closed form, the rotation nearest to identity: a
 *   spatial rotation of at most ~55 degrees taking the axis closest to +-v
 *   onto it, then a rotation in that axis' plane with t; scales from the
 *   2x2 eigenproblem; v = 0 gives identity quaternions and log scales
 *   (log s, log s, log s, log s_t)).
 *   A column whose prediction or spatial scale is not finite is left as it
 *   was (the heuristic initialisation stands). */
int gs4d_motion_init(float *params, const float *pred, int64_t n, void *stream);

/* gs4d_motion_of -- out float [4][n] = (1/2 ln Sigma_tt, Sigma_{xyz,t} /
 *   Sigma_tt) of each Gaussian's 4D covariance: its log temporal scale and
 *   velocity (the training targets of the network, taken from Gaussians the
 *   optimiser converged).  Non-finite or degenerate parameters give NaN. */
int gs4d_motion_of(const float *params, int64_t n, float *out, void *stream);

/* ---------------------------------------------------------------------------
 * gs4d_otsu_mask -- static / dynamic split of a motion-probability map by
 *   Otsu's threshold (Sec. 3.2; Otsu 1979).
 *   prob       float [count], count <= 4,000,000 (one map); values clamped to
 *              [0, 1], NaN read as 0; 256 uniform bins, bin(x) =
 *              min(255, floor(256 x))
 *   threshold  out device float or NULL: k* / 256, where k* in 1..255 is the
 *              first split maximising the between-class variance (256 when
 *              every value falls in one bin)
 *   mask       out uint8 [count] or NULL: 1 (dynamic) where bin(x) >= k*
 *   ws         >= gs4d_otsu_workspace_size() bytes
 *   The split is decided on integer class sums with one fixed FP64
 *   evaluation per candidate, so it is reproducible bit for bit.
 * ------------------------------------------------------------------------- */
/* gs4d_threshold_mask -- mask uint8 [count] = 1 where bin(prob) >= k, with
 *   k / 256 the device float `threshold` that gs4d_otsu_mask wrote (bins as
 *   there): one threshold chosen over several maps (a sequence's frames
 *   pooled) applied to each of them. */
int gs4d_threshold_mask(const float *prob, int64_t count, const float *threshold, uint8_t *mask,
                        void *stream);
size_t gs4d_otsu_workspace_size(void);
int gs4d_otsu_mask(const float *prob, int64_t count, float *threshold, uint8_t *mask, void *ws,
                   size_t ws_bytes, void *stream);

/* Fill count floats with value (graph-capturable replacement of memset). */
int gs4d_fill_f32(float *dst, float value, int64_t count, void *stream);
int gs4d_fill_u32(uint32_t *dst, uint32_t value, int64_t count, void *stream);

/* Diagnostics. */
const char *gs4d_status_string(int status);
const char *gs4d_last_error(void);
int gs4d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GS4D_H */
