/*
 * rade.h -- C ABI of the RaDe-GS rasterizer for AMD Instinct MI355X (gfx950).
 *
 * RaDe-GS (arXiv 2406.01467) renders 3D Gaussians by projecting each one to a
 * screen-space splat (Sec. 3.1, Eq. 1-2) and alpha-blending front to back
 * (Eq. 3).  Besides colour it blends a per-pixel depth that is planar over
 * each splat, d = z_c + p (u_c - u, v_c - v) (Sec. 3.2, Eq. 4, with p from
 * Eq. 13-17), and the splat's normal n = normalize(J^T n'), n' = -(q, 1)
 * (Sec. 3.3, Eq. 21-22).  The depth map is the median depth, the depth at
 * which the accumulated opacity crosses one half (Sec. 1); the normal map is
 * blended like colour.  This library computes that rasterizer and its
 * gradient.
 *
 * The call sequence of one forward + backward pass over V views:
 *   rade_views_prepare (host)      fill per-view pixel / tile offsets
 *   rade_project                   Gaussians -> splats, tiles touched
 *   rade_bin_sort                  (view, tile) lists of splats in depth order
 *   rade_render_fwd                colour / depth / normal / alpha maps
 *   rade_render_bwd                gradients of the Gaussian parameters
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller unless it is
 *   documented as host memory.  The library never allocates or frees device
 *   memory; scratch memory comes from a caller-supplied workspace whose size
 *   the matching *_workspace_bytes function returns.
 * - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *   default stream) and returns without waiting, except where an argument
 *   explicitly asks for a host result.  Arguments are validated on the host
 *   before anything is enqueued; an invalid call enqueues nothing.
 * - Floating-point data are IEEE FP32, row-major.  Gaussian parameters are
 *   already activated: scales are standard deviations (> 0), opacities lie
 *   in (0, 1), quaternions are (w, x, y, z) and need not be normalised (the
 *   library normalises them and differentiates through the normalisation).
 * - Spherical harmonics: N x K x 3 floats, K = (degree + 1)^2 (coefficient
 *   major, RGB minor), real SH with the Condon-Shortley phase in the order
 *   m = -l..l per degree; colour = max(0, sum_k sh_k Y_k(dir) + 1/2) with
 *   dir the unit vector from the camera centre to the mean.
 * - Cameras use OpenCV axes (x right, y down, z forward); pixel (px, py) has
 *   its centre at (px + 1/2, py + 1/2).
 * - Maps are planar per view and views are packed back to back: a map with
 *   C channels holds, for view v, C planes of W_v * H_v floats starting at
 *   C * views[v].pix_offset.  For one view this is the CHW layout.
 * - Return value: RADE_OK (0) or a negative error code (rade_strerror).
 *   Every entry point that enqueues GPU work checks its arguments first
 *   (RADE_ERR_INVALID_ARG, RADE_ERR_WORKSPACE), then that the calling
 *   thread's current HIP device is a gfx950 GPU (RADE_ERR_UNSUPPORTED_DEVICE;
 *   the kernels are compiled for gfx950 only).  The device is queried once
 *   per device ordinal and the answer cached.
 * - Workspaces: each entry point that needs scratch memory has its own size
 *   function (rade_bin_sort_workspace, rade_tile_order_workspace,
 *   rade_render_bwd_workspace, rade_normal_consistency_workspace,
 *   rade_marching_cubes_workspace) taking exactly the sizes that call
 *   depends on, in place of one rade_workspace_bytes(which, ...) selector.
 *   They are host functions, need no GPU and return 0 for invalid sizes.
 */
#ifndef RADE_H
#define RADE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RADE_OK 0
#define RADE_ERR_INVALID_ARG (-1)        /* bad pointer, size or setting; nothing enqueued */
#define RADE_ERR_CAPACITY (-2)           /* more output than the capacity given (pairs, mesh) */
#define RADE_ERR_HIP (-3)                /* a HIP runtime call failed */
#define RADE_ERR_UNSUPPORTED_DEVICE (-4) /* the current device is not a gfx950 GPU (or there
                                            is none); nothing enqueued */
#define RADE_ERR_WORKSPACE (-5)          /* workspace smaller than required; nothing enqueued */
#define RADE_ERR_TOO_LARGE (-6)          /* input larger than the fixed scratch of an
                                            allocation-free entry point; nothing enqueued */

/* Rasterizer settings.  Quantities the paper leaves open default to the
 * values of the 3D Gaussian Splatting code base the paper builds on (it
 * states that it keeps that code base's default parameters, Sec. 4.1). */
/* Work schedules of the tile kernels (rade_settings.schedule). */
#define RADE_SCHEDULE_TILE 0        /* one workgroup per tile, natural order */
#define RADE_SCHEDULE_HEAVY_FIRST 1 /* one workgroup per tile, longest lists first */
#define RADE_SCHEDULE_PERSISTENT 2  /* resident workgroups pull tiles, longest first */

typedef struct rade_settings {
  int32_t tile_w, tile_h;  /* tile size: 8x8, 16x8, 8x16, 16x16, 32x16 or 16x32 pixels */
  int32_t sh_degree;       /* 0..3 */
  int32_t schedule;        /* RADE_SCHEDULE_*; the last two need a tile order */
  double dilation;         /* added to the 2x2 footprint covariance, px^2 (0.3) */
  double near_plane;       /* Gaussians with camera z <= near are culled (0.2) */
  double alpha_min;        /* blends with alpha < alpha_min are skipped (1/255) */
  double alpha_max;        /* alpha is clamped to alpha_max (0.99); below 1 in FP32 */
  double t_min;            /* a pixel stops before the blend that would leave T < t_min (1e-4) */
  double power_cut;        /* blends with 1/2 d^T conic d > power_cut are skipped (4.5, 3 sigma) */
  double fov_clamp;        /* x/z, y/z in the Jacobian clamped to fov_clamp * W/(2 fx) (1.3) */
  double degenerate;       /* q := 0 when det(B0) <= degenerate * tr(B0)^2 (1e-6) */
  double bg[3];            /* background colour, blended with the final transmittance */
  int32_t depth_mode;      /* RADE_DEPTH_*: per-pixel depth of Eq. 4 or of Eq. 7 */
  int32_t wave_w;          /* pixels per wavefront row: 8 (8x8), 16 (16x4) or 32 (32x2);
                              0 = 8.  The blocks must tile the tile exactly. */
  int32_t batch;           /* splats staged per round: 64, 128 or 256; 0 = one per thread
                              of the tile workgroup (tile_w * tile_h).  Shapes other than
                              8x8 waves with one splat per thread are compiled for the
                              plain forward and backward only: with a distortion map, a
                              blend count, an evaluation count or the exact depth, the
                              render calls return RADE_ERR_INVALID_ARG.  Maps do not
                              depend on either field; gradients only up to the order of
                              FP32 additions. */
  int32_t lane_masks;      /* 0 or 1.  Tiles of one 8x8 wave always stage, per splat, the
                              64-bit mask of the wave's pixels its ellipse can reach (the
                              loops skip splats that reach no pixel still working) and walk
                              the backward as four 4x4 quadrant groups per wave; 1 does
                              the same on every wave of larger tiles of 8x8 waves (with
                              batch 0; the plain forward and backward only, as above).
                              Maps do not depend on it; gradients only up to the order of
                              FP32 additions. */
} rade_settings;

/* Per-pixel depth of a splat.  AFFINE: the plane d = z + p . (u_c - u,
 * v_c - v) of Sec. 3.2.2 (Eq. 4), the method's depth, forward and backward.
 * EXACT: the camera z of the maximum of the Gaussian along the ray through
 * the pixel centre (Sec. 3.2.1, Eq. 5-7), an accuracy reference for the
 * plane; forward only (rade_render_bwd rejects it).  It needs the
 * depth_quad records of rade_project. */
#define RADE_DEPTH_AFFINE 0
#define RADE_DEPTH_EXACT 1

/* One camera.  The caller fills the first five rows; rade_views_prepare
 * fills the offsets. */
typedef struct rade_view {
  int32_t width, height;   /* pixels, 1..32767 */
  float fx, fy, cx, cy;    /* pinhole intrinsics in pixels */
  float R[9];              /* world -> camera rotation, row-major */
  float t[3];              /* world -> camera translation: x_cam = R x_world + t */
  int32_t tiles_x, tiles_y;/* tiles per row / column (filled by rade_views_prepare) */
  int64_t pix_offset;      /* first pixel of this view in the packed maps (filled) */
  int64_t tile_offset;     /* first global tile index of this view (filled) */
} rade_view;               /* 96 bytes */

/* Projected splat of one (view, Gaussian), 80 bytes.  The quadratic form of
 * the splat, power = 1/2 d^T B^-1 d with d = (u_c - u, v_c - v) and B the
 * dilated 2x2 footprint covariance, is stored in factored form:
 *   power * log2(e) = (w[0] dx + w[1] dy)^2 + (w[2] dx + w[3] dy)^2,
 * with (w[0], w[1]) and (w[2], w[3]) the eigenvectors of B scaled by
 * sqrt(log2(e) / (2 lambda)); it is exact up to FP32 rounding even for
 * very elongated splats.  rect is the inclusive pixel rectangle that holds
 * every pixel with alpha >= alpha_min; rect[0] > rect[1] marks a splat that
 * is culled or off screen (every other field is then unspecified). */
typedef struct rade_splat {
  double uc, vc;          /* centre in pixels (projected mean) */
  float w[4];             /* factored quadratic form, see above */
  float opacity;
  float rgb[3];           /* SH colour for this view */
  float z;                /* camera-space depth of the centre; sort key */
  float p[2];             /* depth plane: d = z + p . (u_c - u, v_c - v)   (Eq. 4) */
  float n[3];             /* unit normal in camera space, facing the camera (Eq. 22) */
  int16_t rect[4];        /* x0, x1, y0, y1 */
} rade_splat;

/* Host function.  Fills tiles_x, tiles_y, pix_offset and tile_offset of
 * views[0..V) for the tile size of `s`; returns the totals (either pointer
 * may be NULL).  The device copy of the views that the other calls read
 * must be made from the array after this call. */
int rade_views_prepare(const rade_settings* s, rade_view* views, int32_t V,
                       int64_t* total_pixels, int64_t* total_tiles);

/* Projection (Sec. 3.1 Eq. 1-2; Sec. 3.2 Eq. 4, 13-17; Sec. 3.3 Eq. 21-22).
 * For every Gaussian g and view v writes splats[v*N + g] and
 * tiles_touched[v*N + g] = number of tiles its rect covers (0 if culled),
 * and, when bin_records is not NULL, the 16-byte binning record
 * bin_records[4*(v*N + g) .. +3] = {bits of the float32 depth z (as in the
 * splat), tx0 | ty0 << 16, tx1 | ty1 << 16, tiles_touched}: the first and
 * last tile column and row the rect covers (all four words 0 if culled).
 * rade_bin_sort reads these 16 bytes instead of the 80-byte splat.
 *   views_dev : V rade_view structs in device memory (after views_prepare)
 *   means N*3, scales N*3, quats N*4, opacities N, sh N*K*3 (see above)
 * A Gaussian is culled when a parameter is not finite, its camera z <=
 * near_plane, its quaternion is zero or opacity <= alpha_min (then no pixel
 * reaches alpha >= alpha_min).  The rect holds every pixel centre where
 * power <= min(power_cut, ln(opacity / alpha_min)), i.e. every pixel the
 * per-pixel rule of rade_render_fwd can blend.  The geometry is evaluated in
 * FP64 and rounded to the FP32 fields once. */
/* depth_quad (V*N records of 8 floats, 16-byte aligned): required when
 * depth_mode is RADE_DEPTH_EXACT, ignored (may be NULL) otherwise.  With A
 * the camera-space inverse covariance, r_c = (x/z, y/z, 1) the centre's ray
 * and D0 = r_c^T A r_c, the record holds g = (A r_c)_{0,1} / D0 scaled by
 * (1/fx, 1/fy) and H = A_{00,01,11} / D0 scaled by (1/fx^2, 2/(fx fy),
 * 1/fy^2), then three zeros; at pixel offset (dx, dy) = (u_c - u, v_c - v)
 * the ray maximum has depth z (1 - g.d) / (1 - 2 g.d + H0 dx^2 + H1 dx dy +
 * H2 dy^2) (Eq. 7 rewritten around the centre).  A scale below 1e-15 counts
 * as 1e-15 there. */
int rade_project(const rade_settings* s, const rade_view* views_dev, int32_t V, int64_t N,
                 const float* means, const float* scales, const float* quats,
                 const float* opacities, const float* sh, rade_splat* splats,
                 int32_t* tiles_touched, uint32_t* bin_records, float* depth_quad,
                 void* stream);

/* Workspace bytes for rade_bin_sort with V views, N Gaussians, `capacity`
 * pairs and `total_tiles` tiles. */
size_t rade_bin_sort_workspace(int32_t V, int64_t N, int64_t capacity, int64_t total_tiles);

/* Binning and sorting (Sec. 3.1: splats are blended in the order of their
 * centre depth).  Emits one (tile, splat) pair for every tile a splat's rect
 * covers and orders the pairs by (global tile, float32 depth, Gaussian id);
 * equivalently a stable sort by the 64-bit key (tile << 32 | bits(z)).
 *   views_host/views_dev : the same V prepared views, host and device copies
 *   tiles_touched, bin_records: rade_project's outputs (same settings and
 *                           views; bin_records is required)
 *   pair_ids   [capacity] : Gaussian id of each sorted pair
 *   tile_ranges[2*total_tiles]: [begin, end) into pair_ids per global tile
 *   keys       [capacity] : optional (may be NULL), the sorted 64-bit keys
 *   n_pairs_dev           : device int64 receiving the pair count M
 *   n_pairs_host          : optional host int64; when given the call waits
 *                           for the pair count, stores it and returns
 *                           RADE_ERR_CAPACITY at once if M > capacity
 * When M > capacity, pair_ids and keys are left untouched and every tile
 * range is empty ([0, 0)); *n_pairs_dev still holds M so the caller can
 * retry with capacity >= M.  capacity must be < 2^32. */
int rade_bin_sort(const rade_settings* s, const rade_view* views_host,
                  const rade_view* views_dev, int32_t V, int64_t N,
                  const int32_t* tiles_touched, const uint32_t* bin_records,
                  uint32_t* pair_ids, uint32_t* tile_ranges,
                  uint64_t* keys, int64_t capacity, int64_t* n_pairs_dev,
                  int64_t* n_pairs_host, void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes for rade_tile_order over `total_tiles` tiles. */
size_t rade_tile_order_workspace(int64_t total_tiles);

/* Tile visiting order for the HEAVY_FIRST and PERSISTENT schedules: global
 * tile indices sorted by decreasing list length (coarse: 16 buckets per
 * octave of length, stable within a bucket).  tile_order has total_tiles + 1
 * uint32 entries; the last one is scratch (the work-queue counter of the
 * persistent kernels, reset by them before every launch). */
int rade_tile_order(const rade_settings* s, const rade_view* views_host, int32_t V,
                    const uint32_t* tile_ranges, uint32_t* tile_order, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Forward rendering (Eq. 3 applied to colour, the depth of Eq. 4, the normal
 * of Eq. 22 and alpha; median depth of Sec. 1).  For each pixel, splats of
 * its tile list are visited in order; a splat is skipped when its power
 * exceeds power_cut or its alpha = min(alpha_max, opacity * exp(-power)) is
 * below alpha_min; the pixel stops before a splat that would bring its
 * transmittance T below t_min.  Blend weights w_i = alpha_i T_i give
 *   color  (3 planes) = sum w_i rgb_i + T_final bg
 *   depth  (2 planes) = sum w_i d_i  |  d of the median splat (0 if none)
 *   normal (3 planes) = sum w_i n_i (not renormalised)
 *   alpha  (1 plane)  = sum w_i
 * The median splat is the last one blended while the incoming T > 1/2.
 * Saved state for rade_render_bwd (1 plane each):
 *   t_final (float), last (int32: position of the last blended splat within
 *   its tile's list, -1 if none), median (int32: Gaussian id of the median
 *   splat, -1 if none); count (int32, optional, may be NULL): splats blended.
 * evals (int32, 1 plane, optional, may be NULL): splats the pixel evaluated
 *   (power and alpha computed) while it was still blending, i.e. the work the
 *   tile lists and the per-wavefront culling leave to the pixel; sum(evals) /
 *   sum(count) measures how much of that work blends.  A splat counts for
 *   every pixel of a wavefront that evaluates it, whether or not it passes
 *   the per-pixel tests.  Unlike every other output it depends on the tile
 *   size, the wave shape and the staging batch.
 * Every output except evals is independent of the tile size, wave shape,
 * batch and schedule, bit for bit: a pixel blends the same splats in the same
 * order with the same FP32 operations whichever tile holds it (each splat's
 * centre is rounded relative to a 32-pixel-aligned origin that depends on the
 * pixel only).
 * distortion (1 plane, optional, may be NULL): the depth distortion of
 * Sec. 3.4 Eq. 23 per pixel, sum_{i,j} w_i w_j (d_i - d_j)^2 over the blended
 * splats (d_i the depth of Eq. 4 at the pixel, or of Eq. 7 in exact mode).
 * depth_quad: rade_project's exact-depth records, required when depth_mode
 * is RADE_DEPTH_EXACT (both depth planes then hold the exact ray-maximum
 * depth; weights, colour, normals and alpha are those of the affine mode),
 * ignored otherwise.
 * lane_masks (optional, may be NULL; 16-byte aligned): where the launch shape
 * keeps per-lane splat masks (rade_lane_mask_bytes > 0), the forward writes
 * the masks of every (list position, 8x8 wave) pair it stages there, for
 * rade_render_bwd to read instead of computing them again; ignored for other
 * shapes.  Size: rade_lane_mask_bytes(s, n_pairs) for the lists' pair
 * count.  The contents are an opaque cache tied to these lists and this
 * launch shape. */
int rade_render_fwd(const rade_settings* s, const rade_view* views_host,
                    const rade_view* views_dev, int32_t V, int64_t N, const rade_splat* splats,
                    const uint32_t* pair_ids, const uint32_t* tile_ranges,
                    uint32_t* tile_order, float* color,
                    float* depth, float* normal, float* alpha, float* t_final, int32_t* last,
                    int32_t* median, int32_t* count, int32_t* evals, float* distortion,
                    const float* depth_quad, uint64_t* lane_masks, void* stream);

/* Bytes of the lane-mask cache of rade_render_fwd / rade_render_bwd for
 * n_pairs list entries: 8 bytes per (pair, 8x8 wave of a tile) where the
 * launch shape keeps lane masks (8x8 tiles of 8x8 waves, or lane_masks = 1
 * on larger tiles), else 0 (the cache is unused).  Host function. */
size_t rade_lane_mask_bytes(const rade_settings* s, int64_t n_pairs);

/* Workspace bytes for rade_render_bwd; recompute != 0 reserves room to
 * recompute the splats (splats == NULL in rade_render_bwd).  The workspace
 * must be 16-byte aligned (device allocations are); RADE_ERR_INVALID_ARG
 * otherwise.  Layout, each region starting at a multiple of 256 bytes from
 * the workspace start: the per-(view, Gaussian) gradient records (V*N*64
 * bytes), then, with recompute, the recomputed splat records (V*N rade_splat)
 * and tile counts (V*N int32) exactly as rade_project writes them.  A caller
 * may therefore let its forward pass project into those two regions: the
 * recomputing backward overwrites them with the same values, and no second
 * copy of the records is needed. */
size_t rade_render_bwd_workspace(const rade_settings* s, int32_t V, int64_t N, int recompute);

/* Backward pass: gradients of the Gaussian parameters from the upstream
 * gradients of the maps of rade_render_fwd.  The blend state of each pixel
 * is recomputed back to front from the saved final transmittance (no
 * per-blend state is stored).  d_color (3 planes), d_depth (2 planes:
 * expected, median), d_normal (3), d_alpha (1) may each be NULL (zero).  No
 * gradient flows through the choice of the median splat or through the
 * tile lists.  splats may be NULL, in which case they are recomputed from
 * the parameters into the workspace.  The outputs d_means (N*3), d_scales
 * (N*3), d_quats (N*4), d_opacities (N), d_sh (N*K*3) are OVERWRITTEN with
 * the gradient summed over the V views.  tile_order as in rade_render_fwd.
 * d_distortion (1 plane, optional, may be NULL): upstream gradient of the
 * distortion map; its adjoint holds the blend weights constant (they are
 * detached in the training loss of Sec. 4.1), so it reaches each splat
 * through its depth only: 4 g A w_i (d_i - D/A) with A and D the alpha and
 * expected-depth maps of the forward, which must then be passed as `alpha`
 * (1 plane) and `depth` (the 2-plane depth map); both are ignored when
 * d_distortion is NULL.  lane_masks (optional, may be NULL; 16-byte
 * aligned): the cache the forward filled for the same lists, settings and
 * saved state; where the launch shape keeps lane masks the backward reads
 * them instead of computing them (NULL: computed; the gradients are the same
 * either way up to the order of FP32 additions).  Contents that do not come
 * from that forward give undefined gradients. */
int rade_render_bwd(const rade_settings* s, const rade_view* views_host,
                    const rade_view* views_dev, int32_t V, int64_t N, const float* means,
                    const float* scales, const float* quats, const float* opacities,
                    const float* sh, const rade_splat* splats, const uint32_t* pair_ids,
                    const uint32_t* tile_ranges, uint32_t* tile_order,
                    const float* t_final, const int32_t* last,
                    const int32_t* median, const float* d_color, const float* d_depth,
                    const float* d_normal, const float* d_alpha, const float* d_distortion,
                    const float* depth, const float* alpha, const uint64_t* lane_masks,
                    float* d_means, float* d_scales, float* d_quats, float* d_opacities,
                    float* d_sh, void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes for rade_normal_consistency over `total_pixels` pixels. */
size_t rade_normal_consistency_workspace(int64_t total_pixels);

/* Normal-consistency regulariser (Sec. 3.4, Eq. 24) of rendered maps and its
 * gradient.  Per view, over the interior pixels p (not on the border), with
 * P(q) the back-projection of the median depth D (depth plane 1) through
 * pixel q's centre:
 *   c(p)  = (P(p + x) - P(p - x)) x (P(p + y) - P(p - y)),
 *   n~(p) = c / |c| oriented towards the camera (0 where c = 0),
 *   loss[v] = weight / n_interior * sum_p (alpha(p) - N(p) . n~(p)),
 * which equals Eq. 24's sum_i w_i (1 - n_i . n~) because alpha and N are the
 * blended weights and normals.  loss (V floats, device) is overwritten.  With
 * accumulate != 0 the gradient is ADDED to d_depth (plane 1 only), d_normal
 * and d_alpha (same planar layouts as the maps), so other loss terms can be
 * accumulated there first; with accumulate == 0 the three maps are
 * OVERWRITTEN (both depth planes; entries with no gradient become 0), with
 * the same bits as adding into zeroed maps.  n~ is not detached: the
 * gradient reaches the median depth. */
int rade_normal_consistency(const rade_view* views_host, const rade_view* views_dev, int32_t V,
                            const float* depth, const float* normal, const float* alpha,
                            float weight, float* loss, float* d_depth, float* d_normal,
                            float* d_alpha, int32_t accumulate, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Allocation-free form of rade_normal_consistency, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments without the workspace,
 * same kernels, same results bit for bit.  Its scratch (one loss partial per
 * 32x8 pixel block) is a fixed array of RADE_NC_NOALLOC_MAX_BLOCKS floats
 * (512 KiB) that the library holds on every GPU it runs on until the process
 * ends; its device address is looked up once per device, on the first call
 * made with that device current.  Views with more blocks than that in total
 * (sum over views of ceil(W/32) * ceil(H/8); about 33M pixels) are rejected
 * with RADE_ERR_TOO_LARGE before anything is enqueued.  Every call on one
 * GPU shares that one array, and the kernels write every partial they read,
 * so nothing needs clearing between calls; but calls that overlap on one GPU
 * (on different streams, or from threads without ordering) race on it and
 * must be serialised by the caller.  Calls no hipMalloc, hipFree or other
 * allocating routine. */
#define RADE_NC_NOALLOC_MAX_BLOCKS 131072
int rade_normal_consistency_noalloc(const rade_view* views_host, const rade_view* views_dev,
                                    int32_t V, const float* depth, const float* normal,
                                    const float* alpha, float weight, float* loss,
                                    float* d_depth, float* d_normal, float* d_alpha,
                                    int32_t accumulate, void* stream);

/* Gradient of an L1 colour loss, the mean absolute difference of each
 * view's three colour planes to a target (the colour term of the training
 * loss, Sec. 4.1): d_color = weight * sign(color - target) / (3 W H) per
 * view, OVERWRITTEN for every pixel (sign(0) = 0; a NaN difference stays
 * NaN).  color, target, d_color: 3-plane maps of the V prepared views. */
int rade_l1_color_grad(const rade_view* views_host, const rade_view* views_dev, int32_t V,
                       const float* color, const float* target, float weight, float* d_color,
                       void* stream);

/* 3D smoothing filter (the Mip-Splatting filter the paper trains with,
 * Sec. 4.1).  For each Gaussian, rate = max over the views whose camera z >
 * near_plane and whose image widened by `margin` x (width, height) on every
 * side holds the projected mean, of fx / z (pixels per world unit at the
 * mean); var[g] = scale / rate^2, or 0 when no view sees the mean.  means
 * N*3, var N (device).  The variance depends on the means and cameras only;
 * callers recompute it from time to time and treat it as a constant. */
int rade_filter3d_var(const rade_settings* s, const rade_view* views_dev, int32_t V, int64_t N,
                      const float* means, float scale, float margin, float* var, void* stream);

/* Convolution of each Gaussian with its filter: scales_out = sqrt(scales^2 +
 * var) per axis (the covariance R S^2 R^T + var I keeps its rotation) and
 * opacities_out = opacities * sqrt(prod scales^2 / prod scales_out^2), which
 * keeps the Gaussian's integral.  Feed the outputs to rade_project. */
int rade_filter3d_apply(int64_t N, const float* scales, const float* opacities, const float* var,
                        float* scales_out, float* opacities_out, void* stream);

/* Adjoint of rade_filter3d_apply with var held constant: from the gradients
 * of the filtered scales (N*3) and opacities (N) to those of the unfiltered
 * ones.  d_scales / d_opacities may alias d_scales_out / d_opacities_out. */
int rade_filter3d_apply_bwd(int64_t N, const float* scales, const float* opacities,
                            const float* var, const float* d_scales_out,
                            const float* d_opacities_out, float* d_scales, float* d_opacities,
                            void* stream);

/* TSDF fusion of rendered median-depth maps (the mesh extraction of
 * Sec. 4.1, a truncated signed distance field in the manner of Curless and
 * Levoy).  Voxel (i, j, k) of the nx x ny x nz grid has centre origin + (i +
 * 1/2, j + 1/2, k + 1/2) voxel and index (k ny + j) nx + i.  For every view
 * with camera z > near_plane whose projection of the centre falls in pixel
 * (floor(u), floor(v)) of the image and whose median depth D there is
 * positive: s = D - z; views with s >= -trunc contribute min(1, s / trunc)
 * with weight 1.  tsdf (nx ny nz floats) receives the mean contribution (0
 * where none), weight the number of contributing views.
 *   views_host/views_dev : the V prepared views the maps were rendered for
 *   depth                : the 2-plane depth maps of rade_render_fwd
 *   origin               : host, 3 doubles
 * Limit: nx ny nz <= 2^32 - 1. */
int rade_tsdf_fuse(const rade_settings* s, const rade_view* views_host,
                   const rade_view* views_dev, int32_t V, const float* depth,
                   const double* origin, double voxel, int32_t nx, int32_t ny, int32_t nz,
                   float trunc, float* tsdf, float* weight, void* stream);

/* Marching Cubes over a TSDF grid (the mesh extraction of Sec. 4.1,
 * Lorensen and Cline): the triangle mesh of the iso level of an nx x ny x nz
 * grid (tsdf and weight as rade_tsdf_fuse writes them, x fastest, voxel
 * centres at origin + (i + 1/2) voxel).  Cells are the cubes between 2 x 2 x 2
 * neighbouring centres; a cell is meshed only when its eight corners all
 * have weight > 0.  A corner is inside when its value is below iso.
 *
 * Triangulation rule (the same for every cell, fixed at compile time):
 * corner b of a cell is at offset (b & 1, b >> 1 & 1, b >> 2 & 1); local
 * edge 4 a + o1 + 2 o2 runs along axis a at offsets o1, o2 on the other two
 * axes (in increasing axis order).  A face with two sign changes holds one
 * segment between its crossed edges, a face with four holds two, each
 * cutting off one inside corner (no cracks between cells).  Segments are
 * directed so that triangle normals point up the field (from inside to
 * outside), close into cycles taken in the order of their smallest edge,
 * and each cycle becomes a fan from its smallest edge whose chords to the
 * cycle's non-adjacent edges share no cube face.
 *
 * Output: verts (3 floats per vertex): one vertex per grid edge that
 * changes sign between two observed voxels and lies in a meshed cell, at the
 * linear zero of the field along the edge, ordered by the edge's id 3 q + a
 * (q the index of its lower voxel, a its axis); tris (3 vertex indices per
 * triangle) cell by cell in increasing cell index ((k (ny - 1) + j)(nx - 1)
 * + i), then in the rule's order.  Normals (v1 - v0) x (v2 - v0) point to
 * increasing values.
 *
 * At most max_verts / max_tris are written.  The call SYNCHRONISES the
 * stream to return the counts in *n_verts and *n_tris; when either exceeds
 * its capacity it returns RADE_ERR_CAPACITY (the outputs are then
 * incomplete; call again with buffers of the reported size).
 * Limits: 3 nx ny nz <= 2^32 - 1.  Workspace: rade_marching_cubes_workspace
 * bytes (about 15 bytes per voxel). */
size_t rade_marching_cubes_workspace(int32_t nx, int32_t ny, int32_t nz);
int rade_marching_cubes(const float* tsdf, const float* weight, int32_t nx, int32_t ny,
                        int32_t nz, const double* origin, double voxel, float iso,
                        void* workspace, size_t workspace_bytes, float* verts, int64_t max_verts,
                        uint32_t* tris, int64_t max_tris, int64_t* n_verts, int64_t* n_tris,
                        void* stream);

/* The compiled triangulation table (host memory, no GPU needed): ntri[256]
 * triangles per cell code and tri[256 * 15] local edge ids, three per
 * triangle. */
int rade_marching_cubes_table(uint8_t* ntri, uint8_t* tri);

/* Kernel timing without a profiler.  After this call, every launch of the
 * kernel `kernel` (one of RADE_KERNEL_*) is bracketed by hipEventRecord of
 * `start_event` and `stop_event` (hipEvent_t passed as void*) on the stream
 * the kernel is launched on; NULL events switch the recording off.  The
 * setting is process-wide and not thread-safe: it is meant for benchmarks
 * that read hipEventElapsedTime after each call. */
#define RADE_KERNEL_PROJECT 1
#define RADE_KERNEL_RENDER_FWD 2
#define RADE_KERNEL_RENDER_BWD 3
#define RADE_KERNEL_PROJECT_BWD 4
int rade_set_kernel_events(int kernel, void* start_event, void* stop_event);

/* Static description of an error code (never NULL). */
const char* rade_strerror(int code);

/* Device check: RADE_OK when the calling thread's current HIP device is a
 * gfx950 GPU, RADE_ERR_UNSUPPORTED_DEVICE otherwise (also when no device is
 * present).  The entry points above make the same check themselves. */
int rade_device_check(void);

/* ABI version of this header: 8. */
int rade_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RADE_H */
