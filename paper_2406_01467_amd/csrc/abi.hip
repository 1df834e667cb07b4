// extern "C" entry points of librade.so: argument checks and launches.
// Declarations and documentation: include/rade.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace rade {
hipError_t launch_project(const rade_settings& st, const rade_view* views, int V, int64_t N,
                          const float* means, const float* scales, const float* quats,
                          const float* opac, const float* sh, rade_splat* splats,
                          int32_t* tiles_touched, uint32_t* bin_records, float* depth_quad,
                          hipStream_t stream);
hipError_t launch_project_bwd(const rade_settings& st, const rade_view* views, int V, int64_t N,
                              const float* means, const float* scales, const float* quats,
                              const float* opac, const float* sh, const float* gsplat,
                              float* d_means, float* d_scales, float* d_quats, float* d_opac,
                              float* d_sh, hipStream_t stream);
size_t bin_sort_workspace(int64_t VN, int64_t capacity);
hipError_t launch_bin_sort(const rade_settings& s, const rade_view* views_host,
                           const rade_view* views_dev, int V, int64_t N,
                           const int32_t* tt, const uint32_t* bin_records, uint32_t* pair_ids,
                           uint32_t* ranges, uint64_t* keys, int64_t capacity,
                           int64_t* n_pairs_dev, int64_t* n_pairs_host, void* ws,
                           hipStream_t st, int* capacity_exceeded);
bool tile_supported(int tw, int th);
bool wave_shape_supported(int tw, int th, int wave_w);
bool render_shape_is_default(int tw, int th, int wave_w, int batch, int lane_masks);
int lane_masks_per_pair(int tw, int th, int wave_w, int batch, int lane_masks);
hipError_t launch_render_fwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, const uint32_t* order, float* color,
                             float* depth, float* normal, float* alpha, float* tf,
                             int32_t* last, int32_t* med, int32_t* cnt, int32_t* evals,
                             float* distortion, const float* depth_quad, uint64_t* lane_masks,
                             hipStream_t st);
hipError_t launch_render_bwd(const rade_settings& s, const rade_view* views, int V, int64_t N,
                             int64_t tiles, const rade_splat* splats, const uint32_t* ids,
                             const uint32_t* ranges, const uint32_t* order, const float* tf,
                             const int32_t* last, const int32_t* med, const float* dc,
                             const float* dd, const float* dn, const float* da,
                             const float* ddist, const float* fwd_depth, const float* fwd_alpha,
                             float* gsplat, const uint64_t* lane_masks, hipStream_t st);
size_t tile_order_workspace(int64_t tiles);
size_t normal_consistency_workspace(int64_t total_pixels);
hipError_t launch_l1_color_grad(const rade_view* views, int V, int64_t total, const float* color,
                                const float* target, double weight, float* d_color,
                                hipStream_t st);
hipError_t launch_normal_consistency(const rade_view* views_host, const rade_view* views, int V,
                                     int64_t total,
                                     const float* depth, const float* normal,
                                     const float* alpha, float weight, float* loss,
                                     float* d_depth, float* d_normal, float* d_alpha,
                                     bool accumulate, void* ws, hipStream_t st);
hipError_t launch_tile_order(const uint32_t* ranges, int64_t tiles, uint32_t* order, void* ws,
                             hipStream_t st);
int64_t normal_consistency_blocks(const rade_view* views_host, int V);
hipError_t nc_scratch_address(void** out);
hipError_t launch_filter3d_var(const rade_view* views, int V, int64_t N, const float* means,
                               double near_plane, float scale, float margin, float* var,
                               hipStream_t st);
hipError_t launch_filter3d_apply(int64_t N, const float* scales, const float* opac,
                                 const float* var, float* scales_out, float* opac_out,
                                 hipStream_t st);
hipError_t launch_filter3d_apply_bwd(int64_t N, const float* scales, const float* opac,
                                     const float* var, const float* d_scales_f,
                                     const float* d_opac_f, float* d_scales, float* d_opac,
                                     hipStream_t st);
hipError_t launch_tsdf_fuse(const rade_view* views, int V, const float* depth,
                            const double* origin, double voxel, int64_t nx, int64_t ny,
                            int64_t nz, double near_plane, float trunc, float* tsdf,
                            float* weight, hipStream_t st);
size_t marching_cubes_workspace(int64_t nx, int64_t ny, int64_t nz);
void marching_cubes_table(uint8_t* ntri, uint8_t* tri);
hipError_t launch_marching_cubes(const float* tsdf, const float* weight, int64_t nx, int64_t ny,
                                 int64_t nz, const double* origin, double voxel, float iso,
                                 void* ws, float* verts, int64_t max_verts, uint32_t* tris,
                                 int64_t max_tris, const uint32_t** nv_dev,
                                 const uint64_t** nt_dev, hipStream_t st);
}  // namespace rade

namespace {

bool grid_ok(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return false;
  // vertex ids are 32-bit: every grid edge must have one
  return 3 * (int64_t)nx * ny * nz <= (int64_t)UINT32_MAX;
}

bool settings_ok(const rade_settings* s) {
  if (!s) return false;
  if (!rade::tile_supported(s->tile_w, s->tile_h)) return false;
  if (s->sh_degree < 0 || s->sh_degree > 3) return false;
  if (s->schedule < RADE_SCHEDULE_TILE || s->schedule > RADE_SCHEDULE_PERSISTENT) return false;
  // the backward divides by 1 - alpha, so the clamp must stay below 1 in FP32
  if (!(s->alpha_min > 0.0) || !((float)s->alpha_max < 1.0f) || !(s->alpha_min < s->alpha_max))
    return false;
  if (!(s->t_min > 0.0 && s->t_min < 1.0) || !(s->power_cut > 0.0)) return false;
  if (!(s->dilation >= 0.0) || !std::isfinite(s->near_plane) || !(s->fov_clamp > 0.0))
    return false;
  if (!(s->degenerate >= 0.0)) return false;
  if (s->depth_mode != RADE_DEPTH_AFFINE && s->depth_mode != RADE_DEPTH_EXACT) return false;
  if (!rade::wave_shape_supported(s->tile_w, s->tile_h, s->wave_w)) return false;
  if (s->batch != 0 && s->batch != 64 && s->batch != 128 && s->batch != 256) return false;
  if (s->lane_masks != 0 && s->lane_masks != 1) return false;
  return true;
}

bool views_ok(const rade_view* v, int32_t V) {
  if (!v || V < 1) return false;
  for (int i = 0; i < V; ++i) {
    if (v[i].width < 1 || v[i].height < 1 || v[i].width > 32767 || v[i].height > 32767)
      return false;
    if (!(v[i].fx > 0.f) || !(v[i].fy > 0.f)) return false;
  }
  return true;
}

bool counts_ok(int32_t V, int64_t N) {
  return V >= 1 && N >= 0 && (int64_t)V * N < ((int64_t)1 << 32);
}

int64_t total_tiles(const rade_view* v, int32_t V) {
  int64_t t = 0;
  for (int i = 0; i < V; ++i) t += (int64_t)v[i].tiles_x * v[i].tiles_y;
  return t;
}

int hip_status(hipError_t e) { return e == hipSuccess ? RADE_OK : RADE_ERR_HIP; }

// Is the calling thread's current device a gfx950 GPU?  Queried once per
// device ordinal (the answer cannot change while the process runs).
constexpr int kMaxDevices = 64;
std::atomic<int> g_device_state[kMaxDevices];  // 0 unknown, 1 gfx950, 2 other

int device_status() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();  // leave no sticky error for the caller's next call
    return RADE_ERR_UNSUPPORTED_DEVICE;
  }
  int st = g_device_state[dev].load(std::memory_order_relaxed);
  if (st == 0) {
    hipDeviceProp_t prop;
    st = 2;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      // gcnArchName is "gfx950" followed by optional ":feature" suffixes
      const char* a = prop.gcnArchName;
      if (std::strncmp(a, "gfx950", 6) == 0 && (a[6] == '\0' || a[6] == ':')) st = 1;
    } else {
      (void)hipGetLastError();
    }
    g_device_state[dev].store(st, std::memory_order_relaxed);
  }
  return st == 1 ? RADE_OK : RADE_ERR_UNSUPPORTED_DEVICE;
}

}  // namespace

namespace rade {
KernelEvents& kernel_events(int kernel) {
  static KernelEvents table[8];
  return table[(kernel >= 0 && kernel < 8) ? kernel : 0];
}
}  // namespace rade

extern "C" {

int rade_abi_version(void) { return 8; }

int rade_device_check(void) { return device_status(); }

int rade_set_kernel_events(int kernel, void* start_event, void* stop_event) {
  if (kernel < RADE_KERNEL_PROJECT || kernel > RADE_KERNEL_PROJECT_BWD) return RADE_ERR_INVALID_ARG;
  if ((start_event == nullptr) != (stop_event == nullptr)) return RADE_ERR_INVALID_ARG;
  rade::KernelEvents& e = rade::kernel_events(kernel);
  e.start = (hipEvent_t)start_event;
  e.stop = (hipEvent_t)stop_event;
  return RADE_OK;
}

const char* rade_strerror(int code) {
  switch (code) {
    case RADE_OK: return "ok";
    case RADE_ERR_INVALID_ARG: return "invalid argument (nothing enqueued)";
    case RADE_ERR_CAPACITY: return "output capacity exceeded (the count arguments hold the required sizes)";
    case RADE_ERR_HIP: return "HIP runtime error";
    case RADE_ERR_UNSUPPORTED_DEVICE: return "unsupported device (the library runs on gfx950 GPUs only)";
    case RADE_ERR_WORKSPACE: return "workspace too small";
    case RADE_ERR_TOO_LARGE:
      return "input larger than the fixed scratch of an allocation-free entry point";
    default: return "unknown error";
  }
}

int rade_views_prepare(const rade_settings* s, rade_view* views, int32_t V,
                       int64_t* total_pixels, int64_t* total_tiles_out) {
  if (!settings_ok(s) || !views_ok(views, V)) return RADE_ERR_INVALID_ARG;
  int64_t pix = 0, tiles = 0;
  for (int i = 0; i < V; ++i) {
    views[i].tiles_x = (views[i].width + s->tile_w - 1) / s->tile_w;
    views[i].tiles_y = (views[i].height + s->tile_h - 1) / s->tile_h;
    views[i].pix_offset = pix;
    views[i].tile_offset = tiles;
    pix += (int64_t)views[i].width * views[i].height;
    tiles += (int64_t)views[i].tiles_x * views[i].tiles_y;
  }
  if (tiles >= ((int64_t)1 << 31)) return RADE_ERR_INVALID_ARG;
  if (total_pixels) *total_pixels = pix;
  if (total_tiles_out) *total_tiles_out = tiles;
  return RADE_OK;
}

int rade_project(const rade_settings* s, const rade_view* views_dev, int32_t V, int64_t N,
                 const float* means, const float* scales, const float* quats,
                 const float* opacities, const float* sh, rade_splat* splats,
                 int32_t* tiles_touched, uint32_t* bin_records, float* depth_quad,
                 void* stream) {
  if (!settings_ok(s) || !views_dev || !counts_ok(V, N)) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!means || !scales || !quats || !opacities || !sh || !splats || !tiles_touched))
    return RADE_ERR_INVALID_ARG;
  if (((reinterpret_cast<uintptr_t>(quats) | reinterpret_cast<uintptr_t>(bin_records)) & 15) != 0)
    return RADE_ERR_INVALID_ARG;
  const bool exact = s->depth_mode == RADE_DEPTH_EXACT;
  if (exact && N > 0 && (!depth_quad || (reinterpret_cast<uintptr_t>(depth_quad) & 15) != 0))
    return RADE_ERR_INVALID_ARG;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_project(*s, views_dev, V, N, means, scales, quats, opacities,
                                         sh, splats, tiles_touched, bin_records,
                                         exact ? depth_quad : nullptr, (hipStream_t)stream));
}

size_t rade_bin_sort_workspace(int32_t V, int64_t N, int64_t capacity, int64_t total_tiles) {
  (void)total_tiles;
  if (V < 1 || N < 0 || capacity < 0) return 0;
  return rade::bin_sort_workspace((int64_t)V * N, capacity);
}

int rade_bin_sort(const rade_settings* s, const rade_view* views_host,
                  const rade_view* views_dev, int32_t V, int64_t N,
                  const int32_t* tiles_touched, const uint32_t* bin_records,
                  uint32_t* pair_ids, uint32_t* tile_ranges,
                  uint64_t* keys, int64_t capacity, int64_t* n_pairs_dev,
                  int64_t* n_pairs_host, void* workspace, size_t workspace_bytes,
                  void* stream) {
  if (!settings_ok(s) || !views_ok(views_host, V) || !views_dev || !counts_ok(V, N))
    return RADE_ERR_INVALID_ARG;
  if (capacity < 0 || capacity >= ((int64_t)1 << 32)) return RADE_ERR_INVALID_ARG;
  if (!tile_ranges || !n_pairs_dev || (capacity > 0 && !pair_ids)) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!tiles_touched || !bin_records)) return RADE_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(bin_records) & 15) != 0) return RADE_ERR_INVALID_ARG;
  for (int i = 0; i < V; ++i)
    if (views_host[i].tiles_x != (views_host[i].width + s->tile_w - 1) / s->tile_w ||
        views_host[i].tiles_y != (views_host[i].height + s->tile_h - 1) / s->tile_h)
      return RADE_ERR_INVALID_ARG;  // views not prepared for this tile size
  if (!workspace || workspace_bytes < rade_bin_sort_workspace(V, N, capacity, 0))
    return RADE_ERR_WORKSPACE;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  int exceeded = 0;
  const hipError_t e = rade::launch_bin_sort(*s, views_host, views_dev, V, N, tiles_touched,
                                             bin_records, pair_ids, tile_ranges, keys, capacity,
                                             n_pairs_dev, n_pairs_host, workspace,
                                             (hipStream_t)stream, &exceeded);
  if (e != hipSuccess) return RADE_ERR_HIP;
  return exceeded ? RADE_ERR_CAPACITY : RADE_OK;
}

size_t rade_tile_order_workspace(int64_t total_tiles) {
  return total_tiles < 0 ? 0 : rade::tile_order_workspace(total_tiles);
}

int rade_tile_order(const rade_settings* s, const rade_view* views_host, int32_t V,
                    const uint32_t* tile_ranges, uint32_t* tile_order, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (!settings_ok(s) || !views_ok(views_host, V) || !tile_ranges || !tile_order)
    return RADE_ERR_INVALID_ARG;
  const int64_t tiles = total_tiles(views_host, V);
  if (!workspace || workspace_bytes < rade_tile_order_workspace(tiles)) return RADE_ERR_WORKSPACE;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_tile_order(tile_ranges, tiles, tile_order, workspace,
                                            (hipStream_t)stream));
}

size_t rade_normal_consistency_workspace(int64_t total_pixels) {
  return total_pixels < 0 ? 0 : rade::normal_consistency_workspace(total_pixels);
}

namespace {
// Pixel total of prepared views (-1 if pix_offset does not follow the order).
int64_t prepared_pixels(const rade_view* views_host, int32_t V) {
  int64_t total = 0;
  for (int i = 0; i < V; ++i) {
    if (views_host[i].pix_offset != total) return -1;
    total += (int64_t)views_host[i].width * views_host[i].height;
  }
  return total;
}
}  // namespace

int rade_l1_color_grad(const rade_view* views_host, const rade_view* views_dev, int32_t V,
                       const float* color, const float* target, float weight, float* d_color,
                       void* stream) {
  if (!views_ok(views_host, V) || !views_dev || !color || !target || !d_color ||
      !std::isfinite(weight))
    return RADE_ERR_INVALID_ARG;
  const int64_t total = prepared_pixels(views_host, V);
  if (total < 0) return RADE_ERR_INVALID_ARG;  // not prepared
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_l1_color_grad(views_dev, V, total, color, target,
                                               (double)weight, d_color, (hipStream_t)stream));
}

int rade_normal_consistency(const rade_view* views_host, const rade_view* views_dev, int32_t V,
                            const float* depth, const float* normal, const float* alpha,
                            float weight, float* loss, float* d_depth, float* d_normal,
                            float* d_alpha, int32_t accumulate, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!views_ok(views_host, V) || !views_dev || !depth || !normal || !alpha || !loss ||
      !d_depth || !d_normal || !d_alpha || !std::isfinite(weight))
    return RADE_ERR_INVALID_ARG;
  int64_t total = 0;
  for (int i = 0; i < V; ++i) {
    if (views_host[i].pix_offset != total) return RADE_ERR_INVALID_ARG;  // not prepared
    total += (int64_t)views_host[i].width * views_host[i].height;
  }
  if (!workspace || workspace_bytes < rade_normal_consistency_workspace(total))
    return RADE_ERR_WORKSPACE;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_normal_consistency(views_host, views_dev, V, total, depth,
                                                    normal, alpha,
                                                    weight, loss, d_depth, d_normal, d_alpha,
                                                    accumulate != 0, workspace,
                                                    (hipStream_t)stream));
}

int rade_normal_consistency_noalloc(const rade_view* views_host, const rade_view* views_dev,
                                    int32_t V, const float* depth, const float* normal,
                                    const float* alpha, float weight, float* loss,
                                    float* d_depth, float* d_normal, float* d_alpha,
                                    int32_t accumulate, void* stream) {
  if (!views_ok(views_host, V) || !views_dev || !depth || !normal || !alpha || !loss ||
      !d_depth || !d_normal || !d_alpha || !std::isfinite(weight))
    return RADE_ERR_INVALID_ARG;
  const int64_t total = prepared_pixels(views_host, V);
  if (total < 0) return RADE_ERR_INVALID_ARG;  // not prepared
  if (rade::normal_consistency_blocks(views_host, V) > RADE_NC_NOALLOC_MAX_BLOCKS)
    return RADE_ERR_TOO_LARGE;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  void* ws = nullptr;
  if (rade::nc_scratch_address(&ws) != hipSuccess) {
    (void)hipGetLastError();
    return RADE_ERR_HIP;
  }
  return hip_status(rade::launch_normal_consistency(views_host, views_dev, V, total, depth,
                                                    normal, alpha, weight, loss, d_depth,
                                                    d_normal, d_alpha, accumulate != 0, ws,
                                                    (hipStream_t)stream));
}

int rade_render_fwd(const rade_settings* s, const rade_view* views_host,
                    const rade_view* views_dev, int32_t V, int64_t N, const rade_splat* splats,
                    const uint32_t* pair_ids, const uint32_t* tile_ranges,
                    uint32_t* tile_order, float* color,
                    float* depth, float* normal, float* alpha, float* t_final, int32_t* last,
                    int32_t* median, int32_t* count, int32_t* evals, float* distortion,
                    const float* depth_quad, uint64_t* lane_masks, void* stream) {
  if (!settings_ok(s) || !views_ok(views_host, V) || !views_dev || !counts_ok(V, N))
    return RADE_ERR_INVALID_ARG;
  if (!tile_ranges || !color || !depth || !normal || !alpha || !t_final || !last || !median)
    return RADE_ERR_INVALID_ARG;
  const bool exact = s->depth_mode == RADE_DEPTH_EXACT;
  if (exact && N > 0 && (!depth_quad || (reinterpret_cast<uintptr_t>(depth_quad) & 15) != 0))
    return RADE_ERR_INVALID_ARG;
  // tuned wave shapes / batches exist for the plain forward only
  if (!rade::render_shape_is_default(s->tile_w, s->tile_h, s->wave_w, s->batch, s->lane_masks) &&
      (exact || distortion || count || evals))
    return RADE_ERR_INVALID_ARG;
  if (s->schedule != RADE_SCHEDULE_TILE && !tile_order) return RADE_ERR_INVALID_ARG;
  if (N > 0 && !splats) return RADE_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(lane_masks) & 15) != 0) return RADE_ERR_INVALID_ARG;
  const int64_t tiles = total_tiles(views_host, V);
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  const bool keep_masks =
      rade::lane_masks_per_pair(s->tile_w, s->tile_h, s->wave_w, s->batch, s->lane_masks) > 0;
  return hip_status(rade::launch_render_fwd(*s, views_dev, V, N, tiles, splats, pair_ids,
                                            tile_ranges, tile_order, color, depth, normal, alpha,
                                            t_final, last, median, count, evals, distortion,
                                            exact ? depth_quad : nullptr,
                                            keep_masks ? lane_masks : nullptr,
                                            (hipStream_t)stream));
}

size_t rade_lane_mask_bytes(const rade_settings* s, int64_t n_pairs) {
  if (!settings_ok(s) || n_pairs < 0) return 0;
  const int w = rade::lane_masks_per_pair(s->tile_w, s->tile_h, s->wave_w, s->batch, s->lane_masks);
  return (size_t)n_pairs * (size_t)w * sizeof(uint64_t);
}

size_t rade_render_bwd_workspace(const rade_settings* s, int32_t V, int64_t N, int recompute) {
  (void)s;
  if (V < 1 || N < 0) return 0;
  const size_t VN = (size_t)V * (size_t)N;
  size_t bytes = ((VN * 16 * sizeof(float)) + 255) & ~size_t(255);  // per-(view, Gaussian) grads
  if (recompute)
    bytes += ((VN * sizeof(rade_splat) + 255) & ~size_t(255)) + ((VN * 4 + 255) & ~size_t(255));
  return bytes;
}

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
                    float* d_sh, void* workspace, size_t workspace_bytes, void* stream) {
  if (!settings_ok(s) || !views_ok(views_host, V) || !views_dev || !counts_ok(V, N))
    return RADE_ERR_INVALID_ARG;
  if (!tile_ranges || !t_final || !last || !median) return RADE_ERR_INVALID_ARG;
  if (s->depth_mode != RADE_DEPTH_AFFINE) return RADE_ERR_INVALID_ARG;  // forward-only variant
  if (d_distortion && (!depth || !alpha)) return RADE_ERR_INVALID_ARG;
  if (d_distortion && !rade::render_shape_is_default(s->tile_w, s->tile_h, s->wave_w, s->batch, s->lane_masks))
    return RADE_ERR_INVALID_ARG;  // tuned shapes exist for the plain backward only
  if (s->schedule != RADE_SCHEDULE_TILE && !tile_order) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!means || !scales || !quats || !opacities || !sh || !d_means || !d_scales ||
                !d_quats || !d_opacities || !d_sh))
    return RADE_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(quats) & 15) != 0 ||
      (reinterpret_cast<uintptr_t>(d_quats) & 15) != 0 ||
      (reinterpret_cast<uintptr_t>(lane_masks) & 15) != 0)
    return RADE_ERR_INVALID_ARG;
  const int recompute = splats == nullptr ? 1 : 0;
  if (!workspace || workspace_bytes < rade_render_bwd_workspace(s, V, N, recompute))
    return RADE_ERR_WORKSPACE;
  // the per-(view, Gaussian) gradient records move in 16-byte words
  if ((reinterpret_cast<uintptr_t>(workspace) & 15) != 0) return RADE_ERR_INVALID_ARG;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  const hipStream_t st = (hipStream_t)stream;
  const size_t VN = (size_t)V * (size_t)N;
  char* w = static_cast<char*>(workspace);
  float* gsplat = reinterpret_cast<float*>(w);
  if (recompute && N > 0) {
    const size_t g_bytes = ((VN * 16 * sizeof(float)) + 255) & ~size_t(255);
    rade_splat* rs = reinterpret_cast<rade_splat*>(w + g_bytes);
    int32_t* tt = reinterpret_cast<int32_t*>(
        w + g_bytes + (((VN * sizeof(rade_splat)) + 255) & ~size_t(255)));
    const hipError_t e = rade::launch_project(*s, views_dev, V, N, means, scales, quats,
                                              opacities, sh, rs, tt, nullptr, nullptr, st);
    if (e != hipSuccess) return RADE_ERR_HIP;
    splats = rs;
  }
  const int64_t tiles = total_tiles(views_host, V);
  hipError_t e = rade::launch_render_bwd(*s, views_dev, V, N, tiles, splats, pair_ids,
                                         tile_ranges, tile_order, t_final, last, median, d_color,
                                         d_depth, d_normal, d_alpha, d_distortion, depth, alpha,
                                         gsplat,
                                         rade::lane_masks_per_pair(s->tile_w, s->tile_h,
                                                                   s->wave_w, s->batch,
                                                                   s->lane_masks) > 0
                                             ? lane_masks
                                             : nullptr,
                                         st);
  if (e != hipSuccess) return RADE_ERR_HIP;
  e = rade::launch_project_bwd(*s, views_dev, V, N, means, scales, quats, opacities, sh, gsplat,
                               d_means, d_scales, d_quats, d_opacities, d_sh, st);
  return hip_status(e);
}

int rade_filter3d_var(const rade_settings* s, const rade_view* views_dev, int32_t V, int64_t N,
                      const float* means, float scale, float margin, float* var, void* stream) {
  if (!s || !views_dev || !counts_ok(V, N)) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!means || !var)) return RADE_ERR_INVALID_ARG;
  if (!(scale >= 0.0f) || !(margin >= 0.0f)) return RADE_ERR_INVALID_ARG;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_filter3d_var(views_dev, V, N, means, s->near_plane, scale,
                                              margin, var, (hipStream_t)stream));
}

int rade_filter3d_apply(int64_t N, const float* scales, const float* opacities, const float* var,
                        float* scales_out, float* opacities_out, void* stream) {
  if (N < 0) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!scales || !opacities || !var || !scales_out || !opacities_out))
    return RADE_ERR_INVALID_ARG;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_filter3d_apply(N, scales, opacities, var, scales_out,
                                                opacities_out, (hipStream_t)stream));
}

int rade_filter3d_apply_bwd(int64_t N, const float* scales, const float* opacities,
                            const float* var, const float* d_scales_out,
                            const float* d_opacities_out, float* d_scales, float* d_opacities,
                            void* stream) {
  if (N < 0) return RADE_ERR_INVALID_ARG;
  if (N > 0 && (!scales || !opacities || !var || !d_scales_out || !d_opacities_out ||
                !d_scales || !d_opacities))
    return RADE_ERR_INVALID_ARG;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_filter3d_apply_bwd(N, scales, opacities, var, d_scales_out,
                                                    d_opacities_out, d_scales, d_opacities,
                                                    (hipStream_t)stream));
}

int rade_tsdf_fuse(const rade_settings* s, const rade_view* views_host,
                   const rade_view* views_dev, int32_t V, const float* depth,
                   const double* origin, double voxel, int32_t nx, int32_t ny, int32_t nz,
                   float trunc, float* tsdf, float* weight, void* stream) {
  if (!s || !views_ok(views_host, V) || !views_dev || !origin) return RADE_ERR_INVALID_ARG;
  if (!(voxel > 0.0) || !(trunc > 0.0f) || nx < 1 || ny < 1 || nz < 1) return RADE_ERR_INVALID_ARG;
  if ((int64_t)nx * ny * nz > (int64_t)UINT32_MAX) return RADE_ERR_INVALID_ARG;
  if (!std::isfinite(origin[0]) || !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
    return RADE_ERR_INVALID_ARG;
  if (!depth || !tsdf || !weight) return RADE_ERR_INVALID_ARG;
  int64_t total = 0;
  for (int i = 0; i < V; ++i) {
    if (views_host[i].pix_offset != total) return RADE_ERR_INVALID_ARG;  // not prepared
    total += (int64_t)views_host[i].width * views_host[i].height;
  }
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  return hip_status(rade::launch_tsdf_fuse(views_dev, V, depth, origin, voxel, nx, ny, nz,
                                           s->near_plane, trunc, tsdf, weight,
                                           (hipStream_t)stream));
}

size_t rade_marching_cubes_workspace(int32_t nx, int32_t ny, int32_t nz) {
  if (!grid_ok(nx, ny, nz)) return 0;
  return rade::marching_cubes_workspace(nx, ny, nz);
}

int rade_marching_cubes(const float* tsdf, const float* weight, int32_t nx, int32_t ny,
                        int32_t nz, const double* origin, double voxel, float iso,
                        void* workspace, size_t workspace_bytes, float* verts, int64_t max_verts,
                        uint32_t* tris, int64_t max_tris, int64_t* n_verts, int64_t* n_tris,
                        void* stream) {
  if (!grid_ok(nx, ny, nz) || !tsdf || !weight || !origin || !n_verts || !n_tris)
    return RADE_ERR_INVALID_ARG;
  if (!(voxel > 0.0) || !std::isfinite(voxel) || !std::isfinite(iso)) return RADE_ERR_INVALID_ARG;
  if (!std::isfinite(origin[0]) || !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
    return RADE_ERR_INVALID_ARG;
  if (max_verts < 0 || max_tris < 0 || (max_verts > 0 && !verts) || (max_tris > 0 && !tris))
    return RADE_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < rade::marching_cubes_workspace(nx, ny, nz))
    return RADE_ERR_WORKSPACE;
  if (const int dv = device_status(); dv != RADE_OK) return dv;
  const hipStream_t st = (hipStream_t)stream;
  const uint32_t* nv_dev = nullptr;
  const uint64_t* nt_dev = nullptr;
  hipError_t e = rade::launch_marching_cubes(tsdf, weight, nx, ny, nz, origin, voxel, iso,
                                             workspace, verts, max_verts, tris, max_tris, &nv_dev,
                                             &nt_dev, st);
  uint32_t nv = 0;
  uint64_t nt = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nv, nv_dev, sizeof(nv), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nt, nt_dev, sizeof(nt), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return RADE_ERR_HIP;
  *n_verts = (int64_t)nv;
  *n_tris = (int64_t)nt;
  return ((int64_t)nv > max_verts || (int64_t)nt > max_tris) ? RADE_ERR_CAPACITY : RADE_OK;
}

int rade_marching_cubes_table(uint8_t* ntri, uint8_t* tri) {
  if (!ntri || !tri) return RADE_ERR_INVALID_ARG;
  rade::marching_cubes_table(ntri, tri);
  return RADE_OK;
}

}  // extern "C"
