// rt_internal.hpp - host-side types shared by the C ABI and the launch
// wrappers of each kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/rt.h"
#include "trace.hpp"

// Library-owned scene: one device allocation holding the packed arrays the
// kernels read, a staging area for host uploads, and the per-workgroup
// gradient partials of the adjoint.
struct rt_scene_s {
  int device = 0;
  int n_spheres = 0, n_planes = 0, n_lights = 0, spec_model = 0;
  float ambient = 0, spec_strength = 0, t_min = 0, bg[3] = {0, 0, 0};
  void* buffer = nullptr;  // single hipMalloc
  size_t bytes = 0;
  float4* geom = nullptr;  // [n4+kGroup] cx cy cz r^2 (padding spheres: r^2 = -1)
  float2* rad = nullptr;   // [N]   r, 1/r
  float4* mat = nullptr;   // [N+P] albedo, kr
  float* shine = nullptr;  // [N+P]
  float4* pgeom = nullptr; // [P]
  float4* light = nullptr; // [L]
  float4* eye_cone = nullptr;    // [n4+kGroup] rebuilt for the camera of each call
  float4* light_cone = nullptr;  // [L*n4 + kGroup]  rows of n4, rebuilt by every upload/update
  float4* eye_oc = nullptr;      // [n4+kGroup] eye - centre, r^2, with the eye cones
  float4* light_oc = nullptr;    // [L*n4 + kGroup] light - centre, r^2, with the light cones
  float* staging = nullptr;     // raw copy of host desc arrays
  size_t staging_floats = 0;
  float2* soft_table = nullptr; // [RT_MAX_SAMPLES] shadow sample points of the last soft render
  float* partials = nullptr;    // adjoint partials [kAdjointBlocks][grad_stride]
  int grad_stride = 0;          // 7N + 4L (padded)
  float4* sky = nullptr;        // own hipMalloc: [sky_h][sky_w] rgb + unused, or none
  int sky_w = 0, sky_h = 0;
  // tile schedule of the hard-shadow render (schedule.hip): the area of
  // kSchedBytes at `sched` (layout in trace.hpp)
  uint8_t* sched = nullptr;
  int hist_set = 0;                // histogram set holding the last record
  int hist_W = 0, hist_H = 0;      // image of the recorded duration bins (0: none)
  int hist_kind = 0;               // kernel that recorded them (kSchedHard, kSchedSoft)
  int order_W = 0, order_H = 0;    // image the last prepare ordered (0: none)
  int rec_W = 0, rec_H = 0;        // image the next render may record (other set zeroed)
  int sched_kind = 0;              // kernel the last prepare prepared for

  rtk::SceneDev view() const {
    rtk::SceneDev s;
    s.geom = geom; s.rad = rad; s.mat = mat; s.shine = shine; s.pgeom = pgeom; s.light = light;
    s.eye_cone = eye_cone; s.light_cone = light_cone;
    s.eye_oc = eye_oc; s.light_oc = light_oc;
    s.n4 = rtk::pad_spheres(n_spheres);
    s.n_spheres = n_spheres; s.n_planes = n_planes; s.n_lights = n_lights;
    s.spec_model = spec_model;
    s.ambient = ambient; s.spec_strength = spec_strength; s.t_min = t_min;
    s.bg_r = bg[0]; s.bg_g = bg[1]; s.bg_b = bg[2];
    s.sky = sky; s.sky_w = sky_w; s.sky_h = sky_h;
    s.sched = sched;
    s.sched_mode = 0;
    return s;
  }
};

namespace rtk {

// Render launches: one wave per workgroup, an 8 x 8 pixel tile per wave (the
// soft-shadow render of smaller images: two waves per tile, below).
constexpr int kRenderTile = 8;
constexpr int kRenderThreads = 64;
// Soft-shadow renders of images up to kSoftSplitMaxTiles tiles share each
// pixel's samples between two neighbouring lanes (two waves per tile): such
// frames are set by the latency of their slowest tiles, which this halves;
// larger images are set by throughput, which the shared paths would cost.
constexpr int kSoftSplitMaxTiles = 40000;
constexpr int kSoftMaxThreads = 2 * kRenderThreads;
inline dim3 render_grid(int W, int H) {
  return dim3((W + kRenderTile - 1) / kRenderTile, (H + kRenderTile - 1) / kRenderTile);
}
inline int soft_parts(int W, int H) {
  const dim3 g = render_grid(W, H);
  return (int64_t)g.x * g.y <= kSoftSplitMaxTiles ? 2 : 1;
}

// Tile scheduling of the hard-shadow render (schedule.hip): images of at
// least kSchedMinTiles tiles (fewer all start at once) and at most
// kSchedMaxTiles (the scene's tables).
constexpr int kSchedMinTiles = 4096;
// Kernels whose tile durations are recorded apart (a record is used only by
// the same kernel): hard-shadow and soft-shadow renders.
constexpr int kSchedHard = 0, kSchedSoft = 1;

// Workgroups of the persistent adjoint grid (one partial-gradient slot each).
constexpr int kAdjointBlocks = 1024;

void set_error(const std::string& msg);
rt_status fail(rt_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
rt_status hip_fail(hipError_t e, const char* what);
CameraDev camera_dev(const rt_camera& cam, int W, int H);
bool finite_all(const float* a, int64_t n);
rt_status validate_camera(const rt_camera* cam, int32_t W, int32_t H, int32_t depth);

// Raw (desc-layout) arrays the pack kernel reads.
struct RawScene {
  const float* sphere_geom;
  const float* sphere_mat;
  const float* sphere_shine;
  const float* plane_geom;
  const float* plane_mat;
  const float* plane_shine;
  const float* light;
};

hipError_t launch_pack(const rt_scene_s& sc, const RawScene& raw, hipStream_t stream);

// Repack a device skybox [h][w][3] into the scene's float4 texels.
hipError_t launch_sky_pack(const float* rgb, float4* sky, int texels, hipStream_t stream);

// Cones of every sphere seen from the camera's eye, into sc.eye_cone.
hipError_t launch_eye_cones(const rt_scene_s& sc, const CameraDev& c, hipStream_t stream);
// The eye cones and, with `schedule` (only where schedule_applies), the
// scene's tile order for a render of c.W x c.H from the durations the last
// render of that size recorded (*ordered: an order was written), and the
// zeroed histogram the following render records into.
hipError_t launch_prepare(rt_scene_s& sc, const CameraDev& c, bool schedule, int kind,
                          bool* ordered, hipStream_t stream);
bool schedule_applies(const rt_scene_s& sc, int W, int H);
// sched_mode: the tile schedule's mode bits (0: row order, no record).
hipError_t launch_render_soft(const rt_scene_s& sc, const CameraDev& c, int depth, int samples,
                              float radius, float* rgb, int32_t* ids, bool prefilter,
                              int sched_mode, hipStream_t stream);

// The render kernels' entry addresses, for graph nodes built by hand: the
// hard-shadow render without records, and the soft-shadow render, with or
// without the skybox lookup and the wave bounds; the sample-table kernel.
// Their parameters are those of the kernels in render.hip.
const void* render_kernel_fn(bool sky, bool prefilter);
const void* render_soft_kernel_fn(bool sky, bool prefilter);
const void* sample_table_kernel_fn();

hipError_t launch_render(const SceneDev& s, const CameraDev& c, int depth, float* rgb,
                         int32_t* ids, int32_t* rec_ids, uint8_t* rec_lit, bool prefilter,
                         hipStream_t stream);

hipError_t launch_counts(const SceneDev& s, const CameraDev& c, int depth,
                         unsigned long long* counts, bool prefilter, hipStream_t stream);

// Whether the adjoint's per-wave LDS accumulators of a scene with n_spheres
// (and up to RT_MAX_LIGHTS lights) fit a workgroup on `device`, and the
// largest such sphere count.
bool adjoint_supported(int n_spheres, int device);
int adjoint_max_spheres(int device);

// Launch shape of a batch: wave64s per workgroup, pixel columns per wave
// (columns x rows = 64) and persistent workgroups.
struct TunedShape {
  int waves;
  int wave_w;
  int grid;
};
// One of the shapes the batch autotuner times.
bool tuned_shape_valid(const TunedShape& s);
// Autotune cache (memory, then the JSON file): true and *out on a hit.
bool tune_cache_get(const std::string& key, TunedShape* out);
// Stores an entry in memory and in the file; false if the file could not be
// written (the memory entry is kept) or the shape is not valid.
bool tune_cache_put(const std::string& key, const TunedShape& s);
void tune_cache_forget_memory();

// Largest partials of rt_render_backward_static, in floats (16 MiB per GPU).
constexpr size_t kStaticScratchFloats = RT_STATIC_SCRATCH_BYTES / sizeof(float);
// Floats of partials a backward launch of this scene and image writes.
size_t backward_partial_floats(const rt_scene_s& sc, const CameraDev& c);
// Device address of the static partials array on `device` (looked up once per
// device, with that device current).
hipError_t static_scratch(int device, float** out);

// partials: [blocks][grad_stride] floats of device memory (the scene's own),
// every row written before it is read.
hipError_t launch_backward(const rt_scene_s& sc, const CameraDev& c, int depth,
                           const float* grad_rgb, const int32_t* rec_ids, const uint8_t* rec_lit,
                           const rt_grads& g, float* partials, hipStream_t stream);

// Device ordinals the per-device caches of the library hold.
constexpr int kMaxDevices = 64;

}  // namespace rtk
