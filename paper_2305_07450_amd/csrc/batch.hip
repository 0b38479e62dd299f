// batch.hip - many scenes of uneven size in one persistent launch.
//
// The host flattens every image into pixel tiles and orders the tile queue by
// estimated cost, largest first (LPT: a tile's cost is taken as pixels x
// segments x primitives x (1 + lights), the brute-force work of Sections
// 3.4-3.7).  A persistent grid of workgroups pulls tiles from the queue with
// one atomic counter per launch; each workgroup reads the job descriptor of
// its tile through scalar loads and renders it with exactly the per-pixel code
// of rt_render (trace.hpp), so every image is bit-identical to a single
// rt_render of the same scene.  The counter is reset by a one-lane kernel in
// the same stream (no memset node), and both kernels are captured once into a
// HIP graph that rt_batch_launch replays.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <type_traits>
#include <mutex>
#include <new>
#include <string.h>
#include <string>
#include <vector>

#include "rt_internal.hpp"

namespace rtk {

struct BatchJob {
  SceneDev s;
  CameraDev c;
  int depth;
  int tiles_x;
  float* rgb;
};
static_assert(sizeof(BatchJob) % 4 == 0, "descriptor is copied in 32-bit words");

// One queue entry: job index and tile index within the job.
struct TileRef {
  int job;
  int tile;
};

using Shape = TunedShape;

__global__ void reset_counter_kernel(unsigned int* counter) { *counter = 0u; }

// Eye cones and eye - centre table of every job's spheres (grid.y = job), into
// the batch's own tables (the job's eye_cone and eye_oc point there), with the
// arithmetic of the single-image eye-cone kernel.
__global__ void batch_cone_kernel(const BatchJob* __restrict__ jobs, float4* const* cones) {
  const BatchJob& j = jobs[blockIdx.y];
  float4* oc = const_cast<float4*>(j.s.eye_oc);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < j.s.n_spheres) {
    float4 g = j.s.geom[i];
    cones[blockIdx.y][i] = sphere_cone(j.c.ex, j.c.ey, j.c.ez, g.x, g.y, g.z, j.s.rad[i].x);
    oc[i] = make_float4(j.c.ex - g.x, j.c.ey - g.y, j.c.ez - g.z, g.w);
  } else if (i < j.s.n4 + kGroup) {
    cones[blockIdx.y][i] = make_float4(0.0f, 0.0f, 0.0f, kPadConeW);
    oc[i] = make_float4(0.0f, 0.0f, 0.0f, kPadR2);
  }
}

// With Cnt = Count the same launch also adds the work counters of every path
// (trace.hpp) to counts[kNumCounts]; the render instantiation (NoCount) has
// no counter code at all.
template <class Bg, class Cnt>
__global__ __launch_bounds__(256) void batch_kernel(const BatchJob* __restrict__ jobs,
                                                     const TileRef* __restrict__ queue,
                                                     int n_tiles, unsigned int* counter,
                                                     int wave_w,
                                                     unsigned long long* __restrict__ counts) {
  __shared__ unsigned int s_tile;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const int wave_h = 64 / wave_w;
  const int tile_w = wave_w, tile_h = wave_h * waves;
  Cnt cnt;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    // tickets stay unsigned: each workgroup takes one past the last tile, so
    // they reach n_tiles + grid - 1, which a signed cast could turn negative
    // for a queue near 2^31 tiles
    const unsigned int t = s_tile;
    __syncthreads();   // every lane has read s_tile before it is written again
    if (t >= (unsigned int)n_tiles) break;   // uniform: the whole workgroup leaves together
    const TileRef ref = queue[t];
    const BatchJob* jp = jobs + __builtin_amdgcn_readfirstlane(ref.job);
    // copy the descriptor word by word through the constant address space
    // (uniform address -> scalar loads)
    BatchJob job;
    {
      const RT_CONSTANT uint32_t* src = (const RT_CONSTANT uint32_t*)jp;
      uint32_t* dst = (uint32_t*)&job;
#pragma unroll
      for (int i = 0; i < (int)(sizeof(BatchJob) / 4); ++i) dst[i] = src[i];
    }
    const int tile = __builtin_amdgcn_readfirstlane(ref.tile);
    const int tx = tile % job.tiles_x, ty = tile / job.tiles_x;
    const int x = tx * tile_w + (lane % wave_w);
    const int y = ty * tile_h + wave * wave_h + (lane / wave_w);
    // lanes outside the image run along without output (see render_kernel)
    const bool live = x < job.c.W && y < job.c.H;
    if (wave_any(live)) {
      float cr, cg, cb;
      int prim;
      NoRecords sink;
      trace_path<NoRecords, Cnt&, true, HardShadows, Bg>(
          job.s, primary_ray(job.c, live ? x : job.c.W - 1, live ? y : job.c.H - 1), job.depth,
          live, cr, cg, cb, prim, sink, cnt);
      if (live) {
        const int64_t pix = (int64_t)y * job.c.W + x;
        job.rgb[3 * pix + 0] = cr;
        job.rgb[3 * pix + 1] = cg;
        job.rgb[3 * pix + 2] = cb;
      }
    }
  }
  if constexpr (std::is_same<Cnt, Count>::value) {
    // a persistent wave renders many tiles: sum its lanes in 64 bits
    for (int j = 0; j < kNumCounts; ++j) {
      long long v = cnt.c[j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) atomicAdd(counts + j, (unsigned long long)v);
    }
  }
}

}  // namespace rtk

using namespace rtk;

struct rt_batch_s {
  int device = 0;
  int n = 0;
  int n_tiles = 0;
  Shape shape{};
  BatchJob* jobs = nullptr;     // device
  TileRef* queue = nullptr;     // device
  float4* cones = nullptr;      // device: eye cones of every job's spheres, then their
                                // eye - centre tables (the same offsets past the cones)
  float4** cone_ptr = nullptr;  // device: start of each job's cones
  int max_spheres = 0;
  unsigned int* counter = nullptr;
  std::vector<BatchJob> host_jobs;
  std::vector<const rt_scene_s*> scenes;  // the skybox each job was built with is in host_jobs
  std::vector<double> job_cost;  // per tile
  bool any_sky = false;          // some job's scene has a skybox
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string tune_key;          // autotune cache key of this batch
};

namespace {

rt_status err(rt_status st, const std::string& m) {
  set_error(m);
  return st;
}

// Build the LPT-ordered queue for a wave shape.
std::vector<TileRef> build_queue(rt_batch_s* b, int wave_w, int waves) {
  const int tile_w = wave_w, tile_h = (64 / wave_w) * waves;
  std::vector<int> order(b->n);
  for (int i = 0; i < b->n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->job_cost[a] > b->job_cost[c]; });
  std::vector<TileRef> q;
  for (int j : order) {
    BatchJob& job = b->host_jobs[j];
    job.tiles_x = (job.c.W + tile_w - 1) / tile_w;
    const int tiles_y = (job.c.H + tile_h - 1) / tile_h;
    for (int t = 0; t < job.tiles_x * tiles_y; ++t) q.push_back(TileRef{j, t});
  }
  return q;
}

hipError_t upload_shape(rt_batch_s* b, const Shape& sh, hipStream_t stream) {
  std::vector<TileRef> q = build_queue(b, sh.wave_w, sh.waves);
  hipError_t e = hipMemcpyAsync(b->jobs, b->host_jobs.data(), sizeof(BatchJob) * b->n,
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->queue, q.data(), sizeof(TileRef) * q.size(), hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  b->n_tiles = (int)q.size();
  b->shape = sh;
  return e;
}

hipError_t launch_batch(rt_batch_s* b, hipStream_t stream,
                        unsigned long long* counts = nullptr) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, b->counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (b->max_spheres > 0) {
    hipLaunchKernelGGL(batch_cone_kernel, dim3((b->max_spheres + 255) / 256, b->n), dim3(256), 0,
                       stream, (const BatchJob*)b->jobs, (float4* const*)b->cone_ptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  auto kern = b->any_sky ? batch_kernel<SkyBackground, NoCount>
                         : batch_kernel<PlainBackground, NoCount>;
  if (counts)
    kern = b->any_sky ? batch_kernel<SkyBackground, Count> : batch_kernel<PlainBackground, Count>;
  hipLaunchKernelGGL(kern, dim3(b->shape.grid), dim3(64 * b->shape.waves), 0, stream, b->jobs,
                     b->queue, b->n_tiles, b->counter, b->shape.wave_w, counts);
  return hipGetLastError();
}

// Autotune cache key: the device's architecture and compute-unit count, then
// every job's size, depth, sphere and light count and skybox flag.
std::string signature(const rt_batch_s* b, const std::string& arch, int cus) {
  std::string s = arch + ":" + std::to_string(cus) + "cu:" + std::to_string(b->n);
  for (const BatchJob& j : b->host_jobs)
    s += ":" + std::to_string(j.c.W) + "x" + std::to_string(j.c.H) + "d" +
         std::to_string(j.depth) + "n" + std::to_string(j.s.n_spheres) + "l" +
         std::to_string(j.s.n_lights) + (j.s.sky ? "s" : "");
  return s;
}

// Time each candidate shape with events (median of 3 direct launches).
rt_status autotune(rt_batch_s* b, int cus, hipStream_t stream, Shape* best) {
  const int wave_ws[] = {8, 16, 64};
  const int wavess[] = {1, 2, 4};
  const int grid_mult[] = {2, 4, 8};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return err(RT_ERR_DEVICE, "autotune: event creation failed");
  float best_ms = 1e30f;
  rt_status st = RT_OK;
  for (int ww : wave_ws)
    for (int wv : wavess)
      for (int gm : grid_mult) {
        Shape sh{wv, ww, cus * gm * (4 / wv)};
        hipError_t e = upload_shape(b, sh, stream);
        float times[3];
        for (int r = 0; r < 4 && e == hipSuccess; ++r) {
          e = hipEventRecord(e0, stream);
          if (e == hipSuccess) e = launch_batch(b, stream);
          if (e == hipSuccess) e = hipEventRecord(e1, stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess && r > 0) e = hipEventElapsedTime(&times[r - 1], e0, e1);
        }
        if (e != hipSuccess) {
          st = hip_fail(e, "autotune launch");
          goto done;
        }
        std::sort(times, times + 3);
        if (times[1] < best_ms) {
          best_ms = times[1];
          *best = sh;
        }
      }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Queue capacity for one image: the most tiles any candidate shape makes
// (one-wave tiles).
size_t most_tiles(int W, int H) {
  size_t most = 0;
  for (int ww : {8, 16, 64}) {
    const int wh = 64 / ww;
    most = std::max(most, (size_t)((W + ww - 1) / ww) * (size_t)((H + wh - 1) / wh));
  }
  return most;
}

void free_batch(rt_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->jobs) (void)hipFree(b->jobs);
  if (b->queue) (void)hipFree(b->queue);
  if (b->counter) (void)hipFree(b->counter);
  if (b->cones) (void)hipFree(b->cones);
  if (b->cone_ptr) (void)hipFree(b->cone_ptr);
  delete b;
}

// Frees a batch under construction unless released: host allocations below
// may throw, and the exported call turns that into an error code.
struct BatchGuard {
  rt_batch_s* b = nullptr;
  ~BatchGuard() { free_batch(b); }
};

rt_status batch_create(int32_t n, const rt_scene* scenes, const rt_camera* cams,
                       const int32_t* W, const int32_t* H, const int32_t* depth,
                       float* const* rgb_out, int32_t autotune_flag, void* stream_v,
                       rt_batch* out) {
  if (!out) return err(RT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || n > RT_MAX_BATCH)
    return err(RT_ERR_INVALID_ARG, "batch size " + std::to_string(n) + " outside [1, " +
                                       std::to_string(RT_MAX_BATCH) + "]");
  if (!scenes || !cams || !W || !H || !depth || !rgb_out)
    return err(RT_ERR_INVALID_ARG, "a batch array is NULL");
  for (int i = 0; i < n; ++i) {
    if (!scenes[i]) return err(RT_ERR_INVALID_ARG, "scene " + std::to_string(i) + " is NULL");
    if (!rgb_out[i]) return err(RT_ERR_INVALID_ARG, "rgb_out " + std::to_string(i) + " is NULL");
    const rt_camera& c = cams[i];
    float v[6] = {c.eye[0], c.eye[1], c.eye[2], c.yaw_deg, c.pitch_deg, c.fov_deg};
    for (float f : v)
      if (!isfinite(f)) return err(RT_ERR_INVALID_ARG, "camera " + std::to_string(i) + " is not finite");
    if (!(c.fov_deg > 0.0f && c.fov_deg < 180.0f))
      return err(RT_ERR_INVALID_ARG, "camera " + std::to_string(i) + " fov outside (0, 180)");
    if (W[i] <= 0 || H[i] <= 0 || W[i] > RT_MAX_DIM || H[i] > RT_MAX_DIM)
      return err(RT_ERR_INVALID_ARG, "image " + std::to_string(i) + " size out of range");
    if (depth[i] < 0 || depth[i] > RT_MAX_DEPTH)
      return err(RT_ERR_INVALID_ARG, "depth " + std::to_string(i) + " outside [0, 8]");
  }
  // the persistent kernel numbers the queue's tiles with 32-bit integers
  size_t max_tiles = 0;
  for (int i = 0; i < n; ++i) max_tiles += most_tiles(W[i], H[i]);
  if (max_tiles > (size_t)INT32_MAX)
    return err(RT_ERR_INVALID_ARG, "the batch makes " + std::to_string(max_tiles) +
                                       " tiles, more than 2^31 - 1");
  for (int i = 1; i < n; ++i)
    if (scenes[i]->device != scenes[0]->device)
      return err(RT_ERR_INVALID_ARG, "scenes live on different devices");
  hipStream_t stream = (hipStream_t)stream_v;
  rt_batch_s* b = new (std::nothrow) rt_batch_s();
  if (!b) return err(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
  BatchGuard guard{b};
  b->n = n;
  b->device = scenes[0]->device;
  for (int i = 0; i < n; ++i) {
    BatchJob j;
    j.s = scenes[i]->view();
    j.c = camera_dev(cams[i], W[i], H[i]);
    j.depth = depth[i];
    j.tiles_x = 0;
    j.rgb = rgb_out[i];
    b->host_jobs.push_back(j);
    b->scenes.push_back(scenes[i]);
    b->any_sky = b->any_sky || scenes[i]->sky != nullptr;
    const rt_scene_s* sc = scenes[i];
    b->job_cost.push_back(64.0 * (depth[i] + 1) * (sc->n_spheres + sc->n_planes + 1) *
                          (1 + sc->n_lights));
  }
  size_t total_spheres = 0;
  for (int i = 0; i < n; ++i) {
    total_spheres += pad_spheres(scenes[i]->n_spheres) + kGroup;
    b->max_spheres = std::max(b->max_spheres, pad_spheres(scenes[i]->n_spheres) + kGroup);
  }
  int dev = 0, cus = 256;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipMalloc(&b->cones, 2 * sizeof(float4) * std::max<size_t>(total_spheres, 1));
  if (e == hipSuccess) e = hipMalloc(&b->cone_ptr, sizeof(float4*) * n);
  if (e == hipSuccess) {
    std::vector<float4*> ptrs(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      ptrs[i] = b->cones + off;
      b->host_jobs[i].s.eye_cone = ptrs[i];
      b->host_jobs[i].s.eye_oc = ptrs[i] + total_spheres;
      off += pad_spheres(scenes[i]->n_spheres) + kGroup;
    }
    e = hipMemcpy(b->cone_ptr, ptrs.data(), sizeof(float4*) * n, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipMalloc(&b->jobs, sizeof(BatchJob) * n);
  if (e == hipSuccess) e = hipMalloc(&b->queue, sizeof(TileRef) * max_tiles);
  if (e == hipSuccess) e = hipMalloc(&b->counter, sizeof(unsigned int));
  if (e != hipSuccess) return hip_fail(e, "batch allocation");
  Shape sh{4, 8, cus * 4};
  rt_status st = RT_OK;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "device properties");
  b->tune_key = signature(b, prop.gcnArchName, cus);
  if (autotune_flag) {
    if (!tune_cache_get(b->tune_key, &sh)) {
      st = autotune(b, cus, stream, &sh);
      if (st != RT_OK) return st;
      // a cache file that cannot be written only costs the next process a
      // re-tune
      (void)tune_cache_put(b->tune_key, sh);
    }
  }
  e = upload_shape(b, sh, stream);
  // capture reset + persistent kernel into a graph on a private stream
  hipStream_t cap = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch_batch(b, cap);
    e = hipStreamEndCapture(cap, &b->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (cap) (void)hipStreamDestroy(cap);
  if (e != hipSuccess) return hip_fail(e, "batch graph capture");
  guard.b = nullptr;
  *out = b;
  return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_batch_create(int32_t n, const rt_scene* scenes, const rt_camera* cams,
                          const int32_t* W, const int32_t* H, const int32_t* depth,
                          float* const* rgb_out, int32_t autotune_flag, void* stream_v,
                          rt_batch* out) {
  try {
    return batch_create(n, scenes, cams, W, H, depth, rgb_out, autotune_flag, stream_v, out);
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return err(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

// The job descriptors hold each scene's skybox pointer and size as they were
// at creation; a skybox set, removed or resized since then would be read
// through a stale pointer, so the launch refuses it.
static rt_status check_skies(const rt_batch_s* b) {
  for (int i = 0; i < b->n; ++i) {
    const rt_scene_s* sc = b->scenes[i];
    const SceneDev& s = b->host_jobs[i].s;
    if (sc->sky != s.sky || sc->sky_w != s.sky_w || sc->sky_h != s.sky_h)
      return err(RT_ERR_INVALID_ARG, "the skybox of scene " + std::to_string(i) +
                                         " changed since the batch was created");
  }
  return RT_OK;
}

rt_status rt_batch_launch(rt_batch b, void* stream) {
  if (!b) return err(RT_ERR_INVALID_ARG, "batch is NULL");
  rt_status st = check_skies(b);
  if (st != RT_OK) return st;
  return hip_fail(hipGraphLaunch(b->exec, (hipStream_t)stream), "batch graph launch");
}

rt_status rt_batch_launch_direct(rt_batch b, void* stream) {
  if (!b) return err(RT_ERR_INVALID_ARG, "batch is NULL");
  rt_status st = check_skies(b);
  if (st != RT_OK) return st;
  return hip_fail(launch_batch(b, (hipStream_t)stream), "batch launch");
}

rt_status rt_batch_counts(rt_batch b, int64_t* counts, void* stream) {
  if (!b) return err(RT_ERR_INVALID_ARG, "batch is NULL");
  if (!counts) return err(RT_ERR_INVALID_ARG, "counts is NULL");
  rt_status st = check_skies(b);
  if (st != RT_OK) return st;
  return hip_fail(launch_batch(b, (hipStream_t)stream, (unsigned long long*)counts),
                  "batch count launch");
}

rt_status rt_batch_shape(rt_batch b, int32_t* workgroups, int32_t* tile_w, int32_t* tile_h) {
  if (!b) return err(RT_ERR_INVALID_ARG, "batch is NULL");
  if (workgroups) *workgroups = b->shape.grid;
  if (tile_w) *tile_w = b->shape.wave_w;
  if (tile_h) *tile_h = (64 / b->shape.wave_w) * b->shape.waves;
  return RT_OK;
}

rt_status rt_batch_tune_key(rt_batch b, char* buf, int64_t cap, int64_t* len) {
  if (!b) return err(RT_ERR_INVALID_ARG, "batch is NULL");
  if (len) *len = (int64_t)b->tune_key.size();
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>((size_t)cap - 1, b->tune_key.size());
    memcpy(buf, b->tune_key.data(), n);
    buf[n] = '\0';
  }
  return RT_OK;
}

rt_status rt_batch_destroy(rt_batch b) {
  free_batch(b);
  return RT_OK;
}

}  // extern "C"
