// render.hip - forward render kernel and scene packing kernel (gfx950).
//
// Launch shape: one wave64 per workgroup, owning an 8 x 8 pixel tile (one lane
// per pixel, paper Section 3.9: every pixel is an independent work item), so
// the 64 rays of a wave start from the same eye through neighbouring pixels
// and take the same branch over most primitives.  The workgroup is only a
// unit of dispatch: single waves fill the compute units more evenly than
// groups of four did (5 % faster at 1080p).  LDS holds only wave-private data
// (the tile's start time, and in render_kernel the per-lane ray slots of the
// transposed tests, which rely on the workgroup being this one wave).
// The scene is read through scalar loads (trace.hpp), so the inner loops are
// pure VALU arithmetic on SGPR operands.
#include "rt_internal.hpp"

namespace rtk {

constexpr int kTile = kRenderTile;   // wave tile edge = workgroup tile edge
static_assert(kRenderThreads == 64, "one wave per workgroup: the LDS ray slots are the wave's own");

// Records sink: segment ids and lit masks in [depth+1][H][W] planes.
struct RecordSink {
  int32_t* id_plane;
  uint8_t* lit_plane;
  int64_t plane;
  int64_t pix;
  __device__ __forceinline__ void seg(int k, int id) {
    id_plane[k * plane + pix] = id;
    if (id < 0) lit_plane[k * plane + pix] = 0;   // a miss has no lit mask
  }
  __device__ __forceinline__ void lit(int k, uint32_t m) { lit_plane[k * plane + pix] = (uint8_t)m; }
};

// Tile of this workgroup: blockIdx in row order, or the scene's order table.
__device__ __forceinline__ int tile_of(const SceneDev& s) {
  const int n = (int)(gridDim.x * gridDim.y);
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  if (!(s.sched_mode & kSchedOrdered)) return b;
  return min(max(((const RT_CONSTANT int*)(s.sched + kSchedOrder))[sched_slot(b, n)], 0), n - 1);
}

// The tile's duration for the next render's order: core clocks since t_start,
// as bin floor(3 log2(clocks)) - 36 clamped to [0, kSchedBins) (a third of an
// octave each, 4096 to about 200 000 clocks): one byte per tile, and one to
// the histogram of its chunk of kSchedHistChunk tiles (one atomic per tile, a
// cache line of counts per chunk, issued as the tiles finish).
__device__ __forceinline__ void record_duration(const SceneDev& s, int t, uint64_t t_start) {
  const float clocks = (float)(__builtin_amdgcn_s_memtime() - t_start);
  const int bin = min(max((int)(3.0f * __builtin_amdgcn_logf(fmaxf(clocks, 1.0f))) - 36, 0),
                      kSchedBins - 1);
  if (__lane_id() == 0) {
    s.sched[kSchedBin + t] = (uint8_t)bin;
    uint32_t* hist = (uint32_t*)(s.sched + kSchedHist) +
                     ((s.sched_mode & kSchedHistSet1) ? kSchedChunks * kSchedBins : 0);
    atomicAdd(hist + (t / kSchedHistChunk) * kSchedBins + bin, 1u);
  }
}

// With records the LDS ray slots would take the kernel to 82 VGPRs (5 waves
// per SIMD); held to 6 waves it fits them in 79 without scratch.
template <bool kRecords, bool kPrefilter, class Bg>
__global__ __launch_bounds__(kRenderThreads)
__attribute__((amdgpu_waves_per_eu(kRecords ? 6 : 1))) void render_kernel(SceneDev s, CameraDev c, int depth,
                                                      float* __restrict__ rgb,
                                                      int32_t* __restrict__ id_out,
                                                      int32_t* __restrict__ rec_ids,
                                                      uint8_t* __restrict__ rec_lit) {
  const int lane = threadIdx.x;
  // the tile of this workgroup: in row order, or the b-th of the scene's
  // order (longest first, from the durations the last render recorded)
  const int t = tile_of(s);
  const int ty = t / (int)gridDim.x;
  const int tx = t - ty * (int)gridDim.x;
  // the start time waits in LDS, not in registers, until the tile is done
  __shared__ uint64_t s_start;
  if (s.sched_mode & kSchedRecord) s_start = __builtin_amdgcn_s_memtime();
  const int x = tx * kTile + (lane & 7);
  const int y = ty * kTile + (lane >> 3);
  // lanes outside the image run along (clamped pixel, no output) so that the
  // whole wave executes the path code together; a wave with no pixel leaves
  const bool live = x < c.W && y < c.H;
  if (!wave_any(live)) return;
  const int64_t pix = live ? (int64_t)y * c.W + x : 0;
  Ray r = primary_ray(c, live ? x : c.W - 1, live ? y : c.H - 1);
  float cr, cg, cb;
  int prim;
  if (kRecords) {
    RecordSink sink{rec_ids, rec_lit, (int64_t)c.W * c.H, pix};
    int traced = trace_path<RecordSink, NoCount, kPrefilter, HardShadows, Bg, true>(
        s, r, depth, live, cr, cg, cb, prim, sink);
    if (live) {
      for (int k = traced; k <= depth; ++k) {
        rec_ids[k * sink.plane + pix] = kNotTraced;
        rec_lit[k * sink.plane + pix] = 0;
      }
    }
  } else {
    NoRecords sink;
    trace_path<NoRecords, NoCount, kPrefilter, HardShadows, Bg, true>(s, r, depth, live, cr, cg, cb,
                                                                      prim, sink);
  }
  if (live) {
    rgb[3 * pix + 0] = cr;
    rgb[3 * pix + 1] = cg;
    rgb[3 * pix + 2] = cb;
    if (id_out) id_out[pix] = prim;
  }
  if (s.sched_mode & kSchedRecord) record_duration(s, tile_of(s), s_start);
}

// Soft-shadow render: the same paths with every light sampled (SoftShadows).
// Launched with sh.parts waves per tile: the tile's 64 pixels are spread
// over them, sh.parts neighbouring lanes a pixel, each taking its share of
// the samples (soft_visibility adds their counts).
template <bool kPrefilter, class Bg>
__global__ __launch_bounds__(kSoftMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) void render_soft_kernel(
    SceneDev s, CameraDev c, int depth, SoftShadows sh, float* __restrict__ rgb,
    int32_t* __restrict__ id_out) {
  const int wave = (int)threadIdx.x >> 6;
  const int lane = (int)threadIdx.x & 63;
  // the tile: row order, or the scene's order (as render_kernel)
  const int t = tile_of(s);
  const int ty = t / (int)gridDim.x;
  const int tx = t - ty * (int)gridDim.x;
  const int px = wave * (64 / sh.parts) + lane / sh.parts;   // pixel of the tile
  sh.part = lane % sh.parts;
  // the first wave measures the tile for the next render's order (the waves
  // share no data, and none waits for another)
  __shared__ uint64_t s_start;
  if ((s.sched_mode & kSchedRecord) && wave == 0) s_start = __builtin_amdgcn_s_memtime();
  const int x = tx * kTile + (px & 7);
  const int y = ty * kTile + (px >> 3);
  const bool live = x < c.W && y < c.H;
  if (!wave_any(live)) return;
  const int64_t pix = live ? (int64_t)y * c.W + x : 0;
  Ray r = primary_ray(c, live ? x : c.W - 1, live ? y : c.H - 1);
  float cr, cg, cb;
  int prim;
  NoRecords sink;
  // no LDS ray slots: they cost the skybox variant a wave per SIMD (129 VGPRs)
  trace_path<NoRecords, NoCount, kPrefilter, SoftShadows, Bg, false>(s, r, depth, live, cr, cg, cb,
                                                                       prim, sink, NoCount(), sh);
  if (live && sh.part == 0) {
    rgb[3 * pix + 0] = cr;
    rgb[3 * pix + 1] = cg;
    rgb[3 * pix + 2] = cb;
    if (id_out) id_out[pix] = prim;
  }
  if ((s.sched_mode & kSchedRecord) && wave == 0) record_duration(s, tile_of(s), s_start);
}

// Sample points of the sunflower arrangement: point i of n at radius
// 2 sqrt(i/n) and angle i times the golden angle pi (3 - sqrt 5), as (x, y)
// in the disk basis, computed in double and rounded once, then times the
// light radius in FP32 (so the render reads the offsets ready to use).
__global__ void sample_table_kernel(int n, float radius, float2* __restrict__ table) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double golden = 3.14159265358979323846 * (3.0 - sqrt(5.0));
    const double r = 2.0 * sqrt((double)i / (double)n);
    const double th = (double)i * golden;
    table[i] = make_float2(radius * (float)(r * cos(th)), radius * (float)(r * sin(th)));
  }
}

hipError_t launch_render_soft(const rt_scene_s& sc, const CameraDev& c, int depth, int samples,
                              float radius, float* rgb, int32_t* ids, bool prefilter,
                              int sched_mode, hipStream_t stream) {
  hipLaunchKernelGGL(sample_table_kernel, dim3((samples + 255) / 256), dim3(256), 0, stream,
                     samples, radius, sc.soft_table);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SoftShadows sh;
  sh.n = samples;
  sh.radius = radius;
  sh.table = sc.soft_table;
  sh.parts = soft_parts(c.W, c.H);
  const dim3 grid = render_grid(c.W, c.H);
  const bool sky = sc.sky != nullptr;
  auto kern = sky ? (prefilter ? render_soft_kernel<true, SkyBackground>
                               : render_soft_kernel<false, SkyBackground>)
                  : (prefilter ? render_soft_kernel<true, PlainBackground>
                               : render_soft_kernel<false, PlainBackground>);
  SceneDev s = sc.view();
  s.sched_mode = sched_mode;
  hipLaunchKernelGGL(kern, grid, dim3(kRenderThreads * sh.parts), 0, stream, s, c, depth, sh, rgb,
                     ids);
  return hipGetLastError();
}

// Counting launch: the same paths as render_kernel (with or without the cone
// tests and wave bounds), plus the algorithmic and executed-test counters,
// summed per wave (xor butterfly) and added to counts[kNumCounts] with
// integer atomics.  The counters are per-lane adds; every branch of the path
// code is the same as in the render, so the executed counts are those of the
// render kernel.
template <bool kPrefilter>
__global__ __launch_bounds__(kRenderThreads) void count_kernel(SceneDev s, CameraDev c, int depth,
                                                    unsigned long long* __restrict__ counts) {
  const int lane = threadIdx.x;
  const int x = blockIdx.x * kTile + (lane & 7);
  const int y = blockIdx.y * kTile + (lane >> 3);
  Count cnt;
  const bool live = x < c.W && y < c.H;
  if (wave_any(live)) {
    float cr, cg, cb;
    int prim;
    NoRecords sink;
    trace_path<NoRecords, Count&, kPrefilter>(
        s, primary_ray(c, live ? x : c.W - 1, live ? y : c.H - 1), depth, live, cr, cg, cb, prim,
        sink, cnt);
  }
  for (int j = 0; j < kNumCounts; ++j) {
    int v = cnt.c[j];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) atomicAdd(counts + j, (unsigned long long)v);
  }
}

hipError_t launch_counts(const SceneDev& s, const CameraDev& c, int depth,
                         unsigned long long* counts, bool prefilter, hipStream_t stream) {
  const dim3 grid = render_grid(c.W, c.H);
  auto kern = prefilter ? count_kernel<true> : count_kernel<false>;
  hipLaunchKernelGGL(kern, grid, dim3(kRenderThreads), 0, stream, s, c, depth, counts);
  return hipGetLastError();
}

const void* render_kernel_fn(bool sky, bool prefilter) {
  if (sky)
    return prefilter ? (const void*)render_kernel<false, true, SkyBackground>
                     : (const void*)render_kernel<false, false, SkyBackground>;
  return prefilter ? (const void*)render_kernel<false, true, PlainBackground>
                   : (const void*)render_kernel<false, false, PlainBackground>;
}

const void* render_soft_kernel_fn(bool sky, bool prefilter) {
  if (sky)
    return prefilter ? (const void*)render_soft_kernel<true, SkyBackground>
                     : (const void*)render_soft_kernel<false, SkyBackground>;
  return prefilter ? (const void*)render_soft_kernel<true, PlainBackground>
                   : (const void*)render_soft_kernel<false, PlainBackground>;
}

const void* sample_table_kernel_fn() { return (const void*)sample_table_kernel; }

hipError_t launch_render(const SceneDev& s, const CameraDev& c, int depth, float* rgb,
                         int32_t* ids, int32_t* rec_ids, uint8_t* rec_lit, bool prefilter,
                         hipStream_t stream) {
  const dim3 grid = render_grid(c.W, c.H);
  using P = PlainBackground;
  using K = SkyBackground;
  decltype(&render_kernel<false, true, P>) kern;
  if (s.sky)
    kern = rec_ids ? (prefilter ? render_kernel<true, true, K> : render_kernel<true, false, K>)
                   : (prefilter ? render_kernel<false, true, K> : render_kernel<false, false, K>);
  else
    kern = rec_ids ? (prefilter ? render_kernel<true, true, P> : render_kernel<true, false, P>)
                   : (prefilter ? render_kernel<false, true, P> : render_kernel<false, false, P>);
  hipLaunchKernelGGL(kern, grid, dim3(kRenderThreads), 0, stream, s, c, depth, rgb, ids, rec_ids,
                     rec_lit);
  return hipGetLastError();
}

// Pack the desc-layout arrays into the kernels' layout: r^2 beside the centre,
// (r, 1/r), sphere and plane materials in one id-indexed table.
__global__ void pack_kernel(RawScene raw, int N, int P, int L, float4* geom, float2* rad,
                            float4* mat, float* shine, float4* pgeom, float4* light,
                            float4* light_cone, float4* light_oc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n4 = pad_spheres(N);
  if (i >= N && i < n4 + kGroup) {
    // padding spheres: never hit, never inside a cone
    geom[i] = make_float4(0.0f, 0.0f, 0.0f, kPadR2);
    for (int l = 0; l < L; ++l)
      if (i < n4 || l == L - 1) {
        light_cone[(int64_t)l * n4 + i] = make_float4(0.f, 0.f, 0.f, kPadConeW);
        light_oc[(int64_t)l * n4 + i] = make_float4(0.f, 0.f, 0.f, kPadR2);
      }
  }
  if (i < N) {
    const float* g = raw.sphere_geom + 4 * i;
    float r = g[3];
    geom[i] = make_float4(g[0], g[1], g[2], r * r);
    rad[i] = make_float2(r, 1.0f / r);
    const float* m = raw.sphere_mat + 4 * i;
    mat[i] = make_float4(m[0], m[1], m[2], m[3]);
    shine[i] = raw.sphere_shine[i];
    for (int l = 0; l < L; ++l) {
      const float* q = raw.light + 4 * l;
      light_cone[(int64_t)l * n4 + i] = sphere_cone(q[0], q[1], q[2], g[0], g[1], g[2], r);
      light_oc[(int64_t)l * n4 + i] = make_float4(q[0] - g[0], q[1] - g[1], q[2] - g[2], r * r);
    }
  }
  if (i < P) {
    const float* g = raw.plane_geom + 4 * i;
    pgeom[i] = make_float4(g[0], g[1], g[2], g[3]);
    const float* m = raw.plane_mat + 4 * i;
    mat[N + i] = make_float4(m[0], m[1], m[2], m[3]);
    shine[N + i] = raw.plane_shine[i];
  }
  if (i < L) {
    const float* q = raw.light + 4 * i;
    light[i] = make_float4(q[0], q[1], q[2], q[3]);
  }
}

hipError_t launch_pack(const rt_scene_s& sc, const RawScene& raw, hipStream_t stream) {
  int n = pad_spheres(sc.n_spheres) + kGroup;
  if (sc.n_planes > n) n = sc.n_planes;
  if (sc.n_lights > n) n = sc.n_lights;
  hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, raw,
                     sc.n_spheres, sc.n_planes, sc.n_lights, sc.geom, sc.rad, sc.mat, sc.shine,
                     sc.pgeom, sc.light, sc.light_cone, sc.light_oc);
  return hipGetLastError();
}

__global__ void sky_pack_kernel(const float* __restrict__ rgb, float4* __restrict__ sky,
                                int texels) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < texels) sky[i] = make_float4(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], 0.0f);
}

hipError_t launch_sky_pack(const float* rgb, float4* sky, int texels, hipStream_t stream) {
  hipLaunchKernelGGL(sky_pack_kernel, dim3((texels + 255) / 256), dim3(256), 0, stream, rgb, sky,
                     texels);
  return hipGetLastError();
}

__global__ void eye_cone_kernel(const float4* __restrict__ geom, const float2* __restrict__ rad,
                                int N, float ex, float ey, float ez, float4* __restrict__ out,
                                float4* __restrict__ oc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    float4 g = geom[i];
    out[i] = sphere_cone(ex, ey, ez, g.x, g.y, g.z, rad[i].x);
    oc[i] = make_float4(ex - g.x, ey - g.y, ez - g.z, g.w);
  } else if (i < pad_spheres(N) + kGroup) {
    out[i] = make_float4(0.0f, 0.0f, 0.0f, kPadConeW);
    oc[i] = make_float4(0.0f, 0.0f, 0.0f, kPadR2);
  }
}

hipError_t launch_eye_cones(const rt_scene_s& sc, const CameraDev& c, hipStream_t stream) {
  hipLaunchKernelGGL(eye_cone_kernel, dim3((pad_spheres(sc.n_spheres) + kGroup + 255) / 256), dim3(256), 0,
                     stream,
                     (const float4*)sc.geom, (const float2*)sc.rad, sc.n_spheres, c.ex, c.ey,
                     c.ez, sc.eye_cone, sc.eye_oc);
  return hipGetLastError();
}

}  // namespace rtk
