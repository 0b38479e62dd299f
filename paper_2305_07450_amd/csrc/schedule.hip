// schedule.hip - the launch that precedes a render: the spheres' cones seen
// from the eye, and the order in which the render takes its 8 x 8 tiles.
//
// A frame's time is set by its slowest tiles: a tile whose mirror rays fan
// out among many spheres runs ten times longer than the median one (a slow
// tile alone on the GPU takes about half a 1080p frame), and in row order
// such tiles start only after a fifth of the frame has passed.  So the render
// takes its tiles longest first, the order that minimises the makespan of a
// list schedule (LPT), with the lengths measured by the previous render of
// the same scene and image size: every tile's wave writes its own duration as
// a bin of a third of an octave (render.hip).  Consecutive frames of a scene
// are alike, and an order from another view is still a permutation of the
// tiles, so a moved camera or moved spheres only make the order less apt.
// The first render of a size takes row order.  The order changes no pixel:
// every tile is rendered by the same code wherever it falls in the launch.
//
// The render that records also counts its tiles per chunk of 1024 and bin
// (render.hip).  One launch here: blocks [0, cone_blocks) write the eye cones
// and eye - centre table (the arithmetic of eye_cone_kernel, so the same
// bits) and zero the
// histograms the coming render fills; each block of [cone_blocks,
// cone_blocks + chunks) places the 1024 tiles of its chunk in the order,
// longest bin first and row order within a bin: from the chunk histograms it
// sums each bin over the image and over the chunks before its own, and each
// tile's rank among the chunk's tiles of its bin comes from wave ballots.  The
// blocks share nothing but what they read: no atomics, fences or second pass.
#include "rt_internal.hpp"

namespace rtk {

constexpr int kPrepThreads = 1024;
constexpr int kPrepWaves = kPrepThreads / 64;

struct PrepareArgs {
  const float4* geom;       // [n4 + kGroup] centre, r^2
  const float2* rad;        // [N] r, 1/r
  float4* eye_cone;         // [n4 + kGroup] out
  float4* eye_oc;           // [n4 + kGroup] out: eye - centre, r^2
  int n_spheres;
  int cone_blocks, chunks;
  float ex, ey, ez;         // the eye
  int n_tiles;
  const uint8_t* bin;       // [n_tiles] bins the last render recorded
  int hist_chunks;          // histogram chunks of kSchedHistChunk tiles
  const uint32_t* hist;     // [hist_chunks][kSchedBins] its chunk histograms
  uint32_t* next_hist;      // [kSchedChunks][kSchedBins] zeroed for the coming render, or NULL
  int32_t* order;           // out: tiles, longest first, position p at sched_slot(p)
};

__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(PrepareArgs a) {
  static_assert(kSchedChunk == kPrepThreads, "one tile per thread of a chunk block");
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  if (b < a.cone_blocks) {
    const int i = b * kPrepThreads + tid;
    if (i < a.n_spheres) {
      const float4 g = a.geom[i];
      a.eye_cone[i] = sphere_cone(a.ex, a.ey, a.ez, g.x, g.y, g.z, a.rad[i].x);
      a.eye_oc[i] = make_float4(a.ex - g.x, a.ey - g.y, a.ez - g.z, g.w);
    } else if (i < pad_spheres(a.n_spheres) + kGroup) {
      a.eye_cone[i] = make_float4(0.0f, 0.0f, 0.0f, kPadConeW);
      a.eye_oc[i] = make_float4(0.0f, 0.0f, 0.0f, kPadR2);
    }
    if (b == 0 && a.next_hist)
      for (int j = tid; j < kSchedChunks * kSchedBins; j += kPrepThreads) a.next_hist[j] = 0;
    return;
  }
  __shared__ uint32_t s_total[kSchedBins];    // tiles per bin, whole image
  __shared__ uint32_t s_before[kSchedBins];   // tiles per bin before this chunk
  __shared__ uint32_t s_wave[kPrepWaves][kSchedBins];
  __shared__ bool s_bad;
  const int lane = __lane_id();
  const int wave = tid >> 6;
  const int c = b - a.cone_blocks;
  if (tid < kSchedBins) s_total[tid] = s_before[tid] = 0;
  if (tid < kPrepWaves * kSchedBins) (&s_wave[0][0])[tid] = 0;
  const int t = c * kSchedChunk + tid;
  const bool valid = t < a.n_tiles;
  const int k = valid ? (int)(a.bin[t] & (kSchedBins - 1)) : 0;
  __syncthreads();
  // ---- sums over the chunk histograms (two entries a thread) --------------
  static_assert(kSchedChunk % kSchedHistChunk == 0, "histogram chunks tile a block's chunk");
  const int hc0 = c * (kSchedChunk / kSchedHistChunk);   // first histogram of this chunk
  for (int j = tid; j < a.hist_chunks * kSchedBins; j += kPrepThreads) {
    const uint32_t v = a.hist[j];
    const int kk = j & (kSchedBins - 1);
    if (v) {
      atomicAdd(&s_total[kk], v);
      if (j / kSchedBins < hc0) atomicAdd(&s_before[kk], v);
    }
  }
  // ---- this chunk's tiles: rank among the chunk's equal bins, row order ----
  const uint64_t below = (1ull << lane) - 1;
  uint32_t rank = 0;
  uint64_t rem = wave_mask(valid);
  while (rem) {
    const int kk = __builtin_amdgcn_readlane(k, (int)__builtin_ctzll(rem));
    const uint64_t m = wave_mask(valid & (k == kk));
    if (valid & (k == kk)) rank = (uint32_t)__builtin_popcountll(m & below);
    if (lane == 0) s_wave[wave][kk] = (uint32_t)__builtin_popcountll(m);
    rem &= ~m;
  }
  __syncthreads();
  if (tid == 0) {
    // histograms that do not count every tile once (never the case for a
    // render's own record) leave the tiles in row order
    uint32_t n = 0;
    for (int kk = 0; kk < kSchedBins; ++kk) n += s_total[kk];
    s_bad = n != (uint32_t)a.n_tiles;
  }
  __syncthreads();
  if (!valid) return;
  if (s_bad) {
    a.order[sched_slot(t, a.n_tiles)] = t;
    return;
  }
  uint32_t pos = s_before[k] + rank;
  for (int kk = kSchedBins - 1; kk > k; --kk) pos += s_total[kk];   // longer bins first
  for (int w = 0; w < wave; ++w) pos += s_wave[w][k];
  if (pos < (uint32_t)a.n_tiles) a.order[sched_slot((int)pos, a.n_tiles)] = t;
}

bool schedule_applies(const rt_scene_s& sc, int W, int H) {
  const int64_t tiles = (int64_t)((W + kRenderTile - 1) / kRenderTile) *
                        ((H + kRenderTile - 1) / kRenderTile);
  return sc.sched && tiles >= kSchedMinTiles && tiles <= kSchedMaxTiles;
}

hipError_t launch_prepare(rt_scene_s& sc, const CameraDev& c, bool schedule, int kind,
                          bool* ordered, hipStream_t stream) {
  PrepareArgs a;
  a.geom = sc.geom;
  a.rad = sc.rad;
  a.eye_cone = sc.eye_cone;
  a.eye_oc = sc.eye_oc;
  a.n_spheres = sc.n_spheres;
  a.ex = c.ex;
  a.ey = c.ey;
  a.ez = c.ez;
  a.cone_blocks = (pad_spheres(sc.n_spheres) + kGroup + kPrepThreads - 1) / kPrepThreads;
  const dim3 g = render_grid(c.W, c.H);
  a.n_tiles = (int)(g.x * g.y);
  // an order from the last render's measured bins, if it rendered this size
  const bool from_history =
      schedule && sc.hist_W == c.W && sc.hist_H == c.H && sc.hist_kind == kind;
  a.chunks = from_history ? (a.n_tiles + kSchedChunk - 1) / kSchedChunk : 0;
  a.hist_chunks = (a.n_tiles + kSchedHistChunk - 1) / kSchedHistChunk;
  uint32_t* hist = (uint32_t*)(sc.sched + kSchedHist);
  a.bin = sc.sched + kSchedBin;
  a.hist = hist + sc.hist_set * kSchedChunks * kSchedBins;
  // the render that follows records into the other set
  a.next_hist = schedule ? hist + (sc.hist_set ^ 1) * kSchedChunks * kSchedBins : nullptr;
  a.order = (int32_t*)(sc.sched + kSchedOrder);
  hipLaunchKernelGGL(prepare_kernel, dim3(a.cone_blocks + a.chunks), dim3(kPrepThreads), 0,
                     stream, a);
  const hipError_t e = hipGetLastError();
  *ordered = e == hipSuccess && from_history;
  return e;
}

}  // namespace rtk
