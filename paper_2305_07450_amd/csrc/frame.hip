// frame.hip - the interactive per-frame path (rt_frame_*): every frame
// streams the camera, the ray-tracing properties and the sphere positions in
// and the image out, as the paper's task schedule does for its GUI loop
// (Section 3.9), replayed as a HIP graph whose node parameters change from
// frame to frame.
//
// One graph per slot, two slots, so that the host can stage frame k+1 while
// the device renders frame k:
//   positions H2D (pinned slot staging -> device)
//   -> prep kernel (move the spheres, rebuild their light cones and the eye cones)
//   -> [soft frames: sample table] -> render
//   -> [packed pixels: pack kernel] -> [image D2H into the slot's pinned copy]
// Graphs launched on one stream run in order, so the device-side buffers
// (positions, the scene, the image, the packed pixels) are shared by the
// slots; only the host-side staging and image copies are per slot.  The
// copy-out stays in the render's stream: run beside the device-to-host copy
// (a copy kernel), the render kernel slowed down by about the copy's length,
// so the overlap gained nothing.
#include <string.h>

#include <cmath>
#include <new>

#include "rt_internal.hpp"

namespace rtk {

struct PrepArgs {
  const float* pos;   // [N][3] new centres (device)
  int move;           // 0: keep the centres
  int N, L, n4;
  float ex, ey, ez;   // the eye
  float4* geom;
  const float2* rad;
  const float4* light;
  float4* light_cone;
  float4* eye_cone;
  float4* light_oc;
  float4* eye_oc;
};

// One lane per sphere slot (padding included): the new centre, the cones
// and o - c of the sphere seen from every light, then from the eye.  They are
// the same functions of the same floats as at upload and in the eye-cone
// kernel, so a frame renders the bits that rt_scene_update + rt_render give.
__global__ void frame_prep_kernel(PrepArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.N) {
    float4 g = a.geom[i];
    if (a.move) {
      g.x = a.pos[3 * i];
      g.y = a.pos[3 * i + 1];
      g.z = a.pos[3 * i + 2];
      a.geom[i] = g;
      const float r = a.rad[i].x;
      for (int l = 0; l < a.L; ++l) {
        const float4 q = a.light[l];
        a.light_cone[(int64_t)l * a.n4 + i] = sphere_cone(q.x, q.y, q.z, g.x, g.y, g.z, r);
        a.light_oc[(int64_t)l * a.n4 + i] = make_float4(q.x - g.x, q.y - g.y, q.z - g.z, g.w);
      }
    }
    a.eye_cone[i] = sphere_cone(a.ex, a.ey, a.ez, g.x, g.y, g.z, a.rad[i].x);
    a.eye_oc[i] = make_float4(a.ex - g.x, a.ey - g.y, a.ez - g.z, g.w);
  } else if (i < a.n4 + kGroup) {
    a.eye_cone[i] = make_float4(0.0f, 0.0f, 0.0f, kPadConeW);
    a.eye_oc[i] = make_float4(0.0f, 0.0f, 0.0f, kPadR2);
  }
}

// One 8-bit channel of a packed pixel: round(clamp(c, 0, 1) * 255), the
// product and the half added in FP32 (each rounded once), then floored.  A
// NaN clamps to 0.
__device__ __forceinline__ uint32_t channel8(float c) {
  const float x = fminf(fmaxf(c, 0.0f), 1.0f);
  return (uint32_t)floorf(x * 255.0f + 0.5f);
}

// The image as 32-bit ARGB pixels (alpha 255), one lane per pixel.
__global__ void pack_argb_kernel(const float* __restrict__ rgb, uint32_t* __restrict__ px,
                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
    px[i] = 0xFF000000u | (channel8(r) << 16) | (channel8(g) << 8) | channel8(b);
  }
}

}  // namespace rtk

using namespace rtk;

namespace {

struct Slot {
  float* h_pos = nullptr;   // pinned [N][3]
  void* h_img = nullptr;    // pinned image copy (stream_out): float [H][W][3] or uint32 [H][W]
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t prep = nullptr, table = nullptr, render = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;     // submitted, not yet waited for
};

}  // namespace

struct rt_frame_s {
  rt_scene_s* sc = nullptr;
  int W = 0, H = 0;
  bool soft = false, stream_out = false, prefilter = true;
  int format = RT_FRAME_RGB32F;
  float* rgb = nullptr;     // device image (caller's)
  float* d_pos = nullptr;   // device [N][3]
  uint32_t* d_px = nullptr; // device packed pixels (RT_FRAME_ARGB8)
  bool built_sky = false;   // the render nodes use the skybox instantiation
  Slot slot[2];
  int64_t submitted = 0;    // frames launched
  int64_t returned = 0;     // frames handed out by rt_frame_result (or dropped)
};

namespace {

#define FR_TRY(call, what)                      \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Kernel-node parameters of one frame.  The argument storage lives here; the
// node copies it when it is set.
struct NodeArgs {
  PrepArgs prep{};
  SceneDev s{};
  CameraDev c{};
  int depth = 0;
  int samples = 0;
  float radius = 0.0f;
  float2* table = nullptr;
  SoftShadows sh{};
  float* rgb = nullptr;
  int32_t* ids = nullptr;
  int32_t* rec_ids = nullptr;
  uint8_t* rec_lit = nullptr;
  void* prep_args[1];
  void* table_args[3];
  void* render_args[7];
  hipKernelNodeParams prep_p{}, table_p{}, render_p{};
};

void fill_args(const rt_frame_s* f, const rt_camera& cam, int depth, int samples, float radius,
               bool move, NodeArgs& a) {
  const rt_scene_s& sc = *f->sc;
  a.c = camera_dev(cam, f->W, f->H);
  a.s = sc.view();
  a.depth = depth;
  a.rgb = f->rgb;
  const int n4 = pad_spheres(sc.n_spheres);
  a.prep.pos = f->d_pos;
  a.prep.move = move ? 1 : 0;
  a.prep.N = sc.n_spheres;
  a.prep.L = sc.n_lights;
  a.prep.n4 = n4;
  a.prep.ex = a.c.ex;
  a.prep.ey = a.c.ey;
  a.prep.ez = a.c.ez;
  a.prep.geom = sc.geom;
  a.prep.rad = sc.rad;
  a.prep.light = sc.light;
  a.prep.light_cone = sc.light_cone;
  a.prep.eye_cone = sc.eye_cone;
  a.prep.light_oc = sc.light_oc;
  a.prep.eye_oc = sc.eye_oc;
  a.prep_args[0] = &a.prep;
  a.prep_p.func = (void*)frame_prep_kernel;
  a.prep_p.gridDim = dim3((n4 + kGroup + 255) / 256);
  a.prep_p.blockDim = dim3(256);
  a.prep_p.kernelParams = a.prep_args;
  const bool sky = sc.sky != nullptr;
  a.render_p.gridDim = render_grid(f->W, f->H);
  a.render_p.blockDim = dim3(f->soft ? kRenderThreads * soft_parts(f->W, f->H) : kRenderThreads);
  if (f->soft) {
    a.samples = samples;
    a.radius = radius;
    a.table = sc.soft_table;
    a.table_args[0] = &a.samples;   // sample_table_kernel(int n, float radius, float2* table)
    a.table_args[1] = &a.radius;
    a.table_args[2] = &a.table;
    a.table_p.func = (void*)sample_table_kernel_fn();
    a.table_p.gridDim = dim3((samples + 255) / 256);
    a.table_p.blockDim = dim3(256);
    a.table_p.kernelParams = a.table_args;
    a.sh.n = samples;
    a.sh.radius = radius;
    a.sh.table = sc.soft_table;
    a.sh.parts = soft_parts(f->W, f->H);
    // render_soft_kernel(SceneDev, CameraDev, int depth, SoftShadows, float* rgb, int32_t* ids)
    a.render_args[0] = &a.s;
    a.render_args[1] = &a.c;
    a.render_args[2] = &a.depth;
    a.render_args[3] = &a.sh;
    a.render_args[4] = &a.rgb;
    a.render_args[5] = &a.ids;
    a.render_p.func = (void*)render_soft_kernel_fn(sky, f->prefilter);
  } else {
    // render_kernel(SceneDev, CameraDev, int depth, float* rgb, int32_t* ids, int32_t*, uint8_t*)
    a.render_args[0] = &a.s;
    a.render_args[1] = &a.c;
    a.render_args[2] = &a.depth;
    a.render_args[3] = &a.rgb;
    a.render_args[4] = &a.ids;
    a.render_args[5] = &a.rec_ids;
    a.render_args[6] = &a.rec_lit;
    a.render_p.func = (void*)render_kernel_fn(sky, f->prefilter);
  }
  a.render_p.kernelParams = a.render_args;
}

void destroy_graphs(rt_frame_s* f) {
  for (Slot& s : f->slot) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    s.exec = nullptr;
    s.graph = nullptr;
    s.prep = s.table = s.render = nullptr;
  }
}

// Build both slots' graphs for the scene's current skybox state, from the
// parameters of a first frame (every submit sets its own before launching).
rt_status build_graphs(rt_frame_s* f) {
  destroy_graphs(f);
  rt_camera cam{};
  cam.fov_deg = 60.0f;
  NodeArgs a;
  fill_args(f, cam, 0, f->soft ? 2 : 1, 1.0f, false, a);
  const size_t pos_bytes = (size_t)f->sc->n_spheres * 3 * sizeof(float);
  int64_t n_px = (int64_t)f->W * f->H;
  for (Slot& s : f->slot) {
    FR_TRY(hipGraphCreate(&s.graph, 0), "frame graph");
    hipGraphNode_t last = nullptr;
    if (pos_bytes) {
      FR_TRY(hipGraphAddMemcpyNode1D(&last, s.graph, nullptr, 0, f->d_pos, s.h_pos, pos_bytes,
                                     hipMemcpyHostToDevice),
             "frame positions node");
    }
    FR_TRY(hipGraphAddKernelNode(&s.prep, s.graph, last ? &last : nullptr, last ? 1 : 0,
                                 &a.prep_p),
           "frame prep node");
    last = s.prep;
    if (f->soft) {
      FR_TRY(hipGraphAddKernelNode(&s.table, s.graph, &last, 1, &a.table_p), "frame table node");
      last = s.table;
    }
    FR_TRY(hipGraphAddKernelNode(&s.render, s.graph, &last, 1, &a.render_p), "frame render node");
    last = s.render;
    if (f->format == RT_FRAME_ARGB8) {
      const float* src = f->rgb;
      uint32_t* dst = f->d_px;
      void* args[3] = {&src, &dst, &n_px};
      hipKernelNodeParams p{};
      p.func = (void*)pack_argb_kernel;
      p.gridDim = dim3((unsigned)((n_px + 255) / 256));
      p.blockDim = dim3(256);
      p.kernelParams = args;
      hipGraphNode_t pack;
      FR_TRY(hipGraphAddKernelNode(&pack, s.graph, &last, 1, &p), "frame pack node");
      hipGraphNode_t out;
      FR_TRY(hipGraphAddMemcpyNode1D(&out, s.graph, &pack, 1, s.h_img, f->d_px,
                                     (size_t)n_px * sizeof(uint32_t), hipMemcpyDeviceToHost),
             "frame pixels node");
    } else if (f->stream_out) {
      hipGraphNode_t out;
      FR_TRY(hipGraphAddMemcpyNode1D(&out, s.graph, &last, 1, s.h_img, f->rgb,
                                     (size_t)n_px * 3 * sizeof(float), hipMemcpyDeviceToHost),
             "frame image node");
    }
    FR_TRY(hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0), "frame graph instantiate");
  }
  f->built_sky = f->sc->sky != nullptr;
  return RT_OK;
}

void free_frame(rt_frame_s* f) {
  if (!f) return;
  for (Slot& s : f->slot)
    if (s.done) (void)hipEventSynchronize(s.done);
  destroy_graphs(f);
  for (Slot& s : f->slot) {
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.h_pos) (void)hipHostFree(s.h_pos);
    if (s.h_img) (void)hipHostFree(s.h_img);
  }
  if (f->d_px) (void)hipFree(f->d_px);
  if (f->d_pos) (void)hipFree(f->d_pos);
  delete f;
}

}  // namespace

extern "C" {

rt_status rt_frame_create(rt_scene scene, const rt_frame_desc* d, rt_frame* out) {
  if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!scene) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (!d) return fail(RT_ERR_INVALID_ARG, "frame desc is NULL");
  if (d->W <= 0 || d->H <= 0 || d->W > RT_MAX_DIM || d->H > RT_MAX_DIM)
    return fail(RT_ERR_INVALID_ARG, "image %dx%d outside [1, %d]", d->W, d->H, RT_MAX_DIM);
  if (d->soft != 0 && d->soft != 1) return fail(RT_ERR_INVALID_ARG, "soft=%d is not 0 or 1", d->soft);
  if (d->format != RT_FRAME_RGB32F && d->format != RT_FRAME_ARGB8)
    return fail(RT_ERR_INVALID_ARG, "format=%d is not RT_FRAME_RGB32F or RT_FRAME_ARGB8",
                d->format);
  if (d->format == RT_FRAME_ARGB8 && !d->stream_out)
    return fail(RT_ERR_INVALID_ARG, "RT_FRAME_ARGB8 pixels are for streaming out: set stream_out");
  if (d->flags & ~(uint32_t)RT_RENDER_NO_PREFILTER)
    return fail(RT_ERR_INVALID_ARG, "unknown render flags 0x%x", d->flags);
  if (!d->rgb_out) return fail(RT_ERR_INVALID_ARG, "rgb_out is NULL");
  rt_frame_s* f = new (std::nothrow) rt_frame_s();
  if (!f) return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
  f->sc = scene;
  f->W = d->W;
  f->H = d->H;
  f->soft = d->soft != 0;
  f->stream_out = d->stream_out != 0;
  f->format = d->format;
  f->prefilter = !(d->flags & RT_RENDER_NO_PREFILTER);
  f->rgb = d->rgb_out;
  const size_t pos_bytes = (size_t)scene->n_spheres * 3 * sizeof(float);
  const size_t n_px = (size_t)f->W * f->H;
  const size_t img_bytes =
      n_px * (f->format == RT_FRAME_ARGB8 ? sizeof(uint32_t) : 3 * sizeof(float));
  hipError_t e = hipSuccess;
  if (pos_bytes) e = hipMalloc(&f->d_pos, pos_bytes);
  if (e == hipSuccess && f->format == RT_FRAME_ARGB8)
    e = hipMalloc(&f->d_px, n_px * sizeof(uint32_t));
  for (Slot& s : f->slot) {
    if (e == hipSuccess && pos_bytes) {
      e = hipHostMalloc(&s.h_pos, pos_bytes, hipHostMallocDefault);
      if (e == hipSuccess) memset(s.h_pos, 0, pos_bytes);
    }
    if (e == hipSuccess && f->stream_out)
      e = hipHostMalloc(&s.h_img, img_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    rt_status st = hip_fail(e, "frame allocation");
    free_frame(f);
    return st;
  }
  rt_status st = build_graphs(f);
  if (st != RT_OK) {
    free_frame(f);
    return st;
  }
  *out = f;
  return RT_OK;
}

rt_status rt_frame_submit(rt_frame f, const rt_frame_input* in, void* stream) {
  if (!f) return fail(RT_ERR_INVALID_ARG, "frame is NULL");
  if (!in) return fail(RT_ERR_INVALID_ARG, "frame input is NULL");
  rt_status st = validate_camera(&in->cam, f->W, f->H, in->depth);
  if (st != RT_OK) return st;
  if (f->soft) {
    if (in->samples < 2 || in->samples > RT_MAX_SAMPLES)
      return fail(RT_ERR_INVALID_ARG, "soft frame: samples %d outside [2, %d]", in->samples,
                  RT_MAX_SAMPLES);
    if (!(in->light_radius > 0.0f) || !std::isfinite(in->light_radius))
      return fail(RT_ERR_INVALID_ARG, "soft frame: light_radius must be finite and > 0");
  } else if (in->samples != 1) {
    return fail(RT_ERR_INVALID_ARG, "hard frame: samples must be 1, not %d", in->samples);
  }
  const int N = f->sc->n_spheres;
  if (in->sphere_pos && !finite_all(in->sphere_pos, 3 * (int64_t)N))
    return fail(RT_ERR_INVALID_ARG, "non-finite sphere position");
  if ((f->sc->sky != nullptr) != f->built_sky) {
    // the skybox was added or removed: the render node needs the other kernel
    for (Slot& s : f->slot) {
      if (s.pending) FR_TRY(hipEventSynchronize(s.done), "frame wait");
      s.pending = false;
    }
    if ((st = build_graphs(f)) != RT_OK) return st;
  }
  Slot& s = f->slot[f->submitted & 1];
  // at most two frames wait to be returned: the older one is dropped
  if (f->submitted - f->returned >= 2) f->returned = f->submitted - 1;
  // the slot's staging and host image are free once its previous frame ended
  if (s.pending) FR_TRY(hipEventSynchronize(s.done), "frame wait");
  s.pending = false;
  const bool move = in->sphere_pos != nullptr && N > 0;
  if (move) memcpy(s.h_pos, in->sphere_pos, (size_t)N * 3 * sizeof(float));
  NodeArgs a;
  fill_args(f, in->cam, in->depth, in->samples, in->light_radius, move, a);
  FR_TRY(hipGraphExecKernelNodeSetParams(s.exec, s.prep, &a.prep_p), "frame prep params");
  if (f->soft)
    FR_TRY(hipGraphExecKernelNodeSetParams(s.exec, s.table, &a.table_p), "frame table params");
  FR_TRY(hipGraphExecKernelNodeSetParams(s.exec, s.render, &a.render_p), "frame render params");
  FR_TRY(hipGraphLaunch(s.exec, (hipStream_t)stream), "frame graph launch");
  FR_TRY(hipEventRecord(s.done, (hipStream_t)stream), "frame event");
  s.pending = true;
  ++f->submitted;
  return RT_OK;
}

rt_status rt_frame_result(rt_frame f, const void** host_image) {
  if (!f) return fail(RT_ERR_INVALID_ARG, "frame is NULL");
  if (host_image) *host_image = nullptr;
  if (f->returned == f->submitted) return fail(RT_ERR_INVALID_ARG, "no frame is waiting");
  Slot& s = f->slot[f->returned & 1];
  if (s.pending) FR_TRY(hipEventSynchronize(s.done), "frame wait");
  s.pending = false;
  if (host_image) *host_image = s.h_img;
  ++f->returned;
  return RT_OK;
}

rt_status rt_frame_destroy(rt_frame f) {
  free_frame(f);
  return RT_OK;
}

}  // extern "C"
