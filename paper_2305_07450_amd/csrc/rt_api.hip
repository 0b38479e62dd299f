// rt_api.hip - the C ABI of librtmi (include/rt.h): argument validation,
// scene residency and packing, and kernel launches.  Validation runs on the
// host before any HIP call so that argument errors never touch the device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include <cmath>

#include "rt_internal.hpp"

namespace rtk {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

rt_status fail(rt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

rt_status hip_fail(hipError_t e, const char* what) {
  if (e == hipSuccess) return RT_OK;
  rt_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
                     ? RT_ERR_OUT_OF_MEMORY
                     : RT_ERR_DEVICE;
  return fail(st, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                 \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Camera basis in double, rounded once to float.  d = normalize(u right +
// v up + fwd) with right = R e_x, up = R e_y, fwd = R (0, 0, -b),
// b = 1 / tan(fov / 2) (Section 3.2.1) and R = Ry(yaw) Rx(pitch).
CameraDev camera_dev(const rt_camera& cam, int W, int H) {
  const double pi = 3.14159265358979323846;
  double b = 1.0 / tan(0.5 * (double)cam.fov_deg * pi / 180.0);
  double p = (double)cam.pitch_deg * pi / 180.0, y = (double)cam.yaw_deg * pi / 180.0;
  double cp = cos(p), sp = sin(p), cy = cos(y), sy = sin(y);
  // columns of R = Ry(yaw) Rx(pitch)
  double r0[3] = {cy, 0.0, -sy};                      // R e_x
  double r1[3] = {sy * sp, cp, cy * sp};              // R e_y
  double r2[3] = {sy * cp, -sp, cy * cp};             // R e_z
  CameraDev c;
  c.ex = cam.eye[0]; c.ey = cam.eye[1]; c.ez = cam.eye[2];
  c.rx = (float)r0[0]; c.ry = (float)r0[1]; c.rz = (float)r0[2];
  c.ux = (float)r1[0]; c.uy = (float)r1[1]; c.uz = (float)r1[2];
  c.fx = (float)(-b * r2[0]); c.fy = (float)(-b * r2[1]); c.fz = (float)(-b * r2[2]);
  c.inv_s = (float)(1.0 / (double)(W < H ? W : H));
  c.W = W;
  c.H = H;
  return c;
}

bool finite_all(const float* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return false;
  return true;
}

static rt_status validate_desc(const rt_scene_desc* d) {
  if (!d) return fail(RT_ERR_INVALID_ARG, "scene desc is NULL");
  if (d->n_spheres < 0 || d->n_spheres > RT_MAX_SPHERES)
    return fail(RT_ERR_INVALID_ARG, "n_spheres=%d outside [0, %d]", d->n_spheres, RT_MAX_SPHERES);
  if (d->n_planes < 0 || d->n_planes > RT_MAX_PLANES)
    return fail(RT_ERR_INVALID_ARG, "n_planes=%d outside [0, %d]", d->n_planes, RT_MAX_PLANES);
  if (d->n_lights < 0 || d->n_lights > RT_MAX_LIGHTS)
    return fail(RT_ERR_INVALID_ARG, "n_lights=%d outside [0, %d]", d->n_lights, RT_MAX_LIGHTS);
  if (d->spec_model != RT_SPEC_BLINN && d->spec_model != RT_SPEC_PHONG)
    return fail(RT_ERR_INVALID_ARG, "spec_model=%d is not RT_SPEC_BLINN or RT_SPEC_PHONG",
                d->spec_model);
  if (d->mem != RT_HOST && d->mem != RT_DEVICE)
    return fail(RT_ERR_INVALID_ARG, "mem=%d is not RT_HOST or RT_DEVICE", d->mem);
  if (d->n_spheres > 0 && (!d->sphere_geom || !d->sphere_mat || !d->sphere_shine))
    return fail(RT_ERR_INVALID_ARG, "sphere arrays are NULL with n_spheres=%d", d->n_spheres);
  if (d->n_planes > 0 && (!d->plane_geom || !d->plane_mat || !d->plane_shine))
    return fail(RT_ERR_INVALID_ARG, "plane arrays are NULL with n_planes=%d", d->n_planes);
  if (d->n_lights > 0 && !d->light)
    return fail(RT_ERR_INVALID_ARG, "light array is NULL with n_lights=%d", d->n_lights);
  float consts[6] = {d->ambient, d->spec_strength, d->t_min,
                     d->background[0], d->background[1], d->background[2]};
  if (!finite_all(consts, 6)) return fail(RT_ERR_INVALID_ARG, "non-finite scene constant");
  if (d->t_min < 0.0f) return fail(RT_ERR_INVALID_ARG, "t_min=%g < 0", (double)d->t_min);
  if (d->mem == RT_DEVICE) return RT_OK;
  const int N = d->n_spheres, P = d->n_planes, L = d->n_lights;
  if (!finite_all(d->sphere_geom, 4 * (int64_t)N) || !finite_all(d->sphere_mat, 4 * (int64_t)N) ||
      !finite_all(d->sphere_shine, N) || !finite_all(d->plane_geom, 4 * (int64_t)P) ||
      !finite_all(d->plane_mat, 4 * (int64_t)P) || !finite_all(d->plane_shine, P) ||
      !finite_all(d->light, 4 * (int64_t)L))
    return fail(RT_ERR_INVALID_ARG, "non-finite value in a scene array");
  for (int i = 0; i < N; ++i) {
    if (!(d->sphere_geom[4 * i + 3] > 0.0f))
      return fail(RT_ERR_INVALID_ARG, "sphere %d radius %g is not > 0", i,
                  (double)d->sphere_geom[4 * i + 3]);
    if (!(d->sphere_shine[i] > 0.0f))
      return fail(RT_ERR_INVALID_ARG, "sphere %d exponent is not > 0", i);
  }
  for (int j = 0; j < P; ++j) {
    const float* m = d->plane_geom + 4 * j;
    double len = sqrt((double)m[0] * m[0] + (double)m[1] * m[1] + (double)m[2] * m[2]);
    if (fabs(len - 1.0) > 1e-5)
      return fail(RT_ERR_INVALID_ARG, "plane %d normal has length %g, not 1", j, len);
    if (!(d->plane_shine[j] > 0.0f))
      return fail(RT_ERR_INVALID_ARG, "plane %d exponent is not > 0", j);
  }
  for (int l = 0; l < L; ++l)
    if (d->light[4 * l + 3] < 0.0f)
      return fail(RT_ERR_INVALID_ARG, "light %d intensity is < 0", l);
  return RT_OK;
}

rt_status validate_camera(const rt_camera* cam, int32_t W, int32_t H, int32_t depth) {
  if (!cam) return fail(RT_ERR_INVALID_ARG, "camera is NULL");
  float v[6] = {cam->eye[0], cam->eye[1], cam->eye[2], cam->yaw_deg, cam->pitch_deg,
                cam->fov_deg};
  if (!finite_all(v, 6)) return fail(RT_ERR_INVALID_ARG, "non-finite camera value");
  if (!(cam->fov_deg > 0.0f && cam->fov_deg < 180.0f))
    return fail(RT_ERR_INVALID_ARG, "fov=%g outside (0, 180)", (double)cam->fov_deg);
  if (W <= 0 || H <= 0 || W > RT_MAX_DIM || H > RT_MAX_DIM)
    return fail(RT_ERR_INVALID_ARG, "image %dx%d outside [1, %d]", W, H, RT_MAX_DIM);
  if (depth < 0 || depth > RT_MAX_DEPTH)
    return fail(RT_ERR_INVALID_ARG, "depth=%d outside [0, %d]", depth, RT_MAX_DEPTH);
  return RT_OK;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Adjoint grid size for a scene: at most kAdjointBlocks workgroups and at
// most 64 MiB of partials.
int adjoint_blocks(int grad_stride) {
  size_t cap = (64u << 20) / ((size_t)grad_stride * sizeof(float));
  int g = kAdjointBlocks;
  if ((size_t)g > cap) g = (int)cap;
  if (g < 64) g = 64;
  return g;
}

static rt_status upload_values(rt_scene_s* sc, const rt_scene_desc* d, hipStream_t stream) {
  RawScene raw;
  if (d->mem == RT_HOST) {
    const int N = sc->n_spheres, P = sc->n_planes, L = sc->n_lights;
    float* st = sc->staging;
    size_t off = 0;
    auto put = [&](const float* src, size_t n, const float** dst) -> hipError_t {
      *dst = st + off;
      hipError_t e = n ? hipMemcpyAsync(st + off, src, n * sizeof(float), hipMemcpyHostToDevice,
                                        stream)
                       : hipSuccess;
      off += n;
      return e;
    };
    HIP_TRY(put(d->sphere_geom, 4 * (size_t)N, &raw.sphere_geom), "upload spheres");
    HIP_TRY(put(d->sphere_mat, 4 * (size_t)N, &raw.sphere_mat), "upload spheres");
    HIP_TRY(put(d->sphere_shine, (size_t)N, &raw.sphere_shine), "upload spheres");
    HIP_TRY(put(d->plane_geom, 4 * (size_t)P, &raw.plane_geom), "upload planes");
    HIP_TRY(put(d->plane_mat, 4 * (size_t)P, &raw.plane_mat), "upload planes");
    HIP_TRY(put(d->plane_shine, (size_t)P, &raw.plane_shine), "upload planes");
    HIP_TRY(put(d->light, 4 * (size_t)L, &raw.light), "upload lights");
  } else {
    raw.sphere_geom = d->sphere_geom;
    raw.sphere_mat = d->sphere_mat;
    raw.sphere_shine = d->sphere_shine;
    raw.plane_geom = d->plane_geom;
    raw.plane_mat = d->plane_mat;
    raw.plane_shine = d->plane_shine;
    raw.light = d->light;
  }
  HIP_TRY(launch_pack(*sc, raw, stream), "pack kernel");
  if (d->mem == RT_HOST) HIP_TRY(hipStreamSynchronize(stream), "upload sync");
  sc->ambient = d->ambient;
  sc->spec_strength = d->spec_strength;
  sc->t_min = d->t_min;
  sc->bg[0] = d->background[0];
  sc->bg[1] = d->background[1];
  sc->bg[2] = d->background[2];
  return RT_OK;
}

}  // namespace rtk

using namespace rtk;

extern "C" {

const char* rt_status_string(rt_status s) {
  switch (s) {
    case RT_OK: return "RT_OK";
    case RT_ERR_INVALID_ARG: return "RT_ERR_INVALID_ARG";
    case RT_ERR_OUT_OF_MEMORY: return "RT_ERR_OUT_OF_MEMORY";
    case RT_ERR_DEVICE: return "RT_ERR_DEVICE";
    case RT_ERR_UNSUPPORTED: return "RT_ERR_UNSUPPORTED";
  }
  return "unknown rt_status";
}

const char* rt_last_error(void) { return g_last_error.c_str(); }

rt_status rt_scene_upload(const rt_scene_desc* d, void* stream, rt_scene* out) {
  if (!out) return fail(RT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  rt_status st = validate_desc(d);
  if (st != RT_OK) return st;
  rt_scene_s* sc = new (std::nothrow) rt_scene_s();
  if (!sc) return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
  sc->n_spheres = d->n_spheres;
  sc->n_planes = d->n_planes;
  sc->n_lights = d->n_lights;
  sc->spec_model = d->spec_model;
  const size_t N = d->n_spheres, P = d->n_planes, L = d->n_lights;
  sc->grad_stride = (int)align_up(7 * N + 4 * L, 4);
  if (sc->grad_stride == 0) sc->grad_stride = 4;
  const int blocks = adjoint_blocks(sc->grad_stride);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t N4 = pad_spheres((int)N);
  size_t o_geom = take((N4 + kGroup) * sizeof(float4));
  size_t o_rad = take(N * sizeof(float2));
  size_t o_mat = take((N + P) * sizeof(float4));
  size_t o_shine = take((N + P) * sizeof(float));
  size_t o_pgeom = take(P * sizeof(float4));
  size_t o_light = take(L * sizeof(float4));
  size_t o_eye_cone = take((N4 + kGroup) * sizeof(float4));
  size_t o_light_cone = take((L * N4 + kGroup) * sizeof(float4));
  size_t o_eye_oc = take((N4 + kGroup) * sizeof(float4));
  size_t o_light_oc = take((L * N4 + kGroup) * sizeof(float4));
  sc->staging_floats = 9 * N + 9 * P + 4 * L;
  size_t o_stage = take(sc->staging_floats * sizeof(float));
  size_t o_part = take((size_t)blocks * sc->grad_stride * sizeof(float));
  static_assert(RT_MAX_SAMPLES % 8 == 0, "soft sample table is read in blocks of 8");
  size_t o_soft = take((size_t)RT_MAX_SAMPLES * sizeof(float2));
  size_t o_sched = take(kSchedBytes);
  sc->bytes = off;
  hipError_t e = hipGetDevice(&sc->device);
  if (e == hipSuccess) e = hipMalloc(&sc->buffer, sc->bytes);
  if (e != hipSuccess) {
    delete sc;
    return hip_fail(e, "scene allocation");
  }
  char* base = (char*)sc->buffer;
  sc->geom = (float4*)(base + o_geom);
  sc->rad = (float2*)(base + o_rad);
  sc->mat = (float4*)(base + o_mat);
  sc->shine = (float*)(base + o_shine);
  sc->pgeom = (float4*)(base + o_pgeom);
  sc->light = (float4*)(base + o_light);
  sc->eye_cone = (float4*)(base + o_eye_cone);
  sc->light_cone = (float4*)(base + o_light_cone);
  sc->eye_oc = (float4*)(base + o_eye_oc);
  sc->light_oc = (float4*)(base + o_light_oc);
  sc->staging = (float*)(base + o_stage);
  sc->partials = (float*)(base + o_part);
  sc->soft_table = (float2*)(base + o_soft);
  sc->sched = (uint8_t*)(base + o_sched);
  e = hipMemsetAsync(sc->sched + kSchedHist, 0, kSchedBytes - kSchedHist, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipFree(sc->buffer);
    delete sc;
    return hip_fail(e, "scene initialisation");
  }
  st = upload_values(sc, d, (hipStream_t)stream);
  if (st != RT_OK) {
    (void)hipFree(sc->buffer);
    delete sc;
    return st;
  }
  *out = sc;
  return RT_OK;
}

rt_status rt_scene_update(rt_scene sc, const rt_scene_desc* d, void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  rt_status st = validate_desc(d);
  if (st != RT_OK) return st;
  if (d->n_spheres != sc->n_spheres || d->n_planes != sc->n_planes ||
      d->n_lights != sc->n_lights || d->spec_model != sc->spec_model)
    return fail(RT_ERR_INVALID_ARG, "update changes counts or spec_model of the scene");
  return upload_values(sc, d, (hipStream_t)stream);
}

rt_status rt_scene_set_sky(rt_scene sc, const float* rgb, int32_t w, int32_t h, rt_mem mem,
                           void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (!rgb && w == 0 && h == 0) {
    hipError_t e = sc->sky ? hipFree(sc->sky) : hipSuccess;
    sc->sky = nullptr;
    sc->sky_w = sc->sky_h = 0;
    return hip_fail(e, "skybox free");
  }
  if (!rgb) return fail(RT_ERR_INVALID_ARG, "skybox is NULL");
  if (w < 1 || h < 1 || w > RT_MAX_SKY_DIM || h > RT_MAX_SKY_DIM)
    return fail(RT_ERR_INVALID_ARG, "skybox %dx%d outside [1, %d]", w, h, RT_MAX_SKY_DIM);
  if (mem != RT_HOST && mem != RT_DEVICE) return fail(RT_ERR_INVALID_ARG, "mem=%d", (int)mem);
  const size_t texels = (size_t)w * h;
  if (mem == RT_HOST && !finite_all(rgb, 3 * (int64_t)texels))
    return fail(RT_ERR_INVALID_ARG, "non-finite value in the skybox");
  hipStream_t st = (hipStream_t)stream;
  // host staging (up to 4 GiB) before the scene changes: an allocation failure
  // is reported, not thrown, and leaves the scene's skybox as it was
  std::unique_ptr<float4[]> tex;
  if (mem == RT_HOST) {
    tex.reset(new (std::nothrow) float4[texels]);
    if (!tex) return fail(RT_ERR_OUT_OF_MEMORY, "skybox staging: host allocation failed");
  }
  if (sc->sky && (sc->sky_w != w || sc->sky_h != h)) {
    hipError_t e = hipFree(sc->sky);
    sc->sky = nullptr;
    sc->sky_w = sc->sky_h = 0;
    if (e != hipSuccess) return hip_fail(e, "skybox free");
  }
  if (!sc->sky) {
    hipError_t e = hipMalloc(&sc->sky, texels * sizeof(float4));
    if (e != hipSuccess) {
      sc->sky = nullptr;
      return hip_fail(e, "skybox allocation");
    }
  }
  sc->sky_w = w;
  sc->sky_h = h;
  if (mem == RT_HOST) {
    for (size_t i = 0; i < texels; ++i)
      tex[i] = make_float4(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], 0.0f);
    HIP_TRY(hipMemcpyAsync(sc->sky, tex.get(), texels * sizeof(float4), hipMemcpyHostToDevice,
                           st),
            "skybox upload");
    HIP_TRY(hipStreamSynchronize(st), "skybox upload sync");
  } else {
    HIP_TRY(launch_sky_pack(rgb, sc->sky, (int)texels, st), "skybox pack kernel");
  }
  return RT_OK;
}

rt_status rt_scene_destroy(rt_scene sc) {
  if (!sc) return RT_OK;
  hipError_t e = hipFree(sc->buffer);
  hipError_t e2 = sc->sky ? hipFree(sc->sky) : hipSuccess;
  delete sc;
  if (e == hipSuccess) e = e2;
  return hip_fail(e, "scene free");
}

rt_status rt_scene_counts(rt_scene sc, int32_t* n_spheres, int32_t* n_planes,
                          int32_t* n_lights) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (n_spheres) *n_spheres = sc->n_spheres;
  if (n_planes) *n_planes = sc->n_planes;
  if (n_lights) *n_lights = sc->n_lights;
  return RT_OK;
}

int64_t rt_records_bytes(int32_t W, int32_t H, int32_t depth) {
  if (W <= 0 || H <= 0 || depth < 0 || depth > RT_MAX_DEPTH) return -1;
  return (int64_t)W * H * (depth + 1) * (int64_t)(sizeof(int32_t) + sizeof(uint8_t));
}

static rt_status check_records(const rt_records* rec, int32_t W, int32_t H, int32_t depth) {
  if (!rec) return RT_OK;
  if (!rec->ids || !rec->lit) return fail(RT_ERR_INVALID_ARG, "records have a NULL array");
  if (rec->bytes < rt_records_bytes(W, H, depth))
    return fail(RT_ERR_INVALID_ARG, "records hold %lld bytes, %lld needed",
                (long long)rec->bytes, (long long)rt_records_bytes(W, H, depth));
  return RT_OK;
}

rt_status rt_render(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H, int32_t depth,
                    float* rgb_out, int32_t* id_out, const rt_records* rec, void* stream) {
  return rt_render_ex(sc, cam, W, H, depth, rgb_out, id_out, rec, 0, stream);
}

// The launch before a render of `kind` (hard or soft shadows): eye cones and,
// where scheduling applies, the tile order from the durations the last render
// of this kind and size recorded (remembered for RT_RENDER_CONES_READY
// renders of the same size), and the record the render may write.
static hipError_t prepare_render(rt_scene_s* sc, const CameraDev& c, bool row_order, int kind,
                                 hipStream_t stream) {
  const bool sched = !row_order && schedule_applies(*sc, c.W, c.H);
  bool ordered = false;
  hipError_t e = launch_prepare(*sc, c, sched, kind, &ordered, stream);
  const bool ok = e == hipSuccess;
  sc->order_W = (ok && ordered) ? c.W : 0;
  sc->order_H = (ok && ordered) ? c.H : 0;
  sc->rec_W = (ok && sched) ? c.W : 0;
  sc->rec_H = (ok && sched) ? c.H : 0;
  sc->sched_kind = kind;
  return e;
}

// Schedule mode of a render of `kind` at W x H after its preparation: the
// prepared order if it was made for this kind and size, and a record of its
// tile durations into the histogram set the preparation zeroed (once).
static int schedule_mode(const rt_scene_s* sc, int W, int H, int kind, bool row_order,
                         bool brute) {
  if (row_order || brute || !schedule_applies(*sc, W, H) || sc->sched_kind != kind) return 0;
  int mode = 0;
  if (sc->order_W == W && sc->order_H == H) mode |= kSchedOrdered;
  if (sc->rec_W == W && sc->rec_H == H) mode |= kSchedRecord | (sc->hist_set ? 0 : kSchedHistSet1);
  return mode;
}

static void schedule_recorded(rt_scene_s* sc, int mode, int W, int H, int kind) {
  if (!(mode & kSchedRecord)) return;
  sc->hist_set ^= 1;   // the set just filled holds this render's record
  sc->hist_W = W;
  sc->hist_H = H;
  sc->hist_kind = kind;
  sc->rec_W = sc->rec_H = 0;
}

rt_status rt_render_prepare(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H,
                            void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  rt_status st = validate_camera(cam, W, H, 0);
  if (st != RT_OK) return st;
  return hip_fail(prepare_render(sc, camera_dev(*cam, W, H), false, kSchedHard,
                                 (hipStream_t)stream),
                  "prepare launch");
}

rt_status rt_render_ex(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H, int32_t depth,
                       float* rgb_out, int32_t* id_out, const rt_records* rec, uint32_t flags,
                       void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (flags & ~(uint32_t)(RT_RENDER_NO_PREFILTER | RT_RENDER_CONES_READY | RT_RENDER_ROW_ORDER))
    return fail(RT_ERR_INVALID_ARG, "unknown render flags 0x%x", flags);
  rt_status st = validate_camera(cam, W, H, depth);
  if (st != RT_OK) return st;
  if (!rgb_out) return fail(RT_ERR_INVALID_ARG, "rgb_out is NULL");
  if ((st = check_records(rec, W, H, depth)) != RT_OK) return st;
  CameraDev c = camera_dev(*cam, W, H);
  const bool row_order = flags & RT_RENDER_ROW_ORDER;
  hipError_t e = (flags & RT_RENDER_CONES_READY)
                     ? hipSuccess
                     : prepare_render(sc, c, row_order, kSchedHard, (hipStream_t)stream);
  SceneDev s = sc->view();
  // the brute-force variant keeps row order and records nothing
  s.sched_mode = schedule_mode(sc, W, H, kSchedHard, row_order, flags & RT_RENDER_NO_PREFILTER);
  if (e == hipSuccess)
    e = launch_render(s, c, depth, rgb_out, id_out, rec ? rec->ids : nullptr,
                      rec ? rec->lit : nullptr, !(flags & RT_RENDER_NO_PREFILTER),
                      (hipStream_t)stream);
  if (e == hipSuccess) schedule_recorded(sc, s.sched_mode, W, H, kSchedHard);
  return hip_fail(e, "render launch");
}

rt_status rt_render_soft(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H,
                         int32_t depth, int32_t samples, float light_radius, float* rgb_out,
                         int32_t* id_out, uint32_t flags, void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (samples < 1 || samples > RT_MAX_SAMPLES)
    return fail(RT_ERR_INVALID_ARG, "samples %d outside [1, %d]", samples, RT_MAX_SAMPLES);
  if (!(light_radius >= 0.0f) || !std::isfinite(light_radius))
    return fail(RT_ERR_INVALID_ARG, "light_radius must be finite and >= 0");
  if (samples == 1 || light_radius == 0.0f)   // the point light
    return rt_render_ex(sc, cam, W, H, depth, rgb_out, id_out, nullptr, flags, stream);
  if (flags & ~(uint32_t)(RT_RENDER_NO_PREFILTER | RT_RENDER_ROW_ORDER))
    return fail(RT_ERR_INVALID_ARG, "unknown render flags 0x%x", flags);
  rt_status st = validate_camera(cam, W, H, depth);
  if (st != RT_OK) return st;
  if (!rgb_out) return fail(RT_ERR_INVALID_ARG, "rgb_out is NULL");
  CameraDev c = camera_dev(*cam, W, H);
  const bool row_order = flags & RT_RENDER_ROW_ORDER;
  hipError_t e = prepare_render(sc, c, row_order, kSchedSoft, (hipStream_t)stream);
  const int mode =
      schedule_mode(sc, W, H, kSchedSoft, row_order, flags & RT_RENDER_NO_PREFILTER);
  if (e == hipSuccess)
    e = launch_render_soft(*sc, c, depth, samples, light_radius, rgb_out, id_out,
                           !(flags & RT_RENDER_NO_PREFILTER), mode, (hipStream_t)stream);
  if (e == hipSuccess) schedule_recorded(sc, mode, W, H, kSchedSoft);
  return hip_fail(e, "soft render launch");
}

rt_status rt_render_counts(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H,
                           int32_t depth, int64_t* counts, uint32_t flags, void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  if (flags & ~(uint32_t)RT_RENDER_NO_PREFILTER)
    return fail(RT_ERR_INVALID_ARG, "unknown render flags 0x%x", flags);
  rt_status st = validate_camera(cam, W, H, depth);
  if (st != RT_OK) return st;
  if (!counts) return fail(RT_ERR_INVALID_ARG, "counts is NULL");
  CameraDev c = camera_dev(*cam, W, H);
  hipError_t e = launch_eye_cones(*sc, c, (hipStream_t)stream);
  if (e == hipSuccess)
    e = launch_counts(sc->view(), c, depth, (unsigned long long*)counts,
                      !(flags & RT_RENDER_NO_PREFILTER), (hipStream_t)stream);
  return hip_fail(e, "count launch");
}

rt_status rt_render_backward(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H,
                             int32_t depth, const float* grad_rgb, const rt_records* rec,
                             const rt_grads* grads, void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  rt_status st = validate_camera(cam, W, H, depth);
  if (st != RT_OK) return st;
  if (!grad_rgb) return fail(RT_ERR_INVALID_ARG, "grad_rgb is NULL");
  if (!grads) return fail(RT_ERR_INVALID_ARG, "grads is NULL");
  if ((st = check_records(rec, W, H, depth)) != RT_OK) return st;
  if (!adjoint_supported(sc->n_spheres, sc->device))
    return fail(RT_ERR_UNSUPPORTED, "rt_render_backward supports at most %d spheres, scene has %d",
                adjoint_max_spheres(sc->device), sc->n_spheres);
  CameraDev c = camera_dev(*cam, W, H);
  hipError_t e = rec ? hipSuccess : launch_eye_cones(*sc, c, (hipStream_t)stream);
  if (e == hipSuccess)
    e = launch_backward(*sc, c, depth, grad_rgb, rec ? rec->ids : nullptr,
                        rec ? rec->lit : nullptr, *grads, sc->partials, (hipStream_t)stream);
  return hip_fail(e, "backward launch");
}

rt_status rt_render_backward_static(rt_scene sc, const rt_camera* cam, int32_t W, int32_t H,
                                    int32_t depth, const float* grad_rgb, const rt_records* rec,
                                    const rt_grads* grads, void* stream) {
  if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
  rt_status st = validate_camera(cam, W, H, depth);
  if (st != RT_OK) return st;
  if (!grad_rgb) return fail(RT_ERR_INVALID_ARG, "grad_rgb is NULL");
  if (!grads) return fail(RT_ERR_INVALID_ARG, "grads is NULL");
  if ((st = check_records(rec, W, H, depth)) != RT_OK) return st;
  if (!adjoint_supported(sc->n_spheres, sc->device))
    return fail(RT_ERR_UNSUPPORTED,
                "rt_render_backward_static supports at most %d spheres, scene has %d",
                adjoint_max_spheres(sc->device), sc->n_spheres);
  CameraDev c = camera_dev(*cam, W, H);
  const size_t need = backward_partial_floats(*sc, c);
  if (need > kStaticScratchFloats)
    return fail(RT_ERR_INVALID_ARG,
                "rt_render_backward_static: %zu floats of partials (%d spheres, %d lights, "
                "%dx%d image) exceed its static scratch of %zu floats",
                need, sc->n_spheres, sc->n_lights, W, H, kStaticScratchFloats);
  float* part = nullptr;
  hipError_t e = static_scratch(sc->device, &part);
  if (e != hipSuccess) return hip_fail(e, "static scratch lookup");
  if (!rec) e = launch_eye_cones(*sc, c, (hipStream_t)stream);
  if (e == hipSuccess)
    e = launch_backward(*sc, c, depth, grad_rgb, rec ? rec->ids : nullptr,
                        rec ? rec->lit : nullptr, *grads, part, (hipStream_t)stream);
  return hip_fail(e, "backward launch");
}

}  // extern "C"
