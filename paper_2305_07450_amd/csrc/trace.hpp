// trace.hpp - per-ray device code of the Whitted tracer for gfx950.
//
// One lane owns one pixel's whole path: primary ray (paper Sections 3.2-3.3),
// closest hit over every primitive (Section 3.4.1), shading with hard shadow
// rays (Sections 3.5-3.6) and the mirror bounces (Section 3.7) in front-to-back
// form, so the path state stays in registers and no stack is needed:
//   C = sum_k T_k (A_k w_k a_k + S_k),  T_0 = 1,  T_{k+1} = T_k A_k kr_k,
//   w_k = 1 - kr_k below the bounce limit and 1 at it; a miss adds T_k * bg.
// This equals the paper's recursion  C_k = shade(a_k (1 - kr_k) + kr_k C_{k+1})
// with shade(c) = A_k c + S_k.
//
// Every kernel of the library (forward, adjoint re-trace, batch) calls these
// functions, and the library is built with -ffp-contract=off and explicit
// fmaf, so the same pixel gives the same bits in every launch shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

constexpr int kMaxDepth = 8;
constexpr int kMaxLights = 8;
constexpr int kMiss = -1;
constexpr int kNotTraced = -2;

// Pointers into one scene's packed device buffer.  Reads go through the
// constant address space so that uniform indices become scalar loads: every
// lane of a wave tests the same primitive at the same time, so the primitive
// is fetched once per wave into SGPRs and costs no VGPRs or LDS traffic.
struct SceneDev {
  const float4* geom;    // [N]   centre x y z, r^2
  const float2* rad;     // [N]   r, 1/r
  const float4* mat;     // [N+P] albedo r g b, kr (spheres, then planes)
  const float* shine;    // [N+P] specular exponent
  const float4* pgeom;   // [P]   unit normal m, offset h
  const float4* light;   // [L]   position, intensity
  int n_spheres, n_planes, n_lights, spec_model;
  float ambient, spec_strength, t_min;
  float bg_r, bg_g, bg_b;
};

// Camera basis, made on the host in double: right = R e_x, up = R e_y,
// fwd = R (0, 0, -b) with b = 1/tan(fov/2) and R = Ry(yaw) Rx(pitch).
struct CameraDev {
  float ex, ey, ez;
  float rx, ry, rz;
  float ux, uy, uz;
  float fx, fy, fz;
  float inv_s;   // 1 / min(W, H)
  int W, H;
};

#define RT_CONSTANT __attribute__((address_space(4)))

typedef float rt_v4 __attribute__((ext_vector_type(4)));
typedef float rt_v2 __attribute__((ext_vector_type(2)));

// Loads through the constant address space (uniform index -> s_load).
__device__ __forceinline__ float4 ld4(const float4* base, int i) {
  rt_v4 v = ((const RT_CONSTANT rt_v4*)base)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld2(const float2* base, int i) {
  rt_v2 v = ((const RT_CONSTANT rt_v2*)base)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ld1(const float* base, int i) {
  return ((const RT_CONSTANT float*)base)[i];
}

struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
};

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
  return fmaf(ax, bx, fmaf(ay, by, az * bz));
}

// Primary ray through pixel (x, y): viewport point (u, v) with
// u = (2x - W)/s, v = (H - 2y)/s, s = min(W, H) (the paper's NDC mapping with
// the shorter side spanning [-1, 1]), direction normalize(u right + v up + fwd).
__device__ __forceinline__ Ray primary_ray(const CameraDev& c, int x, int y) {
  float u = (float)(2 * x - c.W) * c.inv_s;
  float v = (float)(c.H - 2 * y) * c.inv_s;
  float dx = fmaf(u, c.rx, fmaf(v, c.ux, c.fx));
  float dy = fmaf(u, c.ry, fmaf(v, c.uy, c.fy));
  float dz = fmaf(u, c.rz, fmaf(v, c.uz, c.fz));
  float inv = 1.0f / __builtin_sqrtf(dot3(dx, dy, dz, dx, dy, dz));
  Ray r;
  r.ox = c.ex; r.oy = c.ey; r.oz = c.ez;
  r.dx = dx * inv; r.dy = dy * inv; r.dz = dz * inv;
  return r;
}

// Ray-sphere test, discriminant in the form of Haines et al. ("Precision
// Improvements for Ray/Sphere Intersection", Ray Tracing Gems, 2019):
// with oc = o - c and b = oc.d, the vector f = oc - b d is the offset of the
// centre from the ray, and Delta = r^2 - |f|^2.  Unlike b^2 - (|oc|^2 - r^2)
// it does not cancel when the sphere is far away, and it is insensitive to
// first order to |d| differing from 1 by rounding.  Returns |f|^2; the ray
// meets the sphere iff |f|^2 <= r^2.
__device__ __forceinline__ float sphere_ff(float4 g, const Ray& r, float& b) {
  float ocx = r.ox - g.x, ocy = r.oy - g.y, ocz = r.oz - g.z;
  b = dot3(ocx, ocy, ocz, r.dx, r.dy, r.dz);
  float fx = fmaf(-b, r.dx, ocx);
  float fy = fmaf(-b, r.dy, ocy);
  float fz = fmaf(-b, r.dz, ocz);
  return dot3(fx, fy, fz, fx, fy, fz);
}

// Nearest root above t_min (the far root when the near one is not), or +inf.
// Requires ff <= r^2.
__device__ __forceinline__ float sphere_root(float r2, float ff, float b, float t_min) {
  float sq = __builtin_sqrtf(r2 - ff);
  float t0 = -b - sq;
  float t1 = -b + sq;
  return t0 > t_min ? t0 : (t1 > t_min ? t1 : __builtin_inff());
}

// m.(o + t d) = h; a ray parallel to the plane misses.
__device__ __forceinline__ float plane_root(float4 g, const Ray& r, float t_min) {
  float den = dot3(g.x, g.y, g.z, r.dx, r.dy, r.dz);
  float t = (g.w - dot3(g.x, g.y, g.z, r.ox, r.oy, r.oz)) / den;
  return (den != 0.0f && t > t_min) ? t : __builtin_inff();
}

// Algorithmic work counters (the method's own count: every segment tests every
// primitive; a shadow ray tests primitives in ascending id order up to and
// including its first occluder).  NoCount compiles to nothing.
struct NoCount {
  __device__ __forceinline__ void tests(int, int) {}
  __device__ __forceinline__ void ray(int) {}
};

enum { kCntSphereTests = 0, kCntPlaneTests, kCntPrimary, kCntReflection, kCntShadow, kNumCounts };

struct Count {
  int c[kNumCounts] = {0, 0, 0, 0, 0};
  __device__ __forceinline__ void tests(int sph, int pl) {
    c[kCntSphereTests] += sph;
    c[kCntPlaneTests] += pl;
  }
  __device__ __forceinline__ void ray(int kind) { c[kind] += 1; }
};

// Closest hit over every primitive: smallest root, ties to the lower id
// (strict < while scanning ids in ascending order).  `from_plane` is the
// plane a mirror ray leaves (-1 otherwise): a ray reflected off a plane moves
// away from it and never meets it again, so that plane is not tested; this
// keeps FP32 rounding of the start point from re-hitting it at grazing angles.
__device__ __forceinline__ void closest_hit(const SceneDev& s, const Ray& r, float& t_best,
                                            int& id_best, int from_plane = -1) {
  t_best = __builtin_inff();
  id_best = kMiss;
  const float tmin = s.t_min;
#pragma unroll 4
  for (int i = 0; i < s.n_spheres; ++i) {
    float4 g = ld4(s.geom, i);
    float b;
    float ff = sphere_ff(g, r, b);
    if (ff <= g.w) {
      float t = sphere_root(g.w, ff, b, tmin);
      if (t < t_best) {
        t_best = t;
        id_best = i;
      }
    }
  }
  for (int j = 0; j < s.n_planes; ++j) {
    float t = plane_root(ld4(s.pgeom, j), r, tmin);
    if (t < t_best && s.n_spheres + j != from_plane) {
      t_best = t;
      id_best = s.n_spheres + j;
    }
  }
}

// Shadow ray from p towards a light at distance `dist`: blocked iff some
// primitive has a root in (t_min, dist).  Each lane stops at its first
// occluder; the wave stops when all its lanes have.
template <class Cnt>
__device__ __forceinline__ bool occluded(const SceneDev& s, const Ray& r, float dist, int self,
                                         Cnt& cnt) {
  // `self` is the primitive the ray leaves.  A shadow ray is only traced when
  // n.l > 0, i.e. it leaves that convex surface outwards and cannot meet it
  // again, so its test is skipped: in exact arithmetic it never occludes, and
  // skipping it keeps FP32 rounding of the start point from re-hitting it.
  const float tmin = s.t_min;
#pragma unroll 4
  for (int i = 0; i < s.n_spheres; ++i) {
    float4 g = ld4(s.geom, i);
    float b;
    float ff = sphere_ff(g, r, b);
    if (ff <= g.w && i != self) {
      if (sphere_root(g.w, ff, b, tmin) < dist) {
        cnt.tests(i + 1, 0);
        return true;
      }
    }
  }
  for (int j = 0; j < s.n_planes; ++j)
    if (s.n_spheres + j != self && plane_root(ld4(s.pgeom, j), r, tmin) < dist) {
      cnt.tests(s.n_spheres, j + 1);
      return true;
    }
  cnt.tests(s.n_spheres, s.n_planes);
  return false;
}

// x^e for x > 0 as exp2(e log2 x); 0 otherwise.
__device__ __forceinline__ float spec_pow(float x, float e) {
  return x > 0.0f ? exp2f(e * log2f(x)) : 0.0f;
}

// Surface point of a hit: position, outward normal, material, primitive id.
struct Surface {
  float px, py, pz;
  float nx, ny, nz;
  float ar, ag, ab, kr, shine;
  int id;
};

__device__ __forceinline__ Surface surface_at(const SceneDev& s, const Ray& r, float t, int id) {
  Surface f;
  f.px = fmaf(t, r.dx, r.ox);
  f.py = fmaf(t, r.dy, r.oy);
  f.pz = fmaf(t, r.dz, r.oz);
  f.id = id;
  if (id < s.n_spheres) {
    // (p - c) / |p - c| rather than (p - c) / r: equal on the sphere, but a
    // unit normal keeps the mirror direction unit, so FP32 rounding of the hit
    // point does not grow from bounce to bounce
    float4 g = ld4(s.geom, id);
    float vx = f.px - g.x, vy = f.py - g.y, vz = f.pz - g.z;
    float inv = 1.0f / __builtin_sqrtf(dot3(vx, vy, vz, vx, vy, vz));
    f.nx = vx * inv;
    f.ny = vy * inv;
    f.nz = vz * inv;
  } else {
    float4 g = ld4(s.pgeom, id - s.n_spheres);
    f.nx = g.x; f.ny = g.y; f.nz = g.z;
  }
  float4 m = ld4(s.mat, id);
  f.ar = m.x; f.ag = m.y; f.ab = m.z; f.kr = m.w;
  f.shine = ld1(s.shine, id);
  return f;
}

// Blinn or Phong factor before the exponent, for unit light direction l,
// view v = -d and normal n (Section 3.5).
__device__ __forceinline__ float spec_base(int model, float nx, float ny, float nz, float lx,
                                           float ly, float lz, float vx, float vy, float vz,
                                           float nl) {
  if (model == 1) {
    float two_nl = 2.0f * nl;
    float rx = fmaf(two_nl, nx, -lx);
    float ry = fmaf(two_nl, ny, -ly);
    float rz = fmaf(two_nl, nz, -lz);
    return dot3(vx, vy, vz, rx, ry, rz);
  }
  float hx = lx + vx, hy = ly + vy, hz = lz + vz;
  float hl2 = dot3(hx, hy, hz, hx, hy, hz);
  return hl2 > 0.0f ? dot3(nx, ny, nz, hx, hy, hz) / __builtin_sqrtf(hl2) : 0.0f;
}

// Light terms at a surface point: A = k_a + sum I (n.l), S = sum I k_s spec,
// over lights with n.l > 0 and no occluder; returns the lit-light mask.
template <class Cnt>
__device__ __forceinline__ uint32_t light_terms(const SceneDev& s, const Surface& f, const Ray& r,
                                                float& A, float& S, Cnt& cnt) {
  A = s.ambient;
  S = 0.0f;
  uint32_t lit = 0;
  for (int l = 0; l < s.n_lights; ++l) {
    float4 q = ld4(s.light, l);
    float lx = q.x - f.px, ly = q.y - f.py, lz = q.z - f.pz;
    float dist = __builtin_sqrtf(dot3(lx, ly, lz, lx, ly, lz));
    lx = lx / dist;
    ly = ly / dist;
    lz = lz / dist;
    float nl = dot3(f.nx, f.ny, f.nz, lx, ly, lz);
    if (nl > 0.0f) {
      Ray sr;
      sr.ox = f.px; sr.oy = f.py; sr.oz = f.pz;
      sr.dx = lx; sr.dy = ly; sr.dz = lz;
      cnt.ray(kCntShadow);
      if (!occluded(s, sr, dist, f.id, cnt)) {
        lit |= 1u << l;
        A = fmaf(q.w, nl, A);
        float x = spec_base(s.spec_model, f.nx, f.ny, f.nz, lx, ly, lz, -r.dx, -r.dy, -r.dz, nl);
        S = fmaf(q.w * s.spec_strength, spec_pow(x, f.shine), S);
      }
    }
  }
  return lit;
}

// Mirror direction about the normal (Section 3.7), renormalised so that the
// root formulas, which assume |d| = 1, stay accurate on later bounces.
__device__ __forceinline__ void reflect_ray(Ray& r, const Surface& f) {
  float dn2 = 2.0f * dot3(r.dx, r.dy, r.dz, f.nx, f.ny, f.nz);
  float dx = fmaf(-dn2, f.nx, r.dx);
  float dy = fmaf(-dn2, f.ny, r.dy);
  float dz = fmaf(-dn2, f.nz, r.dz);
  float inv = 1.0f / __builtin_sqrtf(dot3(dx, dy, dz, dx, dy, dz));
  r.dx = dx * inv;
  r.dy = dy * inv;
  r.dz = dz * inv;
  r.ox = f.px; r.oy = f.py; r.oz = f.pz;
}

// No-op sink: plain forward rendering.
struct NoRecords {
  __device__ __forceinline__ void seg(int, int) {}
  __device__ __forceinline__ void lit(int, uint32_t) {}
};

// The whole path of one pixel.  `sink.seg(k, id)` and `sink.lit(k, mask)` see
// every traced segment; the caller marks untraced segments.  Returns the
// number of segments traced.
template <class Sink, class Cnt = NoCount>
__device__ __forceinline__ int trace_path(const SceneDev& s, Ray r, int depth, float& cr,
                                          float& cg, float& cb, int& prim, Sink& sink,
                                          Cnt&& cnt = Cnt()) {
  float T = 1.0f;
  cr = 0.0f; cg = 0.0f; cb = 0.0f;
  prim = kMiss;
  int k = 0;
  int from_plane = -1;
  for (; k <= depth; ++k) {
    float t;
    int id;
    closest_hit(s, r, t, id, from_plane);
    cnt.ray(k == 0 ? kCntPrimary : kCntReflection);
    cnt.tests(s.n_spheres, s.n_planes);
    if (k == 0) prim = id;
    sink.seg(k, id);
    if (id < 0) {
      cr = fmaf(T, s.bg_r, cr);
      cg = fmaf(T, s.bg_g, cg);
      cb = fmaf(T, s.bg_b, cb);
      return k + 1;
    }
    Surface f = surface_at(s, r, t, id);
    float A, S;
    sink.lit(k, light_terms(s, f, r, A, S, cnt));
    if (k < depth) {
      float w = A * (1.0f - f.kr);
      cr = fmaf(T, fmaf(w, f.ar, S), cr);
      cg = fmaf(T, fmaf(w, f.ag, S), cg);
      cb = fmaf(T, fmaf(w, f.ab, S), cb);
      T = T * (A * f.kr);
      reflect_ray(r, f);
      from_plane = id >= s.n_spheres ? id : -1;
    } else {
      cr = fmaf(T, fmaf(A, f.ar, S), cr);
      cg = fmaf(T, fmaf(A, f.ag, S), cg);
      cb = fmaf(T, fmaf(A, f.ab, S), cb);
    }
  }
  return k;
}

}  // namespace rtk
