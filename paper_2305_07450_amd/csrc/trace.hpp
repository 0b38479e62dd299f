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
  const float4* eye_cone;    // [N]    cone of each sphere seen from the eye
  const float4* light_cone;  // [L][N] cone of each sphere seen from each light
  // o - c and r^2 of each sphere for the rays that share an origin: the eye
  // (primary rays) and each light (shadow rays, traced reversed from it).
  // Each is the FP32 difference the per-lane code would form, so a test that
  // reads it gives the same bits.  The scans and candidate loops read them
  // with scalar loads, which saves the three subtractions (and the moves that
  // feed their scalar operands) per sphere and lane.
  const float4* eye_oc;      // [N]    eye - centre, r^2 (padding: r^2 = -1)
  const float4* light_oc;    // [L][N] light - centre, r^2
  int n_spheres, n_planes, n_lights, spec_model;
  int n4;   // sphere tables padded to a multiple of kGroup (+kGroup for prefetch)
  float ambient, spec_strength, t_min;
  float bg_r, bg_g, bg_b;
  const float4* sky;     // [sky_h][sky_w] rgb, unused; NULL: plain background
  int sky_w, sky_h;
  // tile schedule of the render (see render.hip): the scene's schedule area
  // (kSchedOrder: int32 tile order; kSchedBin: uint8 duration bin per tile)
  // and what to do with it
  uint8_t* sched;
  int sched_mode;   // kSchedOrdered | kSchedRecord | kSchedHistSet1
};

// Tile schedule of a render: durations recorded in kSchedBins bins of a third
// of an octave each, for images of at most kSchedMaxTiles tiles; the layout
// of a scene's schedule area (byte offsets) and the render's mode bits.
constexpr int kSchedBins = 16;
constexpr int kSchedMaxTiles = 1 << 17;
constexpr int kSchedChunk = 1024;   // tiles per block of the preparation, per histogram
constexpr int kSchedHistChunk = 256;   // tiles per histogram (one cache line of counts)
constexpr int kSchedChunks = kSchedMaxTiles / kSchedHistChunk;
constexpr size_t kSchedOrder = 0;                                      // int32 [tiles]
constexpr size_t kSchedBin = kSchedOrder + 4 * (size_t)kSchedMaxTiles;     // uint8 [tiles]
// uint32 [2][kSchedChunks][kSchedBins]: tiles of each histogram chunk per bin
constexpr size_t kSchedHist = kSchedBin + (size_t)kSchedMaxTiles;
constexpr size_t kSchedBytes = kSchedHist + 2 * 4 * (size_t)kSchedChunks * kSchedBins;
constexpr int kSchedOrdered = 1, kSchedRecord = 2, kSchedHistSet1 = 4;
// Slot of launch position b (of n) in the order table.  Workgroups are dealt
// to the 8 XCDs in turn (b mod 8), each XCD with an L2 of its own, so the
// table keeps every XCD's positions together: an XCD reads its eighth of the
// table, not a share of every cache line of it.  A permutation of [0, n) into
// [0, 8 ceil(n / 8)), within kSchedMaxTiles for n up to it.
__host__ __device__ __forceinline__ int sched_slot(int b, int n) {
  return (b & 7) * ((n + 7) >> 3) + (b >> 3);
}

// Sphere tables (geom, eye_cone, light_cone) hold n4 = round_up(N, kGroup)
// entries plus one more group, so the loops below read kGroup spheres with
// two 64-byte scalar loads and fetch the next group while testing the current
// one.  Padding spheres can never pass: r^2 = -1 and cone threshold 2.
constexpr int kGroup = 8;
constexpr float kPadConeW = 2.0f;
constexpr float kPadR2 = -1.0f;

__host__ __device__ constexpr int pad_spheres(int n) { return (n + kGroup - 1) / kGroup * kGroup; }

// Cone of a sphere seen from a point q (the eye, or a light): unit axis a
// towards the centre and a threshold w such that every unit direction u with
// a.u < w misses the sphere.  A ray from q meets a sphere of radius r at
// distance D iff the angle to the axis is at most asin(r/D), i.e.
// a.u >= cos(theta) = sqrt(1 - r^2/D^2); w lowers cos(theta) by more than the
// FP32 error of both this test and the exact test that follows it, so the
// cone test only skips spheres the exact test would reject.  (The exact test
// accepts only if sin(angle) <= (r + O(eps D)) / D, i.e. cos(angle) >=
// cos(theta) - O(eps (r/D) / cos(theta)); the margin below is 32x that bound
// plus the rounding of the 3-term dot product and of the table.)  A point
// within 0.5% of a sphere's surface or inside it gets w = -2: every direction
// is a candidate.  Built in double, rounded once.
__device__ __forceinline__ float4 sphere_cone(double qx, double qy, double qz, double cx,
                                              double cy, double cz, double r) {
  const double eps = 1.1920928955078125e-07;   // 2^-23
  double vx = cx - qx, vy = cy - qy, vz = cz - qz;
  double D2 = vx * vx + vy * vy + vz * vz;
  double s2 = r * r / D2;
  double c2 = 1.0 - s2;
  if (!(c2 > 0.01)) return make_float4(0.0f, 0.0f, 0.0f, -2.0f);
  double D = sqrt(D2), c = sqrt(c2);
  double w = c - 64.0 * eps * sqrt(s2) / c - 16.0 * eps;
  return make_float4((float)(vx / D), (float)(vy / D), (float)(vz / D), (float)w);
}

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
typedef float rt_v16 __attribute__((ext_vector_type(16)));
// Four consecutive float4 from index i (a multiple of 4) in one scalar load.
__device__ __forceinline__ rt_v16 ld16(const float4* base, int i) {
  return ((const RT_CONSTANT rt_v16*)base)[i >> 2];
}

// 1-ulp hardware square root and reciprocal square root.  All kernels use
// these same functions, so every launch shape rounds the same way.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
};

// Surface point of a hit: position, outward normal, material, primitive id.
struct Surface {
  float px, py, pz;
  float nx, ny, nz;
  float ar, ag, ab, kr, shine;
  int id;
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
  float inv = frsq(dot3(dx, dy, dz, dx, dy, dz));
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
__device__ __forceinline__ float sphere_ff_oc(float ocx, float ocy, float ocz, const Ray& r,
                                              float& b) {
  b = dot3(ocx, ocy, ocz, r.dx, r.dy, r.dz);
  float fx = fmaf(-b, r.dx, ocx);
  float fy = fmaf(-b, r.dy, ocy);
  float fz = fmaf(-b, r.dz, ocz);
  return dot3(fx, fy, fz, fx, fy, fz);
}
__device__ __forceinline__ float sphere_ff(float4 g, const Ray& r, float& b) {
  return sphere_ff_oc(r.ox - g.x, r.oy - g.y, r.oz - g.z, r, b);
}

// Nearest root above t_min (the far root when the near one is not), or +inf.
// Requires ff <= r^2.
__device__ __forceinline__ float sphere_root(float r2, float ff, float b, float t_min) {
  float sq = fsqrt(r2 - ff);
  float t0 = -b - sq;
  float t1 = -b + sq;
  return t0 > t_min ? t0 : (t1 > t_min ? t1 : __builtin_inff());
}

// m.(o + t d) = h; a ray parallel to the plane misses.  The quotient takes
// the hardware reciprocal (1 ulp) instead of a correctly rounded division.
__device__ __forceinline__ float plane_root(float4 g, const Ray& r, float t_min) {
  float den = dot3(g.x, g.y, g.z, r.dx, r.dy, r.dz);
  float t = (g.w - dot3(g.x, g.y, g.z, r.ox, r.oy, r.oz)) * __builtin_amdgcn_rcpf(den);
  return (den != 0.0f && t > t_min) ? t : __builtin_inff();
}

// Work counters.  tests(): the method's algorithmic count (every segment
// tests every primitive; a shadow ray tests primitives in ascending id order
// up to and including its first occluder).  exec(): the exact ray-primitive
// tests this code actually runs, counted once per ray whose result can still
// matter (a live path, a shadow ray not yet blocked); pairs that a cone test
// or a wave bound decides are not counted, and neither are lanes that only
// run along.  NoCount compiles to nothing.
struct NoCount {
  __device__ __forceinline__ void tests(int, int) {}
  __device__ __forceinline__ void exec(int, int) {}
  __device__ __forceinline__ void ray(int) {}
};

enum {
  kCntSphereTests = 0,
  kCntPlaneTests,
  kCntPrimary,
  kCntReflection,
  kCntShadow,
  kCntExecSphere,
  kCntExecPlane,
  kNumCounts
};

struct Count {
  int c[kNumCounts] = {0, 0, 0, 0, 0, 0, 0};
  __device__ __forceinline__ void tests(int sph, int pl) {
    c[kCntSphereTests] += sph;
    c[kCntPlaneTests] += pl;
  }
  __device__ __forceinline__ void exec(int sph, int pl) {
    c[kCntExecSphere] += sph;
    c[kCntExecPlane] += pl;
  }
  __device__ __forceinline__ void ray(int kind) { c[kind] += 1; }
};

// ---- Wave-level helpers ---------------------------------------------------
// Branches on wave_any() are taken or skipped by the whole wave, so no exec
// mask is saved or restored, and the per-lane effect inside is applied with
// selects.  The path code below keeps every lane of a wave executing (lanes
// without work carry a `live` flag instead of branching away), which the
// cross-lane reductions of the wave bounds rely on; wave_full() checks it and
// a bound is only used when it holds.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
__device__ __forceinline__ uint64_t wave_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wave_full() { return __builtin_amdgcn_read_exec() == ~0ull; }

// The value v of the lanes with `take` when they all hold the same one, else
// -1 (also when no lane takes part).
__device__ __forceinline__ int wave_common(bool take, int v) {
  const uint64_t m = wave_mask(take);
  if (!m) return -1;
  const int v0 = __builtin_amdgcn_readlane(v, (int)__builtin_ctzll(m));
  return wave_any(take & (v != v0)) ? -1 : v0;
}
// Bit of primitive `id` in the 64-sphere chunk starting at `base` (0 when it
// lies outside the chunk or id < 0).
__device__ __forceinline__ uint64_t chunk_bit(int id, int base) {
  const unsigned k = (unsigned)(id - base);
  return k < 64u ? (1ull << k) : 0ull;
}

__device__ __forceinline__ float lane_read(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
// Minimum over all 64 lanes (all executing), as a wave-uniform value.  The
// floats are mapped to integers of the same order (the magnitude bits of
// negatives flipped), so each step is one integer min with a DPP operand:
// quad swaps, half-row and row mirrors within each row of 16, then the row
// broadcasts of lanes 15 and 31, after which lane 63 holds the minimum of all
// four rows (lanes of the first rows hold partial or out-of-row values that
// are not read).  Seven VALU instructions; four readlanes of the row results
// took eight.
__device__ __forceinline__ int float_order(float v) {
  const int i = __builtin_bit_cast(int, v);
  return i ^ ((i >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float order_float(int i) {
  return __builtin_bit_cast(float, i ^ ((i >> 31) & 0x7fffffff));
}
template <int kCtrl>
__device__ __forceinline__ int dpp_min(int v) {
  return min(v, __builtin_amdgcn_mov_dpp(v, kCtrl, 0xf, 0xf, true));
}
__device__ __forceinline__ float wave_min(float x) {
  int v = float_order(x);
  v = dpp_min<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v = dpp_min<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v = dpp_min<0x141>(v);   // row_half_mirror
  v = dpp_min<0x140>(v);   // row_mirror: every lane holds its row's minimum
  v = dpp_min<0x142>(v);   // row_bcast:15: lane 63 holds the minimum of rows 2 and 3
  v = dpp_min<0x143>(v);   // row_bcast:31: and of rows 0 and 1
  return order_float(__builtin_amdgcn_readlane(v, 63));
}

// Keeps root t0 = -b - sq, else t1 = -b + sq (sq = sqrt(r^2 - ff)), when
// above t_min and below t_best: sphere_root's choice, compared once.  Lanes
// whose line misses (ff > r^2) take a NaN root, which every comparison
// rejects, and are masked by `in` as well.
__device__ __forceinline__ void keep_nearest(bool in, float r2, float ff, float b, float tmin,
                                             int i, float& t_best, int& id_best) {
  const float sq = fsqrt(r2 - ff);
  const float t0 = -b - sq, t1 = -b + sq;
  const float t = t0 > tmin ? t0 : t1;
  const bool better = in & (t > tmin) & (t < t_best);
  t_best = better ? t : t_best;
  id_best = better ? i : id_best;
}

// Exact test of sphere i against the ray, given oc = o - c and r^2; keeps
// the nearest.
__device__ __forceinline__ void test_sphere_oc(float ocx, float ocy, float ocz, float r2, int i,
                                               const Ray& r, float tmin, float& t_best,
                                               int& id_best) {
  float b;
  float ff = sphere_ff_oc(ocx, ocy, ocz, r, b);
  const bool in = ff <= r2;
  if (wave_any(in)) keep_nearest(in, r2, ff, b, tmin, i, t_best, id_best);
}

// Exact test of sphere i (geometry g) against the ray; keeps the nearest.
__device__ __forceinline__ void test_sphere(float4 g, int i, const Ray& r, float tmin,
                                            float& t_best, int& id_best) {
  float b;
  float ff = sphere_ff(g, r, b);
  const bool in = ff <= g.w;
  if (wave_any(in)) keep_nearest(in, g.w, ff, b, tmin, i, t_best, id_best);
}

__device__ __forceinline__ float4 part(const rt_v16& v, int k) {
  return make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// Scalar-load scan of a sphere table (geom or cones): calls f(i, entry i) for
// i = lo .. hi-1 in ascending order (lo a multiple of 4, hi <= n4), reading
// kScanBlocks 64-byte blocks (4 entries each) per group and fetching the next
// group while the current one is tested; stops after a group once done()
// holds.  The tables hold one padding group of kGroup entries past n4, which
// covers the look-ahead and a last group that runs past hi.
constexpr int kScanBlocks = 1;
static_assert(4 * kScanBlocks <= kGroup && kGroup % (4 * kScanBlocks) == 0, "scan look-ahead");

template <class F, class Done>
__device__ __forceinline__ void scan_range(const float4* tab, int lo, int hi, F&& f, Done&& done) {
  rt_v16 cur[kScanBlocks];
#pragma unroll
  for (int b = 0; b < kScanBlocks; ++b) cur[b] = ld16(tab, lo + 4 * b);
  for (int i = lo; i < hi; i += 4 * kScanBlocks) {
    rt_v16 nxt[kScanBlocks];
#pragma unroll
    for (int b = 0; b < kScanBlocks; ++b) nxt[b] = ld16(tab, i + 4 * (kScanBlocks + b));
#pragma unroll
    for (int k = 0; k < 4 * kScanBlocks; ++k) f(i + k, part(cur[k >> 2], k & 3));
#pragma unroll
    for (int b = 0; b < kScanBlocks; ++b) cur[b] = nxt[b];
    if (done()) break;
  }
}
template <class F, class Done>
__device__ __forceinline__ void scan_spheres(const float4* tab, int n4, F&& f, Done&& done) {
  scan_range(tab, 0, n4, f, done);
}

// a.u - w for a cone (a, w): >= 0 inside the cone (with the cone's margin).
__device__ __forceinline__ float cone_excess(float4 a, float ux, float uy, float uz) {
  return fmaf(a.x, ux, fmaf(a.y, uy, fmaf(a.z, uz, -a.w)));
}

// ---- Wave cones: one bound for the directions of a whole wave -------------
// The rays of a wave that share an origin (primary rays from the eye, shadow
// rays reversed from one light) point in nearly the same direction.  A cone
// (axis e, half-angle phi) holding every participating direction u lets one
// lane per sphere decide, for 64 spheres at once, whether any lane can pass
// that sphere's own cone test; the other spheres are skipped for the wave.
//
// Axis: the direction of the first participating lane, or for a wider spread
// a bisector (refined_axis).  cos(phi): the least e.u over the participating
// lanes, lowered by 2e-6, which covers the FP32 error of the 3-term dot
// products of near-unit vectors, so the true angle between e and every u is
// at most phi.
struct WaveCone {
  float ex, ey, ez;
  float c, s;   // cos(phi), sin(phi)
  bool full;    // all lanes executing and some participate
  bool on;      // full, and phi small enough to be worth testing against
};

// Widest wave cone still worth its cost (cos of the half-angle).
constexpr float kWaveConeMinCos = 0.5f;

// Least e.u over the lanes with `take` (2 if none), and a lane attaining it.
__device__ __forceinline__ float least_dot(bool take, float ex, float ey, float ez, float ux,
                                           float uy, float uz, int& at) {
  const float d = take ? dot3(ex, ey, ez, ux, uy, uz) : 2.0f;
  const float m = wave_min(d);
  const uint64_t hit = wave_mask(take & (d == m));
  at = hit ? (int)__builtin_ctzll(hit) : 0;
  return m;
}

// Cones wider than this (cos of the half-angle) get a second axis: the
// bisector of the first one and the direction farthest from it, which about
// halves the angle for an elongated spread; the narrower of the two is kept.
constexpr float kRefineCos = 0.9995f;

// Axis e (unit, in/out) and the least e.u over the lanes with `take`.
__device__ __forceinline__ float refined_axis(bool take, float ux, float uy, float uz, float& ex,
                                              float& ey, float& ez) {
  int far;
  float c = least_dot(take, ex, ey, ez, ux, uy, uz, far);
  if (c < kRefineCos) {
    const float sx = ex + lane_read(ux, far), sy = ey + lane_read(uy, far),
                sz = ez + lane_read(uz, far);
    const float n2 = dot3(sx, sy, sz, sx, sy, sz);
    if (n2 > 1e-6f) {
      const float inv = frsq(n2);
      const float fx = sx * inv, fy = sy * inv, fz = sz * inv;
      int unused;
      const float c2 = least_dot(take, fx, fy, fz, ux, uy, uz, unused);
      if (c2 > c) {
        ex = fx; ey = fy; ez = fz;
        c = c2;
      }
    }
  }
  return c;
}

__device__ __forceinline__ WaveCone wave_cone(bool take, float ux, float uy, float uz) {
  WaveCone w;
  const uint64_t m = wave_mask(take);
  w.full = m != 0 && wave_full();
  w.on = w.full;
  w.ex = w.ey = w.ez = 0.0f;
  w.c = -1.0f;
  w.s = 0.0f;
  if (w.on) {
    const int f = (int)__builtin_ctzll(m);
    w.ex = lane_read(ux, f);
    w.ey = lane_read(uy, f);
    w.ez = lane_read(uz, f);
    const float c = refined_axis(take, ux, uy, uz, w.ex, w.ey, w.ez) - 2e-6f;
    w.c = c;
    w.s = fsqrt(fmaxf(fmaf(-c, c, 1.0f), 0.0f));
    w.on = c > kWaveConeMinCos;
  }
  return w;
}

// Whether some direction of the wave cone can pass the cone test of sphere
// cone (a, w) (a.u - w >= 0 in FP32).  A passing u has angle(a, u) <= alpha
// with cos(alpha) = w - 4e-6 (the FP32 error of that test and of |a|, |u|
// differing from 1), and angle(e, u) <= phi, so angle(a, e) <= alpha + phi:
// either alpha + phi >= pi (cos(alpha) <= -cos(phi)), or
// a.e >= cos(alpha + phi) = cos(alpha) cos(phi) - sin(alpha) sin(phi).  The
// 1e-5 slack is several times the rounding of this test itself.  Cones with
// w = -2 (every direction a candidate) always pass.
__device__ __forceinline__ bool cone_may_pass(const WaveCone& wc, float4 a) {
  const float ca = a.w - 4e-6f;
  const float sa = fsqrt(fmaxf(fmaf(-ca, ca, 1.0f), 0.0f));
  const float thr = fmaf(ca, wc.c, -(sa * wc.s));
  return (ca + wc.c <= 1e-6f) | (dot3(a.x, a.y, a.z, wc.ex, wc.ey, wc.ez) >= thr - 1e-5f);
}

// ---- Wave bundles: one bound for mirror rays with different origins --------
// Origins in a ball (centre m: the midpoint of the first participating lane's
// origin and the origin farthest from it; radius rho: the largest distance to
// m, raised by 1e-5 relative for rounding) and directions in a wave cone
// (e, phi), with phi < 90 degrees.  Every point
// o + t d with t >= 0 then lies in the cone with apex v = m - e rho / sin(phi),
// axis e and half-angle phi: that cone holds the ball (the ball's distance to
// its side is rho) and, being convex, every step from a point of it along a
// direction within phi of its axis.  A tiny phi is widened to asin(1e-3) so
// that the apex stays near.
struct WaveBundle {
  float vx, vy, vz;   // apex
  float ex, ey, ez;   // axis
  float c, s;         // cos(phi), sin(phi)
  float reach;        // rho / sin(phi) + rho: farthest origin from the apex
  float mx, my, mz;   // centre of the ball of origins
  float rho;          // its radius
  bool full;          // all lanes executing and some participate
  bool on;            // full, and phi below 60 degrees
};

// Widest bundle still worth its cost (cos of the half-angle).
constexpr float kBundleMinCos = 0.5f;

// Cone half-angle phi = acos(c) for a bundle whose ball is set: the apex
// rho / sin(phi) behind the ball's centre; on when phi is below 60 degrees.
__device__ __forceinline__ void bundle_apex(WaveBundle& b, float c) {
  // decided on phi itself: sin(phi) is also small when phi is near 180 degrees
  b.on = b.full && c > kBundleMinCos;
  float sn = fsqrt(fmaxf(fmaf(-c, c, 1.0f), 0.0f));
  if (sn < 1e-3f) {   // phi near 0 (c > kBundleMinCos > 0 when on)
    sn = 1e-3f;
    c = 0.9999995f;   // below sqrt(1 - 1e-6)
  }
  b.c = c;
  b.s = sn;
  const float back = b.rho / sn;
  b.vx = fmaf(-b.ex, back, b.mx);
  b.vy = fmaf(-b.ey, back, b.my);
  b.vz = fmaf(-b.ez, back, b.mz);
  b.reach = back + b.rho;
}

__device__ __forceinline__ WaveBundle wave_bundle(bool take, const Ray& r) {
  WaveBundle b;
  const uint64_t m = wave_mask(take);
  b.full = m != 0 && wave_full();
  b.on = b.full;
  b.vx = b.vy = b.vz = b.ex = b.ey = b.ez = 0.0f;
  b.c = -1.0f;
  b.s = 0.0f;
  b.reach = 0.0f;
  b.mx = b.my = b.mz = b.rho = 0.0f;
  if (b.on) {
    const int f = (int)__builtin_ctzll(m);
    float mx = lane_read(r.ox, f), my = lane_read(r.oy, f), mz = lane_read(r.oz, f);
    b.ex = lane_read(r.dx, f);
    b.ey = lane_read(r.dy, f);
    b.ez = lane_read(r.dz, f);
    // ball: first origin, then the midpoint of it and the origin farthest away
    float qx = r.ox - mx, qy = r.oy - my, qz = r.oz - mz;
    float nq2 = take ? -dot3(qx, qy, qz, qx, qy, qz) : 0.0f;
    float rho2 = wave_min(nq2);
    if (rho2 < 0.0f) {
      const uint64_t hit = wave_mask(take & (nq2 == rho2));
      const int h = hit ? (int)__builtin_ctzll(hit) : f;
      mx = 0.5f * (mx + lane_read(r.ox, h));
      my = 0.5f * (my + lane_read(r.oy, h));
      mz = 0.5f * (mz + lane_read(r.oz, h));
      qx = r.ox - mx; qy = r.oy - my; qz = r.oz - mz;
      rho2 = wave_min(take ? -dot3(qx, qy, qz, qx, qy, qz) : 0.0f);
    }
    const float rho = fmaf(fsqrt(-rho2), 1.00001f, 1e-6f);
    b.mx = mx; b.my = my; b.mz = mz;
    b.rho = rho;
    bundle_apex(b, refined_axis(take, r.dx, r.dy, r.dz, b.ex, b.ey, b.ez) - 2e-6f);
  }
  return b;
}

// Whether some ray of the bundle can meet sphere (centre g.xyz, radius rad)
// in the exact test: whether the sphere, grown by 1e-4 r + 2e-5 (D + reach)
// + 1e-5 (D = distance to the apex; many times the FP32 error of the exact
// test and of this one), meets the bundle's cone: it holds the apex, or the
// angle between its centre and the axis is at most phi + asin(r'/D).
__device__ __forceinline__ bool sphere_may_meet(const WaveBundle& b, float4 g, float rad) {
  const float wx = g.x - b.vx, wy = g.y - b.vy, wz = g.z - b.vz;
  const float inv = frsq(dot3(wx, wy, wz, wx, wy, wz));
  const float D = dot3(wx, wy, wz, wx, wy, wz) * inv;
  const float rg = fmaf(rad, 1.0001f, fmaf(2e-5f, D + b.reach, 1e-5f));
  const float sb = rg * inv;
  const float cb = fsqrt(fmaxf(fmaf(-sb, sb, 1.0f), 0.0f));
  const float ca = dot3(wx, wy, wz, b.ex, b.ey, b.ez) * inv;
  const float thr = fmaf(b.c, cb, -(b.s * sb));
  return (sb >= 1.0f) | (b.c + cb <= 1e-6f) | (ca >= thr - 1e-5f);
}

// ---- Transposed tests for waves with few live rays -------------------------
// A wave whose bound keeps many spheres but has few live rays (later bounces)
// turns the loop around: for each live ray q in turn, lane j tests sphere
// base + j against ray q (read from lane q), and a wave minimum or ballot
// folds the 64 results into lane q.  Each pair runs the same arithmetic as in
// the per-lane loops, so the results are the same bits.  Per 64 spheres a
// ray costs about kTransHitCost VALU operations in the closest-hit search and
// kTransShadowCost in a shadow test, against about kLaneHitCost and
// kLaneShadowCost per candidate sphere in the per-lane loops.
constexpr int kTransHitCost = 75, kLaneHitCost = 20;
constexpr int kTransShadowCost = 25, kLaneShadowCost = 10;
constexpr bool kTransposedHit = true, kTransposedShadow = true;

// Nearest root over the spheres base + j (j in `cand`, geometry g in lane j)
// for every ray of `rays`; strict < against each ray's running best, and the
// lowest id among equal roots, as the ascending per-lane scan gives.
//
// kLds (kernels whose workgroup is one wave): ray q comes from per-lane LDS
// slots, one broadcast read (no bank conflicts) instead of six readlanes, each
// of which takes a VALU issue slot; a wave reads its own LDS writes in order.
template <bool kLds>
__device__ __forceinline__ void transposed_hit(float4 g, uint64_t cand, int base, uint64_t rays,
                                               const Ray& r, float tmin, float& t_best,
                                               int& id_best) {
  const int lane = __lane_id();
  const bool mine = (cand >> lane) & 1u;
  __shared__ float4 s_ro[kLds ? 64 : 1], s_rd[kLds ? 64 : 1];
  if constexpr (kLds) {
    s_ro[lane] = make_float4(r.ox, r.oy, r.oz, 0.0f);
    s_rd[lane] = make_float4(r.dx, r.dy, r.dz, 0.0f);
  }
  while (rays) {
    const int q = (int)__builtin_ctzll(rays);
    rays &= rays - 1;
    Ray rq;
    if constexpr (kLds) {
      const float4 o4 = s_ro[q], d4 = s_rd[q];
      rq.ox = o4.x; rq.oy = o4.y; rq.oz = o4.z;
      rq.dx = d4.x; rq.dy = d4.y; rq.dz = d4.z;
    } else {
      rq.ox = lane_read(r.ox, q); rq.oy = lane_read(r.oy, q); rq.oz = lane_read(r.oz, q);
      rq.dx = lane_read(r.dx, q); rq.dy = lane_read(r.dy, q); rq.dz = lane_read(r.dz, q);
    }
    float b;
    const float ff = sphere_ff(g, rq, b);
    const bool in = mine & (ff <= g.w);
    const float t = in ? sphere_root(g.w, ff, b, tmin) : __builtin_inff();
    const float tm = wave_min(t);
    if (tm < __builtin_inff()) {
      const int k = (int)__builtin_ctzll(wave_mask(t == tm));
      const bool better = (lane == q) & (tm < t_best);
      t_best = better ? tm : t_best;
      id_best = better ? base + k : id_best;
    }
  }
}

// Shadow occlusion of every not yet occluded lane by the spheres base + j
// (j in `cand`; o - c and r^2 of the reversed ray in lane j); records the
// first occluder, as the ascending per-lane scan does.  kLds: as in
// transposed_hit, for the direction, limit and surface of ray q.
template <bool kLds>
__device__ __forceinline__ void transposed_shadow(float ocx, float ocy, float ocz, float r2,
                                                  uint64_t cand, int base, const Ray& rr,
                                                  float lim, int self, bool& occ, int& first) {
  const int lane = __lane_id();
  const bool mine = (cand >> lane) & 1u;
  uint64_t rays = wave_mask(!occ);
  __shared__ float4 s_sd[kLds ? 64 : 1];
  __shared__ int s_self[kLds ? 64 : 1];
  if constexpr (kLds) {
    s_sd[lane] = make_float4(rr.dx, rr.dy, rr.dz, lim);
    s_self[lane] = self;
  }
  while (rays) {
    const int q = (int)__builtin_ctzll(rays);
    rays &= rays - 1;
    Ray rq = rr;   // the origin is the light for every lane
    float limq;
    int selfq;
    if constexpr (kLds) {
      const float4 d4 = s_sd[q];
      rq.dx = d4.x; rq.dy = d4.y; rq.dz = d4.z;
      limq = d4.w;
      selfq = s_self[q];
    } else {
      rq.dx = lane_read(rr.dx, q); rq.dy = lane_read(rr.dy, q); rq.dz = lane_read(rr.dz, q);
      limq = lane_read(lim, q);
      selfq = __builtin_amdgcn_readlane(self, q);
    }
    float b;
    const float ff = sphere_ff_oc(ocx, ocy, ocz, rq, b);
    const bool in = mine & (ff <= r2) & (base + lane != selfq);
    const float sq = fsqrt(r2 - ff);
    const float t0 = -b - sq, t1 = -b + sq;
    const bool hit = in & (((t0 > 0.0f) & (t0 < limq)) | ((t1 > 0.0f) & (t1 < limq)));
    const uint64_t h = wave_mask(hit);
    if (h) {
      const bool me = lane == q;
      first = me ? base + (int)__builtin_ctzll(h) : first;
      occ = occ | me;
    }
  }
}

// Closest hit over every primitive: smallest root, ties to the lower id
// (strict < while scanning ids in ascending order).  `from_plane` is the
// plane a mirror ray leaves (-1 otherwise): a ray reflected off a plane moves
// away from it and never meets it again, so that plane is not tested; this
// keeps FP32 rounding of the start point from re-hitting it at grazing angles.
// `live` marks the lanes whose result is used; the others run along.
//
// Primary rays (kFromEye) all start at the eye, so each sphere is first
// tested against its cone seen from the eye (3 FMA-class ops and a compare);
// only directions inside the cone run the exact test.  With a wave cone, 64
// spheres at a time are first tested against the whole wave, and only the
// spheres some lane may see run the per-lane cone test.  Mirror rays are
// bounded by a wave bundle, and only the spheres it may meet run the exact
// test.  Skipped spheres are ones the exact test would reject, and the exact
// test is the same code in every path, so all paths give the same bits.
template <bool kFromEye, bool kPrefilter, class Cnt, bool kLds = false>
__device__ __forceinline__ void closest_hit(const SceneDev& s, const Ray& r, bool live,
                                            float& t_best, int& id_best, Cnt& cnt,
                                            int from_plane = -1) {
  t_best = __builtin_inff();
  id_best = kMiss;
  const float tmin = s.t_min;
  if (kFromEye && kPrefilter) {
    const WaveCone wc = wave_cone(live, r.dx, r.dy, r.dz);
    if (wc.on) {
      const int lane = __lane_id();
      for (int base = 0; base < s.n_spheres; base += 64) {
        const int j = base + lane;
        const int jc = j < s.n_spheres ? j : s.n_spheres - 1;
        const float4 a = s.eye_cone[jc];
        uint64_t m = wave_mask((j < s.n_spheres) & cone_may_pass(wc, a));
        while (m) {
          // candidate i: its cone, then (every lane's ray starting at the
          // eye) its o - c, through scalar loads (issue slots of the scalar
          // memory unit, not of the VALU, which bounds this kernel)
          const int i = base + (int)__builtin_ctzll(m);
          m &= m - 1;
          if (wave_any(live & (cone_excess(ld4(s.eye_cone, i), r.dx, r.dy, r.dz) >= 0.0f))) {
            cnt.exec(live ? 1 : 0, 0);
            const float4 oc = ld4(s.eye_oc, i);
            test_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, r, tmin, t_best, id_best);
          }
        }
      }
    } else {
      scan_spheres(
          s.eye_cone, s.n4,
          [&](int i, float4 a) {
            if (wave_any(live & (cone_excess(a, r.dx, r.dy, r.dz) >= 0.0f))) {
              cnt.exec(live ? 1 : 0, 0);
              const float4 oc = ld4(s.eye_oc, i);
              test_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, r, tmin, t_best, id_best);
            }
          },
          [] { return false; });
    }
  } else {
    const WaveBundle wb = (!kFromEye && kPrefilter) ? wave_bundle(live, r) : WaveBundle{};
    if (!kFromEye && kPrefilter && wb.full) {
      // per 64 spheres: the bundle's candidates, then the cheapest of the
      // transposed test, the per-lane candidate loop and the scalar scan
      const int lane = __lane_id();
      const uint64_t rays = wave_mask(live);
      const int n_rays = __builtin_popcountll(rays);
      for (int base = 0; base < s.n_spheres; base += 64) {
        const int j = base + lane;
        const int jc = j < s.n_spheres ? j : s.n_spheres - 1;
        const float4 g = s.geom[jc];
        bool cand = j < s.n_spheres;
        if (wb.on) cand = cand & sphere_may_meet(wb, g, s.rad[jc].x);
        uint64_t m = wave_mask(cand);
        if (kTransposedHit && n_rays * kTransHitCost < __builtin_popcountll(m) * kLaneHitCost) {
          cnt.exec(live ? __builtin_popcountll(m) : 0, 0);
          transposed_hit<kLds>(g, m, base, rays, r, tmin, t_best, id_best);
        } else if (wb.on) {
          cnt.exec(live ? __builtin_popcountll(m) : 0, 0);
          while (m) {
            const int i = base + (int)__builtin_ctzll(m);
            m &= m - 1;
            test_sphere(ld4(s.geom, i), i, r, tmin, t_best, id_best);   // scalar load
          }
        } else {
          cnt.exec(live ? min(64, s.n_spheres - base) : 0, 0);
          scan_range(
              s.geom, base, min(base + 64, s.n4),
              [&](int i, float4 gi) { test_sphere(gi, i, r, tmin, t_best, id_best); },
              [] { return false; });
        }
      }
    } else if (kFromEye) {
      // every ray starts at the eye: o - c and r^2 from the scene's table
      cnt.exec(live ? s.n_spheres : 0, 0);
      scan_spheres(
          s.eye_oc, s.n4,
          [&](int i, float4 a) { test_sphere_oc(a.x, a.y, a.z, a.w, i, r, tmin, t_best, id_best); },
          [] { return false; });
    } else {
      cnt.exec(live ? s.n_spheres : 0, 0);
      scan_spheres(
          s.geom, s.n4, [&](int i, float4 g) { test_sphere(g, i, r, tmin, t_best, id_best); },
          [] { return false; });
    }
  }
  cnt.exec(0, live ? s.n_planes : 0);
  for (int j = 0; j < s.n_planes; ++j) {
    float t = plane_root(ld4(s.pgeom, j), r, tmin);
    if (t < t_best && s.n_spheres + j != from_plane) {
      t_best = t;
      id_best = s.n_spheres + j;
    }
  }
}

// Exact occlusion test of sphere i (geometry g) on the reversed shadow ray rr
// for the lanes not yet occluded; records the first occluder.  Lanes whose
// line misses take a NaN root and are masked by `in`.
__device__ __forceinline__ void shadow_sphere_oc(float ocx, float ocy, float ocz, float r2, int i,
                                                 const Ray& rr, float lim, int self, bool& occ,
                                                 int& first) {
  float b;
  float ff = sphere_ff_oc(ocx, ocy, ocz, rr, b);
  const bool in = !occ & (ff <= r2) & (i != self);
  if (wave_any(in)) {
    float sq = fsqrt(r2 - ff);
    float t0 = -b - sq, t1 = -b + sq;
    const bool hit = in & (((t0 > 0.0f) & (t0 < lim)) | ((t1 > 0.0f) & (t1 < lim)));
    first = hit ? i : first;
    occ = occ | hit;
  }
}
// The same in a scan of every sphere that keeps `open`, the lanes not yet
// occluded, as a wave-uniform mask: the wave takes the root test when the
// sphere meets the line of some open lane, also when that is the sphere the
// lane lies on (the per-lane test then skips it), so the occlusion state and
// the surface id are read per lane only there.
__device__ __forceinline__ void shadow_sphere_open(float ocx, float ocy, float ocz, float r2, int i,
                                                   const Ray& rr, float lim, int self, bool& occ,
                                                   int& first, uint64_t& open) {
  float b;
  const float ff = sphere_ff_oc(ocx, ocy, ocz, rr, b);
  if (wave_mask(ff <= r2) & open) {
    const bool in = !occ & (ff <= r2) & (i != self);
    const float sq = fsqrt(r2 - ff);
    const float t0 = -b - sq, t1 = -b + sq;
    const bool hit = in & (((t0 > 0.0f) & (t0 < lim)) | ((t1 > 0.0f) & (t1 < lim)));
    first = hit ? i : first;
    occ = occ | hit;
    open = wave_mask(!occ);
  }
}
__device__ __forceinline__ void shadow_sphere(float4 g, int i, const Ray& rr, float lim, int self,
                                              bool& occ, int& first) {
  float b;
  float ff = sphere_ff(g, rr, b);
  const bool in = !occ & (ff <= g.w) & (i != self);
  if (wave_any(in)) {
    float sq = fsqrt(g.w - ff);
    float t0 = -b - sq, t1 = -b + sq;
    const bool hit = in & (((t0 > 0.0f) & (t0 < lim)) | ((t1 > 0.0f) & (t1 < lim)));
    first = hit ? i : first;
    occ = occ | hit;
  }
}

// Shadow ray between a surface point p and light l at distance `dist`
// (direction l_dir from p to the light): blocked iff some primitive has a
// root in (t_min, dist) along the ray from p.  Spheres are tested on the
// reversed ray from the light, u = -l_dir, where that interval becomes
// (0, dist - t_min): every shadow ray towards light l shares that origin, so
// a sphere is first tested against its cone seen from the light (and, with a
// wave cone, 64 spheres at a time against the whole wave), and only
// directions inside the cone run the exact root test.  Each lane stops at its
// first occluder (ascending id order); the wave stops when all its lanes
// have.  Lanes with `act` false take no part and report true.
//
// `self` is the primitive p lies on.  A shadow ray is only traced when
// n.l > 0, i.e. it leaves that convex surface outwards and cannot meet it
// again, so its test is skipped: in exact arithmetic it never occludes, and
// skipping it keeps FP32 rounding of p from re-hitting it.
template <bool kPrefilter, bool kDense, class Cnt, bool kLds = false>
__device__ __forceinline__ bool occluded(const SceneDev& s, int l, float4 q, const Surface& f,
                                         float lx, float ly, float lz, float dist, bool act,
                                         Cnt& cnt) {
  const float lim = dist - s.t_min;
  const float ux = -lx, uy = -ly, uz = -lz;
  const float4* cones = s.light_cone + (int64_t)l * s.n4;
  const float4* ocs = s.light_oc + (int64_t)l * s.n4;
  const int self = f.id;
  bool occ = !act;
  int first = 0;   // first occluding sphere, for the work counters
  Ray rr;
  rr.ox = q.x; rr.oy = q.y; rr.oz = q.z;
  rr.dx = ux; rr.dy = uy; rr.dz = uz;
  const WaveCone wc = kPrefilter ? wave_cone(act, ux, uy, uz) : WaveCone{};
  if (kPrefilter && kDense && wc.on) {
    // shadow rays of primary hits: dense, coherent waves; the wave cone's
    // candidates run the per-lane cone test
    const int lane = __lane_id();
    bool done = false;
    for (int base = 0; base < s.n_spheres && !done; base += 64) {
      const int j = base + lane;
      const int jc = j < s.n_spheres ? j : s.n_spheres - 1;
      const float4 a = cones[jc];
      uint64_t m = wave_mask((j < s.n_spheres) & cone_may_pass(wc, a));
      while (m) {
        // candidate i: its cone and (every reversed shadow ray starting at
        // the light) its o - c, through scalar loads (see closest_hit)
        const int i = base + (int)__builtin_ctzll(m);
        m &= m - 1;
        if (wave_any(!occ & (cone_excess(ld4(cones, i), ux, uy, uz) >= 0.0f))) {
          cnt.exec(occ ? 0 : 1, 0);
          const float4 oc = ld4(ocs, i);
          shadow_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, rr, lim, self, occ, first);
          if (!wave_any(!occ)) {   // every lane of the wave is occluded
            done = true;
            break;
          }
        }
      }
    }
  } else if (kPrefilter && !kDense && wc.full) {
    // shadow rays of mirror hits: per 64 spheres, the wave cone's candidates,
    // then the cheapest of the transposed test, the per-lane candidate loop
    // and the scalar scan
    const int lane = __lane_id();
    bool done = false;
    for (int base = 0; base < s.n_spheres && !done; base += 64) {
      const int j = base + lane;
      const int jc = j < s.n_spheres ? j : s.n_spheres - 1;
      const float4 a = cones[jc];
      // every reversed shadow ray starts at the light: this lane's sphere's
      // o - c and r^2, for the transposed test
      const float4 oc = ocs[jc];
      bool cand = j < s.n_spheres;
      if (wc.on) cand = cand & cone_may_pass(wc, a);
      uint64_t m = wave_mask(cand);
      const int n_rays = __builtin_popcountll(wave_mask(!occ));
      if (kTransposedShadow &&
          n_rays * kTransShadowCost < __builtin_popcountll(m) * kLaneShadowCost) {
        // every ray not yet blocked meets every candidate (the transposed
        // loop does not stop a ray at its first occluder within the chunk)
        cnt.exec(occ ? 0 : __builtin_popcountll(m), 0);
        transposed_shadow<kLds>(oc.x, oc.y, oc.z, oc.w, m, base, rr, lim, self, occ, first);
        done = !wave_any(!occ);
      } else if (wc.on) {
        while (m) {
          const int i = base + (int)__builtin_ctzll(m);
          m &= m - 1;
          if (wave_any(!occ & (cone_excess(ld4(cones, i), ux, uy, uz) >= 0.0f))) {
            cnt.exec(occ ? 0 : 1, 0);
            const float4 oc = ld4(ocs, i);
            shadow_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, rr, lim, self, occ, first);
            if (!wave_any(!occ)) {   // every lane of the wave is occluded
              done = true;
              break;
            }
          }
        }
      } else {
        scan_range(
            cones, base, min(base + 64, s.n4),
            [&](int i, float4 ai) {
              if (wave_any(!occ & (cone_excess(ai, ux, uy, uz) >= 0.0f))) {
                cnt.exec(occ ? 0 : 1, 0);
                const float4 oc = ld4(ocs, i);
                shadow_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, rr, lim, self, occ, first);
              }
            },
            [&] { return !wave_any(!occ); });
        done = !wave_any(!occ);
      }
    }
  } else if (!kPrefilter) {
    // every reversed shadow ray starts at the light: o - c and r^2 from the
    // scene's table
    uint64_t open = wave_mask(!occ);
    scan_spheres(
        ocs, s.n4,
        [&](int i, float4 a) {
          cnt.exec((occ || i >= s.n_spheres) ? 0 : 1, 0);   // padding spheres are no work
          shadow_sphere_open(a.x, a.y, a.z, a.w, i, rr, lim, self, occ, first, open);
        },
        [&] { return open == 0; });   // every lane of the wave is occluded
  } else {
    scan_spheres(
        cones, s.n4,
        [&](int i, float4 a) {
          if (wave_any(!occ & (cone_excess(a, ux, uy, uz) >= 0.0f))) {
            cnt.exec((occ || i >= s.n_spheres) ? 0 : 1, 0);   // padding spheres are no work
            const float4 oc = ld4(ocs, i);
            shadow_sphere_oc(oc.x, oc.y, oc.z, oc.w, i, rr, lim, self, occ, first);
          }
        },
        [&] { return !wave_any(!occ); });   // every lane of the wave is occluded
  }
  const bool by_sphere = act && occ;
  int plane_hit = -1;
  Ray sr;
  sr.ox = f.px; sr.oy = f.py; sr.oz = f.pz;
  sr.dx = lx; sr.dy = ly; sr.dz = lz;
  for (int j = 0; j < s.n_planes; ++j) {
    // computed by every lane and combined bitwise: a short-circuit here
    // becomes an exec-mask branch around the root, which cost more
    const float tp = plane_root(ld4(s.pgeom, j), sr, s.t_min);
    cnt.exec(0, occ ? 0 : 1);
    const bool hit = (!occ) & (s.n_spheres + j != self) & (tp < dist);
    plane_hit = hit ? j : plane_hit;
    occ = occ | hit;
  }
  if (act) {
    if (by_sphere)
      cnt.tests(first + 1, 0);
    else if (plane_hit >= 0)
      cnt.tests(s.n_spheres, plane_hit + 1);
    else
      cnt.tests(s.n_spheres, s.n_planes);
  }
  return occ;
}

// x^e for x > 0 as exp2(e log2 x); 0 otherwise.  The hardware base-2
// logarithm and exponential (about 1 ulp) without the library's denormal
// scaling: x <= 1 here, and results below 2^-126 only lose digits that are
// far below the image's precision.
__device__ __forceinline__ float spec_pow(float x, float e) {
  return x > 0.0f ? __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x)) : 0.0f;
}


// Hit point, unit normal and id; the material is left for surface_at or the
// caller to load (the render path loads it after the shadow rays, so that it
// is not held in registers across them).
__device__ __forceinline__ Surface surface_geom(const SceneDev& s, const Ray& r, float t, int id) {
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
    float inv = frsq(dot3(vx, vy, vz, vx, vy, vz));
    f.nx = vx * inv;
    f.ny = vy * inv;
    f.nz = vz * inv;
  } else {
    float4 g = ld4(s.pgeom, id - s.n_spheres);
    f.nx = g.x; f.ny = g.y; f.nz = g.z;
  }
  f.ar = f.ag = f.ab = f.kr = f.shine = 0.0f;
  return f;
}

// Surface point with its material.
__device__ __forceinline__ Surface surface_at(const SceneDev& s, const Ray& r, float t, int id) {
  Surface f = surface_geom(s, r, t, id);
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
  return hl2 > 0.0f ? dot3(nx, ny, nz, hx, hy, hz) * frsq(hl2) : 0.0f;
}

// ---- Soft shadows (Section 3.6.1) -------------------------------------------
// Shadow policies of the path code: point lights (one shadow ray per lit
// light), or spherical lights of radius R sampled at n points of their great
// circle facing the hit point.
struct HardShadows {
  static constexpr bool kSoft = false;
};
struct SoftShadows {
  static constexpr bool kSoft = true;
  int n;                // samples per light
  float radius;         // light radius R
  const float2* table;  // [n, rounded up to 8]: sample i in the disk basis,
                        // R times the FP32 rounding of 2 sqrt(i/n) (cos(i phi),
                        // sin(i phi)), phi the golden angle; 64-byte aligned
  int parts = 1;        // lanes sharing a pixel's samples: 1, 2 or 4, the
                        // neighbouring lanes of an aligned group
  int part = 0;         // this lane's share: the blocks of 8 samples b with
                        // b % parts == part (set per lane by the kernel)
};

// Chunks of 64 spheres whose candidate masks a soft-shadow bound keeps; a
// scene with more spheres tests every sphere for every sample.
constexpr int kSoftChunks = 4;

// An orthonormal pair perpendicular to the unit w (Duff et al., "Building an
// Orthonormal Basis, Revisited", JCGT 2017).
__device__ __forceinline__ void perp_basis(float wx, float wy, float wz, float& ax, float& ay,
                                           float& az, float& bx, float& by, float& bz) {
  const float sign = copysignf(1.0f, wz);
  const float a = -__builtin_amdgcn_rcpf(sign + wz);
  const float b = wx * wy * a;
  ax = fmaf(sign * wx * wx, a, 1.0f);
  ay = sign * b;
  az = -sign * wx;
  bx = b;
  by = fmaf(wy * wy, a, sign);
  bz = -wy;
}

// Sample rays traced together by each lane: independent chains that the
// SIMD interleaves, one ballot per sphere for the whole group, and one o - c
// per sphere, since every sample ray of a lane starts at its hit point.
constexpr int kSoftGroup = 8;

// Exact test of one sphere against a group of sample rays of the lanes, for
// the rays not yet blocked: a root in (t_min, dist) of a sphere other than
// the surface.  The arithmetic per ray is sphere_ff's.  Returns whether the
// wave took the roots (the only case in which a ray can become blocked).
__device__ __forceinline__ bool soft_blockers(float4 g, int i, const Surface& f, const float* dx,
                                              const float* dy, const float* dz,
                                              const float* dist, float tmin, int self,
                                              bool* blk) {
  const float ocx = f.px - g.x, ocy = f.py - g.y, ocz = f.pz - g.z;
  float b[kSoftGroup], ff[kSoftGroup];
  bool in[kSoftGroup];
  bool any = false;
#pragma unroll
  for (int k = 0; k < kSoftGroup; ++k) {
    b[k] = dot3(ocx, ocy, ocz, dx[k], dy[k], dz[k]);
    const float fx = fmaf(-b[k], dx[k], ocx);
    const float fy = fmaf(-b[k], dy[k], ocy);
    const float fz = fmaf(-b[k], dz[k], ocz);
    ff[k] = dot3(fx, fy, fz, fx, fy, fz);
    in[k] = !blk[k] & (ff[k] <= g.w) & (i != self);
    any |= in[k];
  }
  if (wave_any(any)) {
#pragma unroll
    for (int k = 0; k < kSoftGroup; ++k) {
      const float sq = fsqrt(in[k] ? g.w - ff[k] : 0.0f);
      const float t0 = -b[k] - sq, t1 = -b[k] + sq;
      blk[k] = blk[k] | (in[k] & (((t0 > tmin) & (t0 < dist[k])) | ((t1 > tmin) & (t1 < dist[k]))));
    }
    return true;
  }
  return false;
}

__device__ __forceinline__ bool any_open(const bool* blk) {
  bool all = true;
#pragma unroll
  for (int k = 0; k < kSoftGroup; ++k) all &= blk[k];
  return !all;
}

// Share of light l's sample points whose shadow rays from the hit point p
// reach the light, for the lanes with `act` (0 for the others).  The points
// lie on the disk of radius 2R about the light centre q perpendicular to the
// unit direction w from p to q (the light's great circle facing p), at
// q + R (a_i e1 + b_i e2) with (e1, e2) from perp_basis(w).  A sample behind
// the tangent plane at p (n.d <= 0) is blocked; otherwise its ray is blocked
// when a primitive other than the surface itself (which the ray leaves
// outwards) has a root in (t_min, |s - p|).
//
// Spheres are bounded once for all samples of the wave: every sample ray
// starts at a lane's p and points within alpha = atan(2R / |q - p|) of that
// lane's w, so the wave bundle of the hit points and light directions, with
// its cone widened by the largest alpha (less 2e-6 in cos for rounding), holds
// every sample ray, and only the spheres it may meet are tested.
//
// With sh.parts > 1 the sh.parts neighbouring lanes of a pixel (same path,
// same p) each count their share of the blocks of 8 samples, and the counts
// are added across those lanes before the division, so every split gives the
// same share.
template <bool kPrefilter>
__device__ __forceinline__ float soft_visibility(const SceneDev& s, float4 q, const Surface& f,
                                                 float lx, float ly, float lz, float dist,
                                                 bool act, const SoftShadows& sh) {
  float ax, ay, az, bx, by, bz;
  perp_basis(lx, ly, lz, ax, ay, az, bx, by, bz);
  const int self = f.id;
  // the surface every participating lane leaves, when it is the same for all
  // of them: it always passes the bound (the bundle's rays start on it) but
  // no sample ray tests it, so the candidate masks drop it
  const int wself = kPrefilter ? wave_common(act, self) : -1;
  const float tmin = s.t_min;
  uint64_t cand[kSoftChunks];
#pragma unroll
  for (int c = 0; c < kSoftChunks; ++c) cand[c] = 0;
  bool culled = false;
  if (kPrefilter && s.n_spheres <= 64 * kSoftChunks) {
    Ray cr;
    cr.ox = f.px; cr.oy = f.py; cr.oz = f.pz;
    cr.dx = lx; cr.dy = ly; cr.dz = lz;
    WaveBundle wb = wave_bundle(act, cr);
    if (wb.full && wb.c > kBundleMinCos) {
      // widen phi by the largest disk angle: cos(phi + alpha) from the cosines
      const float two_r = 2.0f * sh.radius;
      const float h = fsqrt(fmaf(dist, dist, two_r * two_r));
      const float ca = wave_min(act ? dist * __builtin_amdgcn_rcpf(h) : 2.0f) - 2e-6f;
      const float sa = fsqrt(fmaxf(fmaf(-ca, ca, 1.0f), 0.0f));
      bundle_apex(wb, fmaf(wb.c, ca, -(wb.s * sa)) - 2e-6f);
      if (wb.on) {
        const int lane = __lane_id();
#pragma unroll
        for (int c = 0; c < kSoftChunks; ++c) {
          if (64 * c < s.n_spheres) {
            const int j = 64 * c + lane;
            const int jc = j < s.n_spheres ? j : s.n_spheres - 1;
            cand[c] = wave_mask((j < s.n_spheres) & sphere_may_meet(wb, s.geom[jc], s.rad[jc].x)) &
                      ~chunk_bit(wself, 64 * c);
          }
        }
        culled = true;
      }
    }
  }
  // Planes that no sample ray of the wave can reach (bit j).  Every lane
  // taking part and not lying on plane j has its p above the plane by more
  // than 1e-4 of the terms of its plane equation and 1e-5 of its farthest
  // sample (num = h - m.p < 0 beyond its rounding), and the whole light disk
  // lies above the plane by more than 2 % of the highest such p plus 1e-5 of
  // the farthest sample.  A sample ray's segment from p to its sample point
  // then stays above the plane: descending, it would meet the plane beyond
  // the point, and these margins keep the computed root above the computed
  // distance through the FP32 error of num, den, the root and the distance;
  // ascending, the computed root is negative.  Either way the test reports
  // no block, so skipping it changes no bit.
  uint32_t far_planes = 0;
  if (kPrefilter) {
    const float reach = dist + 2.0001f * sh.radius;   // farthest sample from p
    for (int j = 0; j < s.n_planes && j < 32; ++j) {
      const float4 pg = ld4(s.pgeom, j);
      const float mn = fsqrt(dot3(pg.x, pg.y, pg.z, pg.x, pg.y, pg.z));
      const float num = pg.w - dot3(pg.x, pg.y, pg.z, f.px, f.py, f.pz);
      const float terms = fabsf(pg.x * f.px) + fabsf(pg.y * f.py) + fabsf(pg.z * f.pz) + fabsf(pg.w);
      const bool mine = act & (s.n_spheres + j != self);
      const bool clear = -num > fmaf(1e-4f, terms, 1e-5f * reach * mn);
      const float high = -wave_min(mine ? num : 0.0f);            // highest p
      const float farthest = -wave_min(mine ? -reach : 0.0f);     // farthest sample
      const float low = dot3(pg.x, pg.y, pg.z, q.x, q.y, q.z) - pg.w - 2.0001f * sh.radius * mn;
      if (!wave_any(mine & !clear) && low > fmaf(0.02f, high, 1e-5f * farthest * mn))
        far_planes |= 1u << j;
    }
  }
  int visible = 0;
  // the light centre relative to p, formed once: a sample ray's direction is
  // q - p plus the sample's offset in the disk
  const float qpx = q.x - f.px, qpy = q.y - f.py, qpz = q.z - f.pz;
  // every participating lane has the whole light disk in front of its tangent
  // plane by more than 1e-5 of its farthest sample (below): no sample is
  // behind that plane, and the per-sample test is skipped
  const bool all_front =
      kPrefilter &&
      !wave_any(act & !(dot3(f.nx, f.ny, f.nz, qpx, qpy, qpz) >
                        fmaf(2.0001f, sh.radius, 1e-5f * (dist + 2.0001f * sh.radius))));
  if (kPrefilter && culled && s.n_planes <= 32) {
    // Every sample of every participating lane is visible when no sphere is
    // a candidate, no plane is in reach, and each lane has the whole light
    // disk in front of its tangent plane by more than 1e-5 of its farthest
    // sample: the offset of a sample from q is at most 2R (the table holds
    // R times points of the disk of radius 2), so n.x > 0 for every sample
    // vector x by a margin far above the FP32 error of x, its normalisation
    // and n.d.  The sample loop would then count all n samples, and n / n is
    // exactly 1.
    uint64_t any = 0;
#pragma unroll
    for (int c = 0; c < kSoftChunks; ++c) any |= cand[c];
    const uint32_t planes = s.n_planes == 32 ? ~0u : (1u << s.n_planes) - 1u;
    if (any == 0 && (far_planes & planes) == planes && all_front) return act ? 1.0f : 0.0f;
  }
  // the table is read 8 samples (64 bytes) per scalar load; it holds a
  // multiple of 8 entries, so the last block stays inside it (entries past n
  // are read but count as blocked)
  static_assert(8 % kSoftGroup == 0, "sample groups split a table block");
  const int last_block = (sh.n - 1) >> 3;
  for (int j0 = 0; j0 < sh.n; j0 += 8 * sh.parts) {
    // this lane's block of 8 samples: with one lane a pixel the same for the
    // whole wave (a scalar load); otherwise the lanes of a pixel read
    // different blocks, and past the last block a lane reads the last one
    // and counts its samples as blocked
    const int blk = (j0 >> 3) + sh.part;
    const int i0 = 8 * blk;
    const rt_v16 tb = sh.parts == 1 ? ((const RT_CONSTANT rt_v16*)sh.table)[j0 >> 3]
                                    : ((const rt_v16*)sh.table)[min(blk, last_block)];
#pragma unroll
    for (int k0 = 0; k0 < 8; k0 += kSoftGroup) {
      if (j0 + k0 >= sh.n) break;
      float dx[kSoftGroup], dy[kSoftGroup], dz[kSoftGroup], di[kSoftGroup];
      bool blk[kSoftGroup];
#pragma unroll
      for (int k = 0; k < kSoftGroup; ++k) {
        const int kk = k0 + k;
        const float u = tb[2 * kk], v = tb[2 * kk + 1];   // already times the radius
        float x = fmaf(u, ax, fmaf(v, bx, qpx));
        float y = fmaf(u, ay, fmaf(v, by, qpy));
        float z = fmaf(u, az, fmaf(v, bz, qpz));
        const float d2 = dot3(x, y, z, x, y, z);
        const float inv = frsq(d2);
        di[k] = d2 * inv;
        dx[k] = x * inv; dy[k] = y * inv; dz[k] = z * inv;
        blk[k] = (i0 + kk >= sh.n) | !act;
      }
      if (!all_front) {
#pragma unroll
        for (int k = 0; k < kSoftGroup; ++k)
          blk[k] = blk[k] | !(dot3(f.nx, f.ny, f.nz, dx[k], dy[k], dz[k]) > 0.0f);
      }
      if (wave_any(any_open(blk))) {
        if (culled) {
#pragma unroll
          for (int c = 0; c < kSoftChunks; ++c) {
            uint64_t m = cand[c];
            while (m) {
              const int k = (int)__builtin_ctzll(m);
              m &= m - 1;
              // the samples' state changes only where the roots were taken
              if (soft_blockers(ld4(s.geom, 64 * c + k), 64 * c + k, f, dx, dy, dz, di, tmin,
                                self, blk) &&
                  !wave_any(any_open(blk)))
                m = 0;
            }
          }
        } else {
          scan_spheres(
              s.geom, s.n4,
              [&](int j, float4 g) { soft_blockers(g, j, f, dx, dy, dz, di, tmin, self, blk); },
              [&] { return !wave_any(any_open(blk)); });
        }
        for (int j = 0; j < s.n_planes; ++j) {
          if (j < 32 && ((far_planes >> j) & 1u)) continue;
          const float4 pg = ld4(s.pgeom, j);
          const bool other = s.n_spheres + j != self;
          // plane_root with the origin term, the same for every sample ray of
          // the lane, formed once
          const float num = pg.w - dot3(pg.x, pg.y, pg.z, f.px, f.py, f.pz);
#pragma unroll
          for (int k = 0; k < kSoftGroup; ++k) {
            const float den = dot3(pg.x, pg.y, pg.z, dx[k], dy[k], dz[k]);
            const float t = num * __builtin_amdgcn_rcpf(den);
            blk[k] = blk[k] | (other & (den != 0.0f) & (t > tmin) & (t < di[k]));
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kSoftGroup; ++k) visible += blk[k] ? 0 : 1;
    }
  }
  // the counts of the lanes that share the pixel: integer sums, the same in
  // any order
  if (sh.parts >= 2) visible += __builtin_amdgcn_mov_dpp(visible, 0xB1, 0xf, 0xf, true);
  if (sh.parts >= 4) visible += __builtin_amdgcn_mov_dpp(visible, 0x4E, 0xf, 0xf, true);
  return act ? (float)visible / (float)sh.n : 0.0f;
}

// Light terms at a surface point: A = k_a + sum I (n.l), S = sum I k_s spec,
// over lights with n.l > 0 and no occluder; returns the lit-light mask.
// Only lanes with `on` take part (the others get a mask of 0); the shadow
// rays of a light are traced while any lane of the wave needs one.
template <bool kPrefilter = true, bool kDense = false, class Cnt = NoCount,
          class Shadows = HardShadows, bool kLds = false>
__device__ __forceinline__ uint32_t light_terms(const SceneDev& s, const Surface& f, const Ray& r,
                                                bool on, float& A, float& S, Cnt& cnt,
                                                const Shadows& sh = Shadows()) {
  A = s.ambient;
  S = 0.0f;
  uint32_t lit = 0;
  const float shine = ld1(s.shine, f.id);
  for (int l = 0; l < s.n_lights; ++l) {
    float4 q = ld4(s.light, l);
    float lx = q.x - f.px, ly = q.y - f.py, lz = q.z - f.pz;
    float d2 = dot3(lx, ly, lz, lx, ly, lz);
    float inv = frsq(d2);
    float dist = d2 * inv;
    lx *= inv;
    ly *= inv;
    lz *= inv;
    float nl = dot3(f.nx, f.ny, f.nz, lx, ly, lz);
    const bool act = on && nl > 0.0f;
    if (wave_any(act)) {
      if constexpr (Shadows::kSoft) {
        // area light: scale by the share of sample rays that reach it
        const float vis = soft_visibility<kPrefilter>(s, q, f, lx, ly, lz, dist, act, sh);
        if (act && vis > 0.0f) {
          lit |= 1u << l;
          const float iv = q.w * vis;
          A = fmaf(iv, nl, A);
          float x = spec_base(s.spec_model, f.nx, f.ny, f.nz, lx, ly, lz, -r.dx, -r.dy, -r.dz, nl);
          S = fmaf(iv * s.spec_strength, spec_pow(x, shine), S);
        }
      } else {
        if (act) cnt.ray(kCntShadow);
        const bool occ =
            occluded<kPrefilter, kDense, Cnt, kLds>(s, l, q, f, lx, ly, lz, dist, act, cnt);
        if (act && !occ) {
          lit |= 1u << l;
          A = fmaf(q.w, nl, A);
          float x = spec_base(s.spec_model, f.nx, f.ny, f.nz, lx, ly, lz, -r.dx, -r.dy, -r.dz, nl);
          S = fmaf(q.w * s.spec_strength, spec_pow(x, shine), S);
        }
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
  float inv = frsq(dot3(dx, dy, dz, dx, dy, dz));
  r.dx = dx * inv;
  r.dy = dy * inv;
  r.dz = dz * inv;
  r.ox = f.px; r.oy = f.py; r.oz = f.pz;
}

// Colour of the skybox (Section 3.8) in unit direction d: an equirectangular
// map, longitude u = 1/2 + atan2(d_x, -d_z) / (2 pi) across its width (the
// seam behind the default camera, which looks along -z), latitude
// v = 1/2 - asin(d_y) / pi down its height (row 0 is straight up), read with
// bilinear weights between texel centres, wrapping in u and clamping in v.
// Only lanes whose ray left the scene call it; the four taps are vector loads
// of one float4 texel each.  Every index is clamped into the map, so even a
// non-finite direction reads inside it.
__device__ __forceinline__ void sky_colour(const SceneDev& s, float dx, float dy, float dz,
                                           float& r, float& g, float& b) {
  constexpr float kInvTwoPi = 0.15915494309189535f;
  constexpr float kInvPi = 0.3183098861837907f;
  const int w = s.sky_w, h = s.sky_h;
  const float u = fmaf(atan2f(dx, -dz), kInvTwoPi, 0.5f);
  const float v = fmaf(-asinf(fminf(fmaxf(dy, -1.0f), 1.0f)), kInvPi, 0.5f);
  const float x = fmaf(u, (float)w, -0.5f);
  const float y = fmaf(v, (float)h, -0.5f);
  const float fx = floorf(x), fy = floorf(y);
  const float ax = x - fx, ay = y - fy;
  int x0 = (int)fx, y0 = (int)fy;
  x0 = x0 < 0 ? x0 + w : x0;
  int x1 = x0 + 1 >= w ? x0 + 1 - w : x0 + 1;
  x0 = min(max(x0, 0), w - 1);
  x1 = min(max(x1, 0), w - 1);
  const int y1 = min(max(y0 + 1, 0), h - 1);
  y0 = min(max(y0, 0), h - 1);
  const float4 t00 = s.sky[y0 * w + x0], t10 = s.sky[y0 * w + x1];
  const float4 t01 = s.sky[y1 * w + x0], t11 = s.sky[y1 * w + x1];
  const float bx = 1.0f - ax, by = 1.0f - ay;
  r = by * (bx * t00.x + ax * t10.x) + ay * (bx * t01.x + ax * t11.x);
  g = by * (bx * t00.y + ax * t10.y) + ay * (bx * t01.y + ax * t11.y);
  b = by * (bx * t00.z + ax * t10.z) + ay * (bx * t01.z + ax * t11.z);
}

// What a ray that leaves the scene shows.  PlainBackground: the scene's
// background colour.  SkyBackground: the skybox where the scene has one
// (else the background colour); a separate instantiation, so that scenes
// without a skybox keep the kernel that has no texture lookup in it.
struct PlainBackground {
  __device__ __forceinline__ void colour(const SceneDev& s, const Ray&, float& r, float& g,
                                         float& b) const {
    r = s.bg_r; g = s.bg_g; b = s.bg_b;
  }
};
struct SkyBackground {
  __device__ __forceinline__ void colour(const SceneDev& s, const Ray& ray, float& r, float& g,
                                         float& b) const {
    if (s.sky) {
      sky_colour(s, ray.dx, ray.dy, ray.dz, r, g, b);
    } else {
      r = s.bg_r; g = s.bg_g; b = s.bg_b;
    }
  }
};

// No-op sink: plain forward rendering.
struct NoRecords {
  __device__ __forceinline__ void seg(int, int) {}
  __device__ __forceinline__ void lit(int, uint32_t) {}
};

// State of a path between segments: the ray, its throughput, the colour so
// far and the plane the ray leaves (-1 if none).
struct PathState {
  Ray r;
  float T;
  float cr, cg, cb;
  int from_plane;
};

// Segment k of a path: closest hit, light terms with shadow rays, colour
// contribution T_k (A_k w_k a_k + S_k) (or T_k bg on a miss), then the mirror
// ray when k < depth.  Only lanes with `alive` trace the segment; on return
// `alive` says whether the path goes on (a hit below the bounce limit).
// `sink.seg(k, id)` / `sink.lit(k, mask)` see the segment.  Every kernel runs
// a segment through this one function, with all lanes of the wave executing.
template <bool kFromEye, bool kPrefilter, class Sink, class Cnt, class Shadows = HardShadows,
          class Bg = PlainBackground, bool kLds = false>
__device__ __forceinline__ int trace_segment(const SceneDev& s, PathState& ps, int k, int depth,
                                             bool& alive, Sink& sink, Cnt& cnt,
                                             const Shadows& sh = Shadows()) {
  float t;
  int id;
  if (kFromEye)
    closest_hit<true, kPrefilter, Cnt, kLds>(s, ps.r, alive, t, id, cnt);
  else
    closest_hit<false, kPrefilter, Cnt, kLds>(s, ps.r, alive, t, id, cnt, ps.from_plane);
  if (alive) {
    cnt.ray(k == 0 ? kCntPrimary : kCntReflection);
    cnt.tests(s.n_spheres, s.n_planes);
    sink.seg(k, id);
    if (id < 0) {
      float br, bg, bb;
      Bg().colour(s, ps.r, br, bg, bb);
      ps.cr = fmaf(ps.T, br, ps.cr);
      ps.cg = fmaf(ps.T, bg, ps.cg);
      ps.cb = fmaf(ps.T, bb, ps.cb);
    }
  }
  const bool hit = alive && id >= 0;
  alive = hit && k < depth;
  if (wave_any(hit)) {
    // lanes without a hit shade primitive 0 along and keep nothing of it
    Surface f = surface_geom(s, ps.r, t, hit ? id : 0);
    float A, S;
    const uint32_t lit =
        light_terms<kPrefilter, kFromEye, Cnt, Shadows, kLds>(s, f, ps.r, hit, A, S, cnt, sh);
    const float4 mat = ld4(s.mat, f.id);
    f.ar = mat.x; f.ag = mat.y; f.ab = mat.z; f.kr = mat.w;
    if (hit) {
      sink.lit(k, lit);
      if (k < depth) {
        float w = A * (1.0f - f.kr);
        ps.cr = fmaf(ps.T, fmaf(w, f.ar, S), ps.cr);
        ps.cg = fmaf(ps.T, fmaf(w, f.ag, S), ps.cg);
        ps.cb = fmaf(ps.T, fmaf(w, f.ab, S), ps.cb);
        ps.T = ps.T * (A * f.kr);
        reflect_ray(ps.r, f);
        ps.from_plane = id >= s.n_spheres ? id : -1;
      } else {
        ps.cr = fmaf(ps.T, fmaf(A, f.ar, S), ps.cr);
        ps.cg = fmaf(ps.T, fmaf(A, f.ag, S), ps.cg);
        ps.cb = fmaf(ps.T, fmaf(A, f.ab, S), ps.cb);
      }
    }
  }
  return id;
}

// The whole path of one pixel in one lane; lanes with `live` false (outside
// the image) run along without a path, so that every lane of the wave
// executes the segment code together.  `sink.seg(k, id)` and
// `sink.lit(k, mask)` see every traced segment; the caller marks untraced
// segments.  Returns the number of segments traced (0 when not live).
// kLds: the transposed tests pass rays through LDS slots indexed by lane
// alone, so only a kernel whose workgroup is a single wave may set it.
template <class Sink, class Cnt = NoCount, bool kPrefilter = true, class Shadows = HardShadows,
          class Bg = PlainBackground, bool kLds = false>
__device__ __forceinline__ int trace_path(const SceneDev& s, Ray r, int depth, bool live,
                                          float& cr, float& cg, float& cb, int& prim, Sink& sink,
                                          Cnt&& cnt = Cnt(), const Shadows& sh = Shadows()) {
  PathState ps;
  ps.r = r;
  ps.T = 1.0f;
  ps.cr = 0.0f; ps.cg = 0.0f; ps.cb = 0.0f;
  ps.from_plane = -1;
  bool alive = live;
  prim = trace_segment<true, kPrefilter, Sink, Cnt, Shadows, Bg, kLds>(s, ps, 0, depth, alive,
                                                                          sink, cnt, sh);
  int traced = live ? 1 : 0;
  for (int k = 1; k <= depth; ++k) {
    if (!wave_any(alive)) break;
    traced = alive ? k + 1 : traced;
    trace_segment<false, kPrefilter, Sink, Cnt, Shadows, Bg, kLds>(s, ps, k, depth, alive, sink,
                                                                   cnt, sh);
  }
  cr = ps.cr; cg = ps.cg; cb = ps.cb;
  return traced;
}

}  // namespace rtk
