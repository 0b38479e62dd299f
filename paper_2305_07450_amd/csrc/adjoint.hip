// adjoint.hip - reverse mode of the render with visibility held fixed.
//
// For each pixel the path is replayed from its decisions (primitive hit by
// each segment and lit-light mask, read from records or recomputed by the
// same closest-hit and shadow code as the forward pass), giving bit-identical
// hit points.  The reverse sweep runs over the segments from the last to the
// first:
//   C = sum_k T_k (A_k w_k a_k + S_k) [+ T_K bg, or T_K sky(d_K), at a miss],
//   T_{k+1} = T_k A_k kr_k,  w_k = 1 - kr_k (k < depth), 1 (k = depth),
//   U_k = dL/dT_k = A_k (w_k g.a_k + kr_k U_{k+1}) + S_k (g_r + g_g + g_b),
// then through the Blinn/Phong light terms (Section 3.5) into the normal, the
// hit point and the light, and through p = o + t d, n = (p - c)/r, the root
// t(o, d, c) (dt/dc = n/(n.d)) and the mirror ray (Section 3.7) into the
// previous segment's ray.  Shadow occluders, radii, exponents and planes are
// constants.  A miss under a skybox (Section 3.8) also feeds the mirror
// direction d_K through the UV mapping and the bilinear weights (the texels
// and their indices are constants).
//
// Summation is deterministic: each wave reduces the contributions of one
// sphere id in a fixed order and one of its lanes adds them into the wave's
// own LDS accumulator (an LDS add instruction with no other writer, so in
// program order); each workgroup then writes one partial vector, and a
// second kernel adds the partials in a fixed order.  No two lanes or waves
// ever add into the same float.
#include <mutex>
#include <type_traits>

#include "rt_internal.hpp"

namespace rtk {

constexpr int kTileA = 8;
constexpr int kBlockA = 16;        // pixels per workgroup tile edge (2 x 2 wave tiles)
constexpr int kLdsFloats = 16384;  // 64 KiB: accumulator budget per workgroup when it fits

// Sum over the 64 lanes in a fixed order, so that runs repeat bit for bit.
// With every lane executing: DPP adds within each row of 16 (quad swaps, half
// mirror, mirror; both lanes of a pair add the same two values, so a row ends
// with one value R_r), then the row broadcasts of lanes 15 and 31, which
// leave (R3 + R2) + (R1 + R0) in lane 63 (lanes of the first rows hold
// partial or out-of-row values that are not read).  Otherwise an xor
// butterfly through the LDS crossbar.  Every lane gets the sum.
template <int kCtrl>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kCtrl,
                                                                0xf, 0xf, true));
}
__device__ __forceinline__ float wave_sum(float v) {
  if (wave_full()) {
    v = dpp_add<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141>(v);   // row_half_mirror
    v = dpp_add<0x140>(v);   // row_mirror
    v = dpp_add<0x142>(v);   // row_bcast:15
    v = dpp_add<0x143>(v);   // row_bcast:31
    return lane_read(v, 63);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// wave_sum of kN values at once, each in the same steps and order as
// wave_sum (so the same bits), with the kN chains of dependent DPP steps
// interleaved step by step so that each step's latency is hidden behind the
// other values' steps.
template <int kN>
__device__ __forceinline__ void wave_sums(float (&v)[kN]) {
  if (wave_full()) {
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0xB1>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0x4E>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0x141>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0x140>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0x142>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = dpp_add<0x143>(v[j]);
#pragma unroll
    for (int j = 0; j < kN; ++j) v[j] = lane_read(v[j], 63);
    return;
  }
#pragma unroll
  for (int j = 0; j < kN; ++j) v[j] = wave_sum(v[j]);
}

// Light terms with a fixed lit mask (no shadow rays): the same arithmetic
// and order as light_terms() in trace.hpp for the lights that were lit.
__device__ __forceinline__ void light_terms_fixed(const SceneDev& s, const Surface& f,
                                                  const Ray& r, uint32_t lit, float& A, float& S) {
  A = s.ambient;
  S = 0.0f;
  for (int l = 0; l < s.n_lights; ++l) {
    if (!((lit >> l) & 1u)) continue;
    float4 q = ld4(s.light, l);
    float lx = q.x - f.px, ly = q.y - f.py, lz = q.z - f.pz;
    float d2 = dot3(lx, ly, lz, lx, ly, lz);
    float inv = frsq(d2);
    lx *= inv;
    ly *= inv;
    lz *= inv;
    float nl = dot3(f.nx, f.ny, f.nz, lx, ly, lz);
    A = fmaf(q.w, nl, A);
    float x = spec_base(s.spec_model, f.nx, f.ny, f.nz, lx, ly, lz, -r.dx, -r.dy, -r.dz, nl);
    S = fmaf(q.w * s.spec_strength, spec_pow(x, f.shine), S);
  }
}

// Gradient with respect to the unit direction d of g . sky(d), the skybox
// colour that sky_colour() looks up: u = 1/2 + atan2(d_x, -d_z) / (2 pi),
// v = 1/2 - asin(d_y) / pi, bilinear weights (x - x0, y - y0) with
// x = u w - 1/2, y = v h - 1/2.  Within a texel cell the colour is bilinear in
// (x, y); clamped rows give equal texels and no v term.  The result is
// projected onto the plane orthogonal to d (the colour depends on the
// direction only); at the poles, where u is undefined, its u term is dropped.
__device__ __forceinline__ void sky_grad(const SceneDev& s, float dx, float dy, float dz,
                                         float gr, float gg, float gb, float& ox, float& oy,
                                         float& oz) {
  constexpr float kInvTwoPi = 0.15915494309189535f;
  constexpr float kInvPi = 0.3183098861837907f;
  const int w = s.sky_w, h = s.sky_h;
  const float u = fmaf(atan2f(dx, -dz), kInvTwoPi, 0.5f);
  const float cdy = fminf(fmaxf(dy, -1.0f), 1.0f);
  const float v = fmaf(-asinf(cdy), kInvPi, 0.5f);
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
  // g . texel
  const float c00 = gr * t00.x + gg * t00.y + gb * t00.z;
  const float c10 = gr * t10.x + gg * t10.y + gb * t10.z;
  const float c01 = gr * t01.x + gg * t01.y + gb * t01.z;
  const float c11 = gr * t11.x + gg * t11.y + gb * t11.z;
  const float dax = (1.0f - ay) * (c10 - c00) + ay * (c11 - c01);   // d/d ax
  const float day = ((1.0f - ax) * c01 + ax * c11) - ((1.0f - ax) * c00 + ax * c10);
  const float du = dax * (float)w, dv = day * (float)h;
  const float rxz = dx * dx + dz * dz;
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (rxz > 1e-12f) {
    gx = du * kInvTwoPi * (-dz / rxz);
    gz = du * kInvTwoPi * (dx / rxz);
  }
  const float cy2 = 1.0f - cdy * cdy;
  if (cy2 > 1e-12f) gy = -dv * kInvPi / sqrtf(cy2);
  const float rad = gx * dx + gy * dy + gz * dz;
  ox = gx - rad * dx;
  oy = gy - rad * dy;
  oz = gz - rad * dz;
}

// Hit distance of a known primitive: the same root the closest-hit search
// produced for it.
__device__ __forceinline__ float root_of(const SceneDev& s, const Ray& r, int id) {
  if (id < s.n_spheres) {
    float4 g = ld4(s.geom, id);
    float b;
    float ff = sphere_ff(g, r, b);
    return sphere_root(g.w, ff, b, s.t_min);
  }
  return plane_root(ld4(s.pgeom, id - s.n_spheres), r, s.t_min);
}

// Sink that keeps the decisions of a re-traced path in registers (kD: the
// depth the arrays are sized for).
template <int kD>
struct RegRecords {
  int ids[kD + 1];
  uint32_t lits[kD + 1];
  __device__ __forceinline__ void seg(int k, int id) {
    ids[k] = id;
    lits[k] = 0;
  }
  __device__ __forceinline__ void lit(int k, uint32_t m) { lits[k] = m; }
};

struct V3 {
  float x, y, z;
};

__device__ __forceinline__ float dotv(V3 a, V3 b) { return dot3(a.x, a.y, a.z, b.x, b.y, b.z); }

// kL: lights the per-lane light accumulators are sized for (a bound on the
// scene's light count, so that a 1-light scene does not hold registers for 8).
// kD: the same for the depth.  Up to depth 4 the segment loops are unrolled
// over kD, so the per-segment rays, throughputs and decisions sit in
// registers at fixed indices instead of in private memory.
template <bool kHasRecords, int kL, int kD>
__global__ __launch_bounds__(256) void adjoint_kernel(SceneDev s, CameraDev c, int depth,
                                                       const float* __restrict__ grad_rgb,
                                                       const int32_t* __restrict__ rec_ids,
                                                       const uint8_t* __restrict__ rec_lit,
                                                       float* __restrict__ partials, int stride,
                                                       int n_tiles_x, int n_tiles) {
  extern __shared__ float acc[];  // [waves][7N] sphere accumulators, then [waves][4L] lights
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const int N = s.n_spheres, L = s.n_lights;
  const int per_wave = 7 * N;
  float* my_acc = acc + wave * per_wave;
  for (int i = threadIdx.x; i < waves * per_wave; i += blockDim.x) acc[i] = 0.0f;
  __syncthreads();

  float qbar[kL][3];
  float ibar[kL];
  for (int l = 0; l < kL; ++l) {
    qbar[l][0] = qbar[l][1] = qbar[l][2] = 0.0f;
    ibar[l] = 0.0f;
  }
  const int64_t plane = (int64_t)c.W * c.H;
  // wave tiles of 8 x 8 pixels; a workgroup of `waves` waves covers a strip of
  // `waves` tiles inside a 16 x 16 block (waves 0..3 -> quadrants)
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int bx = tile % n_tiles_x, by = tile / n_tiles_x;
    for (int q = wave; q < 4; q += waves) {
      const int x = bx * kBlockA + (q & 1) * kTileA + (lane & 7);
      const int y = by * kBlockA + (q >> 1) * kTileA + (lane >> 3);
      const bool valid = x < c.W && y < c.H;
      const int64_t pix = valid ? (int64_t)y * c.W + x : 0;

      // decisions of the path
      RegRecords<kD> rr;
      int K = 0;          // segments with a hit
      bool ends_in_miss = false;
      float gr = 0.f, gg = 0.f, gb = 0.f;
      if (!kHasRecords) {
        // re-trace with the forward kernel's code; lanes outside the image
        // run along (the path code needs the whole wave), without a path
#pragma unroll
        for (int k = 0; k <= kD; ++k) rr.ids[k] = kNotTraced;
        if (wave_any(valid)) {
          float cr, cg, cb;
          int prim;
          trace_path(s, primary_ray(c, valid ? x : c.W - 1, valid ? y : c.H - 1), depth, valid,
                     cr, cg, cb, prim, rr);
        }
      }
      if (valid) {
        gr = grad_rgb[3 * pix + 0];
        gg = grad_rgb[3 * pix + 1];
        gb = grad_rgb[3 * pix + 2];
        if (kHasRecords) {
#pragma unroll
          for (int k = 0; k <= kD; ++k) {
            if (k > depth) break;
            rr.ids[k] = rec_ids[k * plane + pix];
            rr.lits[k] = rec_lit[k * plane + pix];
          }
        }
        const int n_prims = s.n_spheres + s.n_planes;
#pragma unroll
        for (int k = 0; k <= kD; ++k) {
          if (k > depth) break;
          // ids outside the scene (records of another scene) end the path
          if (rr.ids[k] >= 0 && rr.ids[k] < n_prims) {
            K = k + 1;
          } else {
            ends_in_miss = rr.ids[k] == kMiss;
            break;
          }
        }
      }

      // forward replay: ray and throughput of every hit segment, then those of
      // the segment after the last hit
      Ray rays[kD + 1];
      float Ts[kD + 1];
      // each hit segment's root, kept for the reverse sweep when the path comes
      // from records (the re-trace variant has no registers to spare: 130
      // VGPRs would leave it 3 waves per SIMD)
      float ts[kD + 1];
      Ray r_end;
      float T_end;
      {
        Ray r = primary_ray(c, valid ? x : 0, valid ? y : 0);
        float T = 1.0f;
#pragma unroll
        for (int k = 0; k <= kD; ++k) {
          if (k >= K) break;
          rays[k] = r;
          Ts[k] = T;
          const int id = rr.ids[k];
          ts[k] = root_of(s, r, id);
          Surface f = surface_at(s, r, ts[k], id);
          float A, S;
          light_terms_fixed(s, f, r, rr.lits[k], A, S);
          if (k < depth) {
            T = T * (A * f.kr);
            reflect_ray(r, f);
          }
        }
        r_end = r;
        T_end = T;
      }

      // reverse sweep
      const float gsum = gr + gg + gb;
      float U = ends_in_miss ? (gr * s.bg_r + gg * s.bg_g + gb * s.bg_b) : 0.0f;
      V3 obar = {0.f, 0.f, 0.f}, dbar = {0.f, 0.f, 0.f};
      if (s.sky && ends_in_miss) {
        // the miss shows the sky in the direction of the segment after the
        // last hit: U = g . sky(d_K), and d_K gets T_K grad_d (g . sky)
        float br, bgc, bb;
        sky_colour(s, r_end.dx, r_end.dy, r_end.dz, br, bgc, bb);
        U = gr * br + gg * bgc + gb * bb;
        if (K > 0) {
          sky_grad(s, r_end.dx, r_end.dy, r_end.dz, gr, gg, gb, dbar.x, dbar.y, dbar.z);
          dbar.x *= T_end; dbar.y *= T_end; dbar.z *= T_end;
        }
      }
#pragma unroll
      for (int k = kD; k >= 0; --k) {
        if (k > depth) continue;
        // every lane runs the same k so that the wave-wide reductions below line up
        const bool active = valid && k < K;
        int sid = -1;
        float sa0 = 0.f, sa1 = 0.f, sa2 = 0.f, skr = 0.f, sc0 = 0.f, sc1 = 0.f, sc2 = 0.f;
        if (active) {
          const Ray r = rays[k];
          const float T = Ts[k];
          const int id = rr.ids[k];
          const float t = kHasRecords ? ts[k] : root_of(s, r, id);
          Surface f = surface_at(s, r, t, id);
          float A, S;
          light_terms_fixed(s, f, r, rr.lits[k], A, S);
          const float Ga = gr * f.ar + gg * f.ag + gb * f.ab;
          float Abar, Sbar = T * gsum, krbar = 0.f, wa;
          if (k < depth) {
            const float w = 1.0f - f.kr;
            Abar = T * (w * Ga + f.kr * U);
            krbar = T * A * (U - Ga);
            wa = T * A * w;
            U = A * (w * Ga + f.kr * U) + S * gsum;
          } else {
            Abar = T * Ga;
            wa = T * A;
            U = A * Ga + S * gsum;
          }
          V3 n = {f.nx, f.ny, f.nz}, d = {r.dx, r.dy, r.dz};
          V3 nbar = {0.f, 0.f, 0.f}, pbar = {0.f, 0.f, 0.f};
          V3 dloc = {0.f, 0.f, 0.f};  // adjoint of d through the view vector
          // light terms (unrolled over kL so the accumulators stay in registers)
#pragma unroll
          for (int l = 0; l < kL; ++l) {
            if (l >= L || !((rr.lits[k] >> l) & 1u)) continue;
            float4 q = ld4(s.light, l);
            V3 lv = {q.x - f.px, q.y - f.py, q.z - f.pz};
            float d2 = dotv(lv, lv);
            float inv = frsq(d2);
            float dist = d2 * inv;
            V3 ld = {lv.x * inv, lv.y * inv, lv.z * inv};
            float nl = dotv(n, ld);
            V3 ldbar = {Abar * q.w * n.x, Abar * q.w * n.y, Abar * q.w * n.z};
            nbar.x += Abar * q.w * ld.x;
            nbar.y += Abar * q.w * ld.y;
            nbar.z += Abar * q.w * ld.z;
            float ibar_l = Abar * nl;
            float x = spec_base(s.spec_model, n.x, n.y, n.z, ld.x, ld.y, ld.z, -d.x, -d.y, -d.z,
                                nl);
            float spec = spec_pow(x, f.shine);
            ibar_l += Sbar * s.spec_strength * spec;
            if (x > 0.0f) {
              float xbar = Sbar * q.w * s.spec_strength * f.shine * spec / x;
              V3 v = {-d.x, -d.y, -d.z};
              V3 vbar = {0.f, 0.f, 0.f};
              if (s.spec_model == 1) {
                // x = v . (2 nl n - l)
                V3 rv = {2.f * nl * n.x - ld.x, 2.f * nl * n.y - ld.y, 2.f * nl * n.z - ld.z};
                vbar = {xbar * rv.x, xbar * rv.y, xbar * rv.z};
                V3 rbar = {xbar * v.x, xbar * v.y, xbar * v.z};
                float rn = dotv(rbar, n);
                nbar.x += 2.f * rn * ld.x + 2.f * nl * rbar.x;
                nbar.y += 2.f * rn * ld.y + 2.f * nl * rbar.y;
                nbar.z += 2.f * rn * ld.z + 2.f * nl * rbar.z;
                ldbar.x += 2.f * rn * n.x - rbar.x;
                ldbar.y += 2.f * rn * n.y - rbar.y;
                ldbar.z += 2.f * rn * n.z - rbar.z;
              } else {
                // x = n . h / |h|, h = l + v
                V3 h = {ld.x + v.x, ld.y + v.y, ld.z + v.z};
                float hl = __builtin_sqrtf(dotv(h, h));
                V3 hh = {h.x / hl, h.y / hl, h.z / hl};
                nbar.x += xbar * hh.x;
                nbar.y += xbar * hh.y;
                nbar.z += xbar * hh.z;
                float proj = dotv(hh, n);
                V3 hbar = {xbar * (n.x - hh.x * proj) / hl, xbar * (n.y - hh.y * proj) / hl,
                           xbar * (n.z - hh.z * proj) / hl};
                ldbar.x += hbar.x; ldbar.y += hbar.y; ldbar.z += hbar.z;
                vbar = hbar;
              }
              dloc.x -= vbar.x; dloc.y -= vbar.y; dloc.z -= vbar.z;
            }
            // l = lv / |lv|
            float lp = dotv(ld, ldbar);
            V3 lvbar = {(ldbar.x - ld.x * lp) / dist, (ldbar.y - ld.y * lp) / dist,
                        (ldbar.z - ld.z * lp) / dist};
            qbar[l][0] += lvbar.x; qbar[l][1] += lvbar.y; qbar[l][2] += lvbar.z;
            ibar[l] += ibar_l;
            pbar.x -= lvbar.x; pbar.y -= lvbar.y; pbar.z -= lvbar.z;
          }
          // mirror ray of this segment feeds segment k+1: o' = p, d' = d - 2 (d.n) n
          const float dn = dotv(d, n);
          const float nd1 = dotv(n, dbar);
          V3 dprev = {dbar.x - 2.f * nd1 * n.x, dbar.y - 2.f * nd1 * n.y,
                      dbar.z - 2.f * nd1 * n.z};
          nbar.x -= 2.f * (dn * dbar.x + nd1 * d.x);
          nbar.y -= 2.f * (dn * dbar.y + nd1 * d.y);
          nbar.z -= 2.f * (dn * dbar.z + nd1 * d.z);
          pbar.x += obar.x; pbar.y += obar.y; pbar.z += obar.z;
          // normal and root
          V3 cbar = {0.f, 0.f, 0.f};
          const bool sph = id < s.n_spheres;
          if (sph) {
            const float inv_r = ld2(s.rad, id).y;
            pbar.x += nbar.x * inv_r; pbar.y += nbar.y * inv_r; pbar.z += nbar.z * inv_r;
            cbar = {-nbar.x * inv_r, -nbar.y * inv_r, -nbar.z * inv_r};
          }
          // p = o + t d
          const float tbar = dotv(pbar, d);
          V3 onew = pbar;
          V3 dnew = {dprev.x + dloc.x + t * pbar.x, dprev.y + dloc.y + t * pbar.y,
                     dprev.z + dloc.z + t * pbar.z};
          // t(o, d, c): dt = n.(dc - do - t dd) / (n.d)  (plane: m, no dc)
          const float g = tbar / dn;
          onew.x -= g * n.x; onew.y -= g * n.y; onew.z -= g * n.z;
          dnew.x -= g * t * n.x; dnew.y -= g * t * n.y; dnew.z -= g * t * n.z;
          if (sph) {
            cbar.x += g * n.x; cbar.y += g * n.y; cbar.z += g * n.z;
            sid = id;
            sa0 = wa * gr; sa1 = wa * gg; sa2 = wa * gb;
            skr = krbar;
            sc0 = cbar.x; sc1 = cbar.y; sc2 = cbar.z;
          }
          obar = onew;
          dbar = dnew;
        }
        // scatter this segment's sphere gradients: one butterfly per distinct id
        uint64_t pending = __ballot(sid >= 0);
        while (pending) {
          const int leader = __builtin_ctzll(pending);
          const int key = __builtin_amdgcn_readlane(sid, leader);
          const bool mine = sid == key;
          float v[7] = {mine ? sa0 : 0.f, mine ? sa1 : 0.f, mine ? sa2 : 0.f, mine ? skr : 0.f,
                        mine ? sc0 : 0.f, mine ? sc1 : 0.f, mine ? sc2 : 0.f};
          wave_sums(v);
          // one lane adds to its wave's own accumulator, in program order:
          // the LDS add instruction replaces a read, an add and a write,
          // with no other writer and no change of order
          if (lane == 0) {
#pragma unroll
            for (int j = 0; j < 7; ++j) atomicAdd(&my_acc[7 * key + j], v[j]);
          }
          pending &= ~__ballot(mine);
        }
      }
    }
  }
  // light gradients: wave butterfly, then one LDS slot per wave
  __syncthreads();
  float* lacc = acc + waves * per_wave;
#pragma unroll
  for (int l = 0; l < kL; ++l) {
    if (l >= L) break;
    float v[4] = {qbar[l][0], qbar[l][1], qbar[l][2], ibar[l]};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float tot = wave_sum(v[j]);
      if (lane == 0) lacc[wave * 4 * L + 4 * l + j] = tot;
    }
  }
  __syncthreads();
  // workgroup partial = waves' accumulators added in wave order
  float* out = partials + (int64_t)blockIdx.x * stride;
  for (int i = threadIdx.x; i < per_wave; i += blockDim.x) {
    float sum = 0.0f;
    for (int w = 0; w < waves; ++w) sum += acc[w * per_wave + i];
    out[i] = sum;
  }
  for (int i = threadIdx.x; i < 4 * L; i += blockDim.x) {
    float sum = 0.0f;
    for (int w = 0; w < waves; ++w) sum += lacc[w * 4 * L + i];
    out[per_wave + i] = sum;
  }
}

// Sum the workgroup partials and scatter to the caller's arrays.  A workgroup
// owns 64 consecutive entries; its sixteen waves add every sixteenth partial
// (rows b = w, w + 16, ...; one coalesced 256-byte row read per wave per
// step), then wave 0 adds the sixteen wave sums in wave order.  The order is
// fixed, so the result does not depend on timing.  There are only about
// (7N + 4L) / 64 workgroups, so the reads are latency bound: sixteen short
// chains of rows per column group keep more of them in flight than four long
// ones.
constexpr int kReduceCols = 64;
constexpr int kReduceWaves = 16;

__global__ __launch_bounds__(64 * kReduceWaves) void reduce_kernel(const float* __restrict__ partials,
                                                      int stride, int blocks, int N, int L,
                                                      rt_grads g) {
  __shared__ float part[kReduceWaves][kReduceCols];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int total = 7 * N + 4 * L;
  const int j = blockIdx.x * kReduceCols + lane;
  float sum = 0.0f;
  if (j < total) {
#pragma unroll 8
    for (int b = wave; b < blocks; b += kReduceWaves) sum += partials[(int64_t)b * stride + j];
  }
  part[wave][lane] = sum;
  __syncthreads();
  if (wave != 0 || j >= total) return;
  sum = part[0][lane];
  for (int w = 1; w < kReduceWaves; ++w) sum += part[w][lane];
  if (j < 7 * N) {
    const int i = j / 7, c = j % 7;
    if (c < 3) {
      if (g.d_albedo) g.d_albedo[3 * i + c] = sum;
    } else if (c == 3) {
      if (g.d_refl) g.d_refl[i] = sum;
    } else {
      if (g.d_center) g.d_center[3 * i + (c - 4)] = sum;
    }
  } else {
    const int l = (j - 7 * N) / 4, c = (j - 7 * N) % 4;
    if (c < 3) {
      if (g.d_light_pos) g.d_light_pos[3 * l + c] = sum;
    } else {
      if (g.d_light_int) g.d_light_int[l] = sum;
    }
  }
}

int adjoint_blocks(int grad_stride);

// LDS a workgroup may allocate on a device, in floats (gfx950: 160 KiB),
// queried once per device.  Scenes whose accumulators do not fit the 64 KiB
// budget run one wave per workgroup with up to this much.
static int lds_limit_floats(int device) {
  static std::mutex mu;
  static int cache[kMaxDevices];
  if (device < 0 || device >= kMaxDevices) return kLdsFloats;
  std::lock_guard<std::mutex> lk(mu);
  if (!cache[device]) {
    int bytes = 0;
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
            hipSuccess ||
        bytes < (int)(kLdsFloats * sizeof(float)))
      bytes = kLdsFloats * sizeof(float);
    cache[device] = bytes / (int)sizeof(float);
  }
  return cache[device];
}

// Floats of LDS a one-wave workgroup needs: 7N sphere accumulators, 4L light
// slots and 4 spare.
static int lds_one_wave(int n_spheres, int n_lights) { return 7 * n_spheres + 4 * n_lights + 4; }

bool adjoint_supported(int n_spheres, int device) {
  return lds_one_wave(n_spheres, kMaxLights) <= lds_limit_floats(device);
}

int adjoint_max_spheres(int device) {
  return (lds_limit_floats(device) - lds_one_wave(0, kMaxLights)) / 7;
}

// Workgroups of the adjoint grid for an image: one per 16 x 16 tile, at most
// adjoint_blocks() (the partial rows the scene's buffer holds).
static int backward_blocks(const rt_scene_s& sc, const CameraDev& c, int* n_tiles_x,
                           int* n_tiles) {
  *n_tiles_x = (c.W + kBlockA - 1) / kBlockA;
  *n_tiles = *n_tiles_x * ((c.H + kBlockA - 1) / kBlockA);
  int blocks = adjoint_blocks(sc.grad_stride);
  return blocks > *n_tiles ? *n_tiles : blocks;
}

// Floats of partials one backward launch writes: a row of grad_stride floats
// per workgroup of its grid.
size_t backward_partial_floats(const rt_scene_s& sc, const CameraDev& c) {
  int n_tiles_x, n_tiles;
  return (size_t)backward_blocks(sc, c, &n_tiles_x, &n_tiles) * (size_t)sc.grad_stride;
}

// Partials of rt_render_backward_static: a file-scope device array that every
// GPU the library runs on holds until the process ends, so that the call
// needs no allocation.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in); it uses the device address that
// hipGetSymbolAddress gives on each device.
static __device__ __align__(256) float scratch[kStaticScratchFloats];

hipError_t static_scratch(int device, float** out) {
  static std::mutex mu;
  static float* addr[kMaxDevices];
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t back = cur != device ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (back != hipSuccess) return back;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = (float*)p;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_backward(const rt_scene_s& sc, const CameraDev& c, int depth,
                           const float* grad_rgb, const int32_t* rec_ids, const uint8_t* rec_lit,
                           const rt_grads& g, float* partials, hipStream_t stream) {
  const int N = sc.n_spheres, L = sc.n_lights;
  // up to four waves per workgroup within the 64 KiB budget; past it, one
  // wave with all the LDS the scene needs (adjoint_supported() checked it)
  int waves = 4;
  while (waves > 1 && waves * (7 * N + 4 * L) + 4 > kLdsFloats) --waves;
  const size_t lds = (size_t)(waves * 7 * N + waves * 4 * L + 4) * sizeof(float);
  int n_tiles_x, n_tiles;
  const int blocks = backward_blocks(sc, c, &n_tiles_x, &n_tiles);
  SceneDev s = sc.view();
  // the smallest light bucket that holds the scene's lights
  // ... and depth bucket
  auto pick_d = [&](auto with_records, auto lights) {
    constexpr bool kRec = decltype(with_records)::value;
    constexpr int kLb = decltype(lights)::value;
    if (depth <= 1) return adjoint_kernel<kRec, kLb, 1>;
    if (depth <= 2) return adjoint_kernel<kRec, kLb, 2>;
    if (depth <= 4) return adjoint_kernel<kRec, kLb, 4>;
    return adjoint_kernel<kRec, kLb, kMaxDepth>;
  };
  auto pick = [&](auto with_records) {
    if (L <= 1) return pick_d(with_records, std::integral_constant<int, 1>{});
    if (L <= 2) return pick_d(with_records, std::integral_constant<int, 2>{});
    if (L <= 4) return pick_d(with_records, std::integral_constant<int, 4>{});
    return pick_d(with_records, std::integral_constant<int, kMaxLights>{});
  };
  auto kern = rec_ids ? pick(std::true_type{}) : pick(std::false_type{});
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * waves), lds, stream, s, c, depth, grad_rgb,
                     rec_ids, rec_lit, partials, sc.grad_stride, n_tiles_x, n_tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int total = 7 * N + 4 * L;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3((total + kReduceCols - 1) / kReduceCols),
                     dim3(64 * kReduceWaves), 0, stream,
                     (const float*)partials, sc.grad_stride, blocks, N, L, g);
  return hipGetLastError();
}

}  // namespace rtk
