/*
 * rt_oracle.c - FP64 CPU reference Whitted ray tracer.
 *
 * TEST INFRASTRUCTURE ONLY (see rt_oracle.h).  Plain, slow and direct:
 *   - one pixel at a time, every primitive tested by every ray, no acceleration
 *     structure (the paper's brute force, Sections 3.4.1 and 3.6);
 *   - reflections by recursion, in the order of the paper's reflection
 *     pseudocode (Section 3.7.1), not the iterative form a GPU needs;
 *   - double precision throughout, no fast-math, no FMA contraction.
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - pixel (x, y) maps to NDC with no half-pixel offset (Section 3.2 worked
 *     example: the centre pixel lands exactly on the viewport origin);
 *   - the field of view spans the shorter image side (the NDC listing);
 *   - the view direction is normalize(P - C), towards the scene (Section 3.3);
 *   - scene frame: x right, y up, the camera looks down -z; yaw turns about +y,
 *     pitch about +x, applied pitch first (d = Ry(yaw) Rx(pitch) d0);
 *   - sphere root: textbook quadratic; nearest root above t_min, else the far
 *     root above t_min (a ray that starts inside a sphere leaves it);
 *   - ties in hit distance go to the lower primitive id (spheres 0..N-1, then
 *     planes N..N+P-1);
 *   - one reflectivity per body in the paper is split into a specular exponent
 *     and a mix ratio kr in [0, 1] used directly as the reflection ratio;
 *   - shade(c) = c * A + S, with A = ambient + sum over lit lights of I (n.L)
 *     and S = sum over lit lights of I k_s spec (white lights, no falloff);
 *   - a light with n.L <= 0 gets no diffuse, no specular and no shadow ray;
 *   - occluded iff some primitive has a root in (t_min, |q - p|);
 *   - soft shadows (Section 3.6.1): the light's sample points lie on the disk
 *     about q perpendicular to the direction from p, at radius 2 R sqrt(i/n)
 *     and angle i times the golden angle, as printed; the disk's in-plane
 *     orientation, which the paper does not fix, follows Duff et al. (2017);
 *     "blocked / total" is read as the share of light removed, so diffuse
 *     and specular are scaled by the unblocked share; a sample behind the
 *     tangent plane at p is blocked; the shading direction is the centre's;
 *   - the view vector on every bounce is minus the incoming ray direction;
 *   - a miss returns the background colour (black by default), or with a
 *     skybox (Section 3.8) the map's colour in the ray's direction by the
 *     textbook spherical UV mapping (longitude from atan2, latitude from
 *     asin, straight ahead at the map's centre), filtered bilinearly: the
 *     paper names UV mapping but gives neither the axes nor the filter.
 */
#include "rt_oracle.h"

#include <math.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double OR_PI = 3.14159265358979323846;

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void normalize3(double v[3]) {
  double len = sqrt(dot3(v, v));
  v[0] /= len;
  v[1] /= len;
  v[2] /= len;
}

/* ---- Sections 3.2, 3.2.1 and 3.3: camera, viewport and primary rays ------ */

/* Section 3.2: the shorter window side spans [-1, 1] of the viewport and
 * screen rows grow downwards.  A pixel's viewport coordinates are therefore
 * its offset from the image centre (W/2, H/2), in units of half the shorter
 * side, with the row offset negated so that up is positive.  The worked
 * example of that section (the centre pixel of 1280x720 at the origin) has no
 * half-pixel offset, and neither has this mapping. */
static void ndc_coords(int32_t W, int32_t H, int32_t x, int32_t y, double* u, double* v) {
  double half_short = 0.5 * (double)(W < H ? W : H);
  *u = ((double)x - 0.5 * (double)W) / half_short;
  *v = (0.5 * (double)H - (double)y) / half_short;
}

void or_camera_ray(const or_camera* cam, int32_t W, int32_t H, int32_t x, int32_t y,
                   double o[3], double d[3]) {
  double u, v;
  ndc_coords(W, H, x, y, &u, &v);
  /* Section 3.2.1: camera distance b = 1 / tan(alpha / 2) from the viewport. */
  double alpha = cam->fov_deg * OR_PI / 180.0;
  double b = 1.0 / tan(alpha / 2.0);
  /* Section 3.3: viewport in the xy plane through the origin, pixel P = (u, v, 0),
   * camera C = (0, 0, -b); direction P - C = (u, v, b) in the paper's frame,
   * whose forward axis is +z.  The scene frame looks down -z, so the forward
   * component changes sign. */
  double d0[3] = {u, v, -b};
  normalize3(d0);
  /* Rotate by pitch (about +x), then yaw (about +y). */
  double pitch = cam->pitch_deg * OR_PI / 180.0, yaw = cam->yaw_deg * OR_PI / 180.0;
  double cp = cos(pitch), sp = sin(pitch), cy = cos(yaw), sy = sin(yaw);
  double d1[3] = {d0[0], cp * d0[1] - sp * d0[2], sp * d0[1] + cp * d0[2]};
  d[0] = cy * d1[0] + sy * d1[2];
  d[1] = d1[1];
  d[2] = -sy * d1[0] + cy * d1[2];
  o[0] = cam->eye[0];
  o[1] = cam->eye[1];
  o[2] = cam->eye[2];
}

/* ---- Section 3.4.1: intersections and the closest hit ------------------- */

/* |o + t d - c|^2 = r^2 with |d| = 1:  t^2 + 2 b t + q = 0,  b = (o-c).d,
 * q = |o-c|^2 - r^2.  Roots -b -/+ sqrt(b^2 - q). */
int or_sphere_root(const double o[3], const double d[3], const double* g, double t_min,
                   double* t) {
  double oc[3] = {o[0] - g[0], o[1] - g[1], o[2] - g[2]};
  double b = dot3(oc, d);
  double q = dot3(oc, oc) - g[3] * g[3];
  double disc = b * b - q;
  if (disc < 0.0) return 0;
  double s = sqrt(disc);
  double t0 = -b - s, t1 = -b + s;
  if (t0 > t_min) {
    *t = t0;
    return 1;
  }
  if (t1 > t_min) {
    *t = t1;
    return 1;
  }
  return 0;
}

/* m.(o + t d) = h  ->  t = (h - m.o) / (m.d); a ray parallel to the plane misses. */
int or_plane_root(const double o[3], const double d[3], const double* g, double t_min,
                  double* t) {
  double den = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
  if (den == 0.0) return 0;
  double tt = (g[3] - (g[0] * o[0] + g[1] * o[1] + g[2] * o[2])) / den;
  if (tt > t_min) {
    *t = tt;
    return 1;
  }
  return 0;
}

/* Every primitive is tested; the nearest root wins, ties to the lower id. */
int32_t or_closest_hit(const or_scene* s, const double o[3], const double d[3], double* t,
                       int64_t* tests) {
  int32_t best = OR_MISS;
  double best_t = INFINITY, tt;
  for (int32_t i = 0; i < s->n_spheres; ++i) {
    if (or_sphere_root(o, d, s->sphere_geom + 4 * i, s->t_min, &tt) && tt < best_t) {
      best_t = tt;
      best = i;
    }
  }
  for (int32_t j = 0; j < s->n_planes; ++j) {
    if (or_plane_root(o, d, s->plane_geom + 4 * j, s->t_min, &tt) && tt < best_t) {
      best_t = tt;
      best = s->n_spheres + j;
    }
  }
  if (tests) {
    tests[OR_CNT_SPHERE_TESTS] += s->n_spheres;
    tests[OR_CNT_PLANE_TESTS] += s->n_planes;
  }
  *t = best_t;
  return best;
}

/* ---- Section 3.6: hard cast shadows ------------------------------------- */

/* Shadow ray from p towards the light: any primitive with a root between
 * t_min and the light distance blocks it; the scan stops at the first one. */
static int in_cast_shadow(const or_scene* s, const double p[3], const double l[3], double dist,
                          int64_t* tests) {
  double tt;
  for (int32_t i = 0; i < s->n_spheres; ++i) {
    if (tests) tests[OR_CNT_SPHERE_TESTS] += 1;
    if (or_sphere_root(p, l, s->sphere_geom + 4 * i, s->t_min, &tt) && tt < dist) return 1;
  }
  for (int32_t j = 0; j < s->n_planes; ++j) {
    if (tests) tests[OR_CNT_PLANE_TESTS] += 1;
    if (or_plane_root(p, l, s->plane_geom + 4 * j, s->t_min, &tt) && tt < dist) return 1;
  }
  return 0;
}

/* ---- Section 3.6.1: soft shadows ---------------------------------------- */

/* An orthonormal pair (b1, b2) spanning the plane perpendicular to the unit
 * vector w, by the branchless construction of Duff et al., "Building an
 * Orthonormal Basis, Revisited" (JCGT 6(1), 2017). */
static void perp_basis(const double w[3], double b1[3], double b2[3]) {
  double sign = copysign(1.0, w[2]);
  double a = -1.0 / (sign + w[2]);
  double b = w[0] * w[1] * a;
  b1[0] = 1.0 + sign * w[0] * w[0] * a;
  b1[1] = sign * b;
  b1[2] = -sign * w[0];
  b2[0] = b;
  b2[1] = sign + w[1] * w[1] * a;
  b2[2] = -w[1];
}

/* Fraction of the light's sample points visible from p.  The light is a
 * sphere of radius R about q; its great circle facing p is the disk about q
 * perpendicular to w = (q - p)/|q - p|.  Point i of n follows the sunflower
 * arrangement (Vogel): radius 2 R sqrt(i/n) and angle i * phi, phi the golden
 * angle pi (3 - sqrt 5), measured from b1 towards b2.  A point's shadow ray
 * from p is blocked when it points into the surface (n.d <= 0: the point lies
 * behind the tangent plane at p) or when some primitive has a root in
 * (t_min, |s - p|); the fraction is unblocked / n. */
static double soft_visibility(const or_scene* s, const double p[3], const double n[3],
                              const double q[3], const double w[3], int64_t* tests) {
  const int32_t ns = s->shadow_samples;
  const double phi = OR_PI * (3.0 - sqrt(5.0));
  double b1[3], b2[3];
  perp_basis(w, b1, b2);
  int32_t visible = 0;
  for (int32_t i = 0; i < ns; ++i) {
    double r = 2.0 * s->light_radius * sqrt((double)i / (double)ns);
    double th = (double)i * phi;
    double c = cos(th), sn = sin(th);
    double pt[3], d[3];
    for (int k = 0; k < 3; ++k) pt[k] = q[k] + r * (c * b1[k] + sn * b2[k]);
    for (int k = 0; k < 3; ++k) d[k] = pt[k] - p[k];
    double dist = sqrt(dot3(d, d));
    for (int k = 0; k < 3; ++k) d[k] /= dist;
    if (!(dot3(n, d) > 0.0)) continue;
    if (tests) tests[OR_CNT_SHADOW_RAYS] += 1;
    if (!in_cast_shadow(s, p, d, dist, tests)) ++visible;
  }
  return (double)visible / (double)ns;
}

/* ---- Section 3.5: Phong / Blinn-Phong local illumination ---------------- */

/* Light terms at a hit point: A (multiplies the surface colour) and S (added,
 * white).  Ambient is a constant share of the colour (Section 3.5.1); diffuse is
 * n.L (Section 3.5.1); specular is Phong's reflect-vector form (the Phong
 * pseudocode in Section 3.5.1) or Blinn's halfway-vector form (Section 3.5.2),
 * raised to the body's exponent.  Returns the lit-light bitmask. */
static uint32_t light_terms(const or_scene* s, const double p[3], const double n[3],
                            const double view[3], double shine, double* A, double* S,
                            int64_t* tests) {
  uint32_t lit = 0;
  *A = s->ambient;
  *S = 0.0;
  for (int32_t l = 0; l < s->n_lights; ++l) {
    const double* q = s->light + 4 * l;
    double ld[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double dist = sqrt(dot3(ld, ld));
    ld[0] /= dist;
    ld[1] /= dist;
    ld[2] /= dist;
    double nl = dot3(n, ld);
    if (!(nl > 0.0)) continue;
    /* the share of the light that reaches p: 0 or 1 for a point light, the
     * visible fraction of the samples for an area light (Section 3.6.1) */
    double vis;
    if (s->shadow_samples > 1) {
      vis = soft_visibility(s, p, n, q, ld, tests);
      if (!(vis > 0.0)) continue;
    } else {
      if (tests) tests[OR_CNT_SHADOW_RAYS] += 1;
      if (in_cast_shadow(s, p, ld, dist, tests)) continue;
      vis = 1.0;
    }
    lit |= 1u << l;
    double intensity = q[3] * vis;
    *A += intensity * nl;
    double x;
    if (s->spec_model == OR_SPEC_PHONG) {
      /* reflect the light-to-surface direction about n; compare with the view */
      double r[3] = {2.0 * nl * n[0] - ld[0], 2.0 * nl * n[1] - ld[1], 2.0 * nl * n[2] - ld[2]};
      x = dot3(view, r);
    } else {
      double h[3] = {ld[0] + view[0], ld[1] + view[1], ld[2] + view[2]};
      double hl = sqrt(dot3(h, h));
      x = hl > 0.0 ? dot3(n, h) / hl : 0.0;
    }
    double spec = x > 0.0 ? pow(x, shine) : 0.0;
    *S += intensity * s->spec_strength * spec;
  }
  return lit;
}

/* ---- Section 3.8: skybox --------------------------------------------------- */

/* Colour of the map in direction d (unit), by spherical UV mapping: the
 * longitude u = 1/2 + atan2(d_x, -d_z) / (2 pi) (u = 1/2 straight ahead, down
 * -z) and the latitude v = 1/2 - asin(d_y) / pi (v = 0 straight up) index an
 * equirectangular image, whose texel (i, j) covers u in [i/w, (i+1)/w) and v
 * in [j/h, (j+1)/h); bilinear between texel centres, wrapping around in u and
 * clamped to the first and last row in v. */
static void sky_colour(const or_scene* s, const double d[3], double out[3]) {
  double u = 0.5 + atan2(d[0], -d[2]) / (2.0 * OR_PI);
  double dy = d[1] < -1.0 ? -1.0 : (d[1] > 1.0 ? 1.0 : d[1]);
  double v = 0.5 - asin(dy) / OR_PI;
  double x = u * s->sky_w - 0.5, y = v * s->sky_h - 0.5;
  double fx = floor(x), fy = floor(y);
  double ax = x - fx, ay = y - fy;
  int64_t x0 = (int64_t)fx, y0 = (int64_t)fy;
  int64_t xs[2], ys[2];
  for (int k = 0; k < 2; ++k) {
    int64_t xi = (x0 + k) % s->sky_w;
    xs[k] = xi < 0 ? xi + s->sky_w : xi;
    int64_t yi = y0 + k;
    ys[k] = yi < 0 ? 0 : (yi >= s->sky_h ? s->sky_h - 1 : yi);
  }
  for (int c = 0; c < 3; ++c) {
    double t00 = s->sky[3 * (ys[0] * s->sky_w + xs[0]) + c];
    double t10 = s->sky[3 * (ys[0] * s->sky_w + xs[1]) + c];
    double t01 = s->sky[3 * (ys[1] * s->sky_w + xs[0]) + c];
    double t11 = s->sky[3 * (ys[1] * s->sky_w + xs[1]) + c];
    out[c] = (1.0 - ay) * ((1.0 - ax) * t00 + ax * t10) + ay * ((1.0 - ax) * t01 + ax * t11);
  }
}

/* ---- Section 3.7: recursive reflections --------------------------------- */

typedef struct {
  int32_t* seg_id;   /* [depth+1] or NULL */
  uint32_t* lit;     /* [depth+1] or NULL */
  int64_t* counts;   /* [OR_NCOUNTS]      */
  double jitter;
  uint64_t seed;
  int64_t pixel;
} trace_ctx;

/* SplitMix64 (Steele, Lea and Flood, "Fast Splittable Pseudorandom Number
 * Generators", OOPSLA 2014), with the increment and the two multipliers of
 * its published 64-bit finaliser.  It only seeds the jitter of the
 * conditioning re-traces, never a rendered value. */
static uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* uniform in [-1, 1) from (seed, pixel, level, component) */
static double jitter_unit(const trace_ctx* c, int level, int comp) {
  uint64_t k = splitmix64(c->seed ^ splitmix64((uint64_t)c->pixel * 64u + (uint64_t)level * 8u +
                                               (uint64_t)comp));
  return (double)(k >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

/* Conditioning runs only: move the origin by jitter*|o| and the direction by
 * jitter (each component uniform in [-1, 1) times that size), renormalise d. */
static void jitter_ray(const trace_ctx* c, int level, double o[3], double d[3]) {
  double on = sqrt(dot3(o, o));
  for (int k = 0; k < 3; ++k) o[k] += c->jitter * on * jitter_unit(c, level, k);
  for (int k = 0; k < 3; ++k) d[k] += c->jitter * jitter_unit(c, level, 3 + k);
  normalize3(d);
}

/* rayTrace(ray, depth) of the paper's reflection pseudocode: the closest hit;
 * black (background) on a miss; shade(colour) at the depth limit; otherwise
 * trace the mirror ray, mix the body colour with the reflected colour by the
 * reflection ratio, and shade the mix.  `level` counts segments from the
 * primary ray (level 0). */
static void ray_trace(const or_scene* s, const double o_in[3], const double d_in[3], int depth,
                      int level, const trace_ctx* c, double color[3]) {
  double o[3] = {o_in[0], o_in[1], o_in[2]}, d[3] = {d_in[0], d_in[1], d_in[2]};
  if (c->jitter > 0.0) jitter_ray(c, level, o, d);
  if (level > 0) c->counts[OR_CNT_REFLECTION_RAYS] += 1;
  double t;
  int32_t id = or_closest_hit(s, o, d, &t, c->counts);
  if (c->seg_id) c->seg_id[level] = id;
  if (id == OR_MISS) {
    if (s->sky && s->sky_w > 0 && s->sky_h > 0) {
      sky_colour(s, d, color);
    } else {
      color[0] = s->background[0];
      color[1] = s->background[1];
      color[2] = s->background[2];
    }
    return;
  }
  double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
  double n[3];
  const double *mat, *shine;
  if (id < s->n_spheres) {
    const double* g = s->sphere_geom + 4 * id;
    n[0] = (p[0] - g[0]) / g[3];
    n[1] = (p[1] - g[1]) / g[3];
    n[2] = (p[2] - g[2]) / g[3];
    mat = s->sphere_mat + 4 * id;
    shine = s->sphere_shine + id;
  } else {
    int32_t j = id - s->n_spheres;
    n[0] = s->plane_geom[4 * j];
    n[1] = s->plane_geom[4 * j + 1];
    n[2] = s->plane_geom[4 * j + 2];
    mat = s->plane_mat + 4 * j;
    shine = s->plane_shine + j;
  }
  double view[3] = {-d[0], -d[1], -d[2]};
  double A, S;
  uint32_t lit = light_terms(s, p, n, view, *shine, &A, &S, c->counts);
  if (c->lit) c->lit[level] = lit;
  double base[3] = {mat[0], mat[1], mat[2]};
  if (depth == 0) {
    for (int k = 0; k < 3; ++k) color[k] = base[k] * A + S;
    return;
  }
  /* mirror direction about the normal (Section 3.7) */
  double dn = dot3(d, n);
  double rd[3] = {d[0] - 2.0 * dn * n[0], d[1] - 2.0 * dn * n[1], d[2] - 2.0 * dn * n[2]};
  double refl[3];
  ray_trace(s, p, rd, depth - 1, level + 1, c, refl);
  double ratio = mat[3];
  for (int k = 0; k < 3; ++k) {
    double mixed = base[k] * (1.0 - ratio) + refl[k] * ratio;
    color[k] = mixed * A + S;
  }
}

/* ---- decision margin of the primary segment ----------------------------- */

/* Smallest relative distance to a discrete decision change along the primary
 * ray: the gap to the next primitive's root, the angle to tangency of any
 * sphere that could change the winner, and the horizon of a plane that is hit
 * (or of every plane on a miss). */
static double primary_margin(const or_scene* s, const double o[3], const double d[3], int32_t id,
                             double t1) {
  double m = INFINITY, tt;
  if (id != OR_MISS) {
    for (int32_t i = 0; i < s->n_spheres; ++i)
      if (i != id && or_sphere_root(o, d, s->sphere_geom + 4 * i, s->t_min, &tt))
        m = fmin(m, (tt - t1) / t1);
    for (int32_t j = 0; j < s->n_planes; ++j)
      if (s->n_spheres + j != id && or_plane_root(o, d, s->plane_geom + 4 * j, s->t_min, &tt))
        m = fmin(m, (tt - t1) / t1);
  }
  for (int32_t i = 0; i < s->n_spheres; ++i) {
    const double* g = s->sphere_geom + 4 * i;
    double oc[3] = {o[0] - g[0], o[1] - g[1], o[2] - g[2]};
    double tca = -dot3(oc, d);
    double occ = dot3(oc, oc);
    if (tca <= 0.0 || occ <= g[3] * g[3]) continue;   /* behind, or origin inside */
    if (i != id && id != OR_MISS && tca >= t1 * (1.0 + 1e-6)) continue;  /* behind the hit */
    double h = sqrt(fmax(occ - tca * tca, 0.0));
    m = fmin(m, fabs(h - g[3]) / tca);
  }
  for (int32_t j = 0; j < s->n_planes; ++j) {
    if (id == OR_MISS || id == s->n_spheres + j) {
      const double* g = s->plane_geom + 4 * j;
      m = fmin(m, fabs(g[0] * d[0] + g[1] * d[1] + g[2] * d[2]));
    }
  }
  return m;
}

/* ---- pixel loop ---------------------------------------------------------- */

int or_render_pixels(const or_scene* s, const or_camera* cam, int32_t W, int32_t H,
                     int32_t depth, int64_t n_pix, const int64_t* pix, double jitter,
                     uint64_t seed, int32_t n_threads, const or_outputs* out) {
  if (!s || !cam || !out || W <= 0 || H <= 0 || depth < 0 || depth > 30 || n_pix < 0 ||
      (n_pix > 0 && !pix) || s->n_lights > 32)
    return -1;
  for (int64_t i = 0; i < n_pix; ++i)
    if (pix[i] < 0 || pix[i] >= (int64_t)W * H) return -1;
  int64_t total[OR_NCOUNTS] = {0, 0, 0, 0, 0};
  int nt = n_threads > 0 ? n_threads : 1;
  (void)nt;
#pragma omp parallel num_threads(nt)
  {
    int64_t local[OR_NCOUNTS] = {0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_pix; ++i) {
      int32_t x = (int32_t)(pix[i] % W), y = (int32_t)(pix[i] / W);
      double o[3], d[3], color[3];
      or_camera_ray(cam, W, H, x, y, o, d);
      int32_t seg_local[32];
      uint32_t lit_local[32];
      for (int k = 0; k <= depth; ++k) {
        seg_local[k] = OR_NOT_TRACED;
        lit_local[k] = 0;
      }
      trace_ctx c = {seg_local, lit_local, local, jitter, seed, pix[i]};
      local[OR_CNT_PRIMARY_RAYS] += 1;
      ray_trace(s, o, d, depth, 0, &c, color);
      if (out->rgb) {
        out->rgb[3 * i] = color[0];
        out->rgb[3 * i + 1] = color[1];
        out->rgb[3 * i + 2] = color[2];
      }
      if (out->prim_id) out->prim_id[i] = seg_local[0];
      if (out->seg_id)
        for (int k = 0; k <= depth; ++k) out->seg_id[i * (depth + 1) + k] = seg_local[k];
      if (out->lit)
        for (int k = 0; k <= depth; ++k) out->lit[i * (depth + 1) + k] = lit_local[k];
      if (out->margin) {
        double t;
        int32_t id = or_closest_hit(s, o, d, &t, NULL);
        out->margin[i] = primary_margin(s, o, d, id, t);
      }
    }
#pragma omp critical
    for (int k = 0; k < OR_NCOUNTS; ++k) total[k] += local[k];
  }
  if (out->counts)
    for (int k = 0; k < OR_NCOUNTS; ++k) out->counts[k] = total[k];
  return 0;
}

void or_camera_rays(const or_camera* cam, int32_t W, int32_t H, int64_t n, const int64_t* pix,
                    double* o, double* d) {
  for (int64_t i = 0; i < n; ++i)
    or_camera_ray(cam, W, H, (int32_t)(pix[i] % W), (int32_t)(pix[i] / W), o + 3 * i, d + 3 * i);
}

void or_closest_hits(const or_scene* s, int64_t n, const double* o, const double* d,
                     int32_t* ids, double* ts) {
  for (int64_t i = 0; i < n; ++i) ids[i] = or_closest_hit(s, o + 3 * i, d + 3 * i, ts + i, NULL);
}
