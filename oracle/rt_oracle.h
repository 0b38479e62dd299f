/*
 * rt_oracle.h - FP64 CPU reference Whitted ray tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never includes, links or calls it,
 * and this file shares no code with the HIP kernels.
 *
 * Every floating-point quantity is double precision.  Inputs are the canonical
 * FP32 scene promoted exactly to double.
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MISS (-1)        /* segment traced, no primitive hit                */
#define OR_NOT_TRACED (-2)  /* segment after a miss or beyond the depth limit  */

#define OR_SPEC_BLINN 0
#define OR_SPEC_PHONG 1

/* Counter slots filled by or_render_pixels (algorithmic counts, Section 3.4.1
 * and 3.6: every ray tests every primitive; a shadow ray stops at its first
 * occluder in ascending primitive order and is traced only when n.L > 0). */
enum {
  OR_CNT_SPHERE_TESTS = 0,
  OR_CNT_PLANE_TESTS = 1,
  OR_CNT_PRIMARY_RAYS = 2,
  OR_CNT_REFLECTION_RAYS = 3,
  OR_CNT_SHADOW_RAYS = 4,
  OR_NCOUNTS = 5
};

typedef struct {
  int32_t n_spheres, n_planes, n_lights, spec_model;
  const double* sphere_geom;   /* [N][4] centre x y z, radius           */
  const double* sphere_mat;    /* [N][4] albedo r g b, reflection ratio */
  const double* sphere_shine;  /* [N]    specular exponent              */
  const double* plane_geom;    /* [P][4] unit normal m, offset h: m.x=h */
  const double* plane_mat;     /* [P][4]                                */
  const double* plane_shine;   /* [P]                                   */
  const double* light;         /* [L][4] position, intensity            */
  double ambient, spec_strength, t_min;
  double background[3];
  /* Soft shadows (Section 3.6.1): with shadow_samples > 1 every light is a
   * sphere of radius light_radius sampled at shadow_samples points of its
   * great circle facing the hit point; 0 or 1 sample: hard shadows. */
  int32_t shadow_samples;
  double light_radius;
  /* Skybox (Section 3.8): an equirectangular map sky[h][w][3] that replaces
   * the background colour of a miss; NULL (or w = 0): the background. */
  const double* sky;
  int32_t sky_w, sky_h;
} or_scene;

typedef struct {
  double eye[3];
  double yaw_deg, pitch_deg, fov_deg;
} or_camera;

/* Optional per-pixel outputs of or_render_pixels; any pointer may be NULL.
 * Index i runs over the requested pixels in the order given. */
typedef struct {
  double* rgb;        /* [n][3] linear colour                                 */
  int32_t* prim_id;   /* [n]    primary-segment hit id, OR_MISS on a miss     */
  int32_t* seg_id;    /* [n][depth+1] hit id per segment                      */
  uint32_t* lit;      /* [n][depth+1] bit l: light l lit the hit (n.L>0 and no
                         occluder; with soft shadows: some sample unblocked)  */
  double* margin;     /* [n]    decision margin of the primary segment        */
  int64_t* counts;    /* [OR_NCOUNTS] summed over the requested pixels        */
} or_outputs;

/* Primary ray through pixel (x, y) of a W x H window (Sections 3.1-3.3). */
void or_camera_ray(const or_camera* cam, int32_t W, int32_t H, int32_t x, int32_t y,
                   double o[3], double d[3]);

/* Nearest root t > t_min of a ray with unit d against one sphere / plane;
 * returns 1 and sets *t when there is one (Section 3.4.1). */
int or_sphere_root(const double o[3], const double d[3], const double* geom4, double t_min,
                   double* t);
int or_plane_root(const double o[3], const double d[3], const double* geom4, double t_min,
                  double* t);

/* Closest hit over every primitive (Section 3.4.1); returns id or OR_MISS. */
int32_t or_closest_hit(const or_scene* s, const double o[3], const double d[3], double* t,
                       int64_t* tests);

/* Render the listed pixels (index y*W + x).  jitter > 0 perturbs each
 * segment's origin and direction by that relative amount (conditioning runs);
 * seed selects the perturbation.  Returns 0, or -1 on bad arguments. */
int or_render_pixels(const or_scene* s, const or_camera* cam, int32_t W, int32_t H,
                     int32_t depth, int64_t n_pix, const int64_t* pix, double jitter,
                     uint64_t seed, int32_t n_threads, const or_outputs* out);

/* Batch helpers for the tests: primary rays and closest hits of given rays. */
void or_camera_rays(const or_camera* cam, int32_t W, int32_t H, int64_t n, const int64_t* pix,
                    double* o, double* d);
void or_closest_hits(const or_scene* s, int64_t n, const double* o, const double* d,
                     int32_t* ids, double* ts);

#ifdef __cplusplus
}
#endif
#endif
