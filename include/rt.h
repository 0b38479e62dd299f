/*
 * rt.h - C ABI of librtmi, a Whitted ray-tracing render kernel for AMD
 * Instinct MI355X (gfx950).
 *
 * The library renders scenes of spheres and planes lit by point lights:
 * pinhole primary rays (paper Sections 3.1-3.3), brute-force closest hit
 * over every primitive (Section 3.4.1), Phong or Blinn-Phong shading
 * (Section 3.5) with hard cast shadows (Section 3.6), and mirror
 * reflections up to a fixed bounce limit (Section 3.7).  Around that: soft
 * shadows of spherical lights (Section 3.6.1), a skybox (Section 3.8), the
 * adjoint of the image with visibility held fixed, a batched launch of many
 * scenes, and an interactive per-frame path that streams camera, settings
 * and body positions in and the image out (Section 3.9).
 *
 * Conventions for every call:
 *   - All calls are C, never throw, and return rt_status.  On failure a
 *     detail message is available from rt_last_error() (per thread).
 *   - Argument errors are found on the host before any HIP call and return
 *     RT_ERR_INVALID_ARG; nothing is launched or written then.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is asynchronous on that stream; a device fault surfaces at a later
 *     call or synchronisation as RT_ERR_DEVICE.
 *   - Pointers named *_out, records and gradients are caller-owned device
 *     memory.  rt_scene, rt_batch and rt_frame objects are library-owned and
 *     freed by their destroy call.
 *   - Images are row-major, row 0 at the top: element (y, x) of a W x H image
 *     is at index y * W + x (the paper's pixel index, Section 3.9).
 *   - Camera frame: x right, y up, the camera looks down -z; yaw turns about
 *     +y and pitch about +x, pitch applied first.  Pixel (x, y) maps to
 *     viewport coordinates u = (2x - W) / s, v = (H - 2y) / s, s = min(W, H),
 *     with no half-pixel offset (Section 3.2 and its worked example); the
 *     viewport sits at distance 1 / tan(fov / 2) (Section 3.2.1).
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MAX_DEPTH 8        /* reflection bounce limit (segments = depth + 1)  */
#define RT_MAX_LIGHTS 8
#define RT_MAX_SPHERES 4096
#define RT_MAX_PLANES 16
#define RT_MAX_DIM 16384      /* largest W or H                                 */
#define RT_MAX_BATCH 4096     /* largest number of scenes in one batch          */
#define RT_MAX_SAMPLES 4096   /* most shadow samples per light (rt_render_soft)  */
#define RT_MAX_SKY_DIM 16384  /* largest skybox width or height                 */

typedef enum {
  RT_OK = 0,
  RT_ERR_INVALID_ARG = 1,
  RT_ERR_OUT_OF_MEMORY = 2,
  RT_ERR_DEVICE = 3,
  RT_ERR_UNSUPPORTED = 4
} rt_status;

/* Where the arrays of an rt_scene_desc live. */
typedef enum { RT_HOST = 0, RT_DEVICE = 1 } rt_mem;

/* Specular model: Blinn's halfway vector (Section 3.5.2, the paper's final
 * model) or Phong's reflected light vector (the Phong pseudocode of Section
 * 3.5.1). */
typedef enum { RT_SPEC_BLINN = 0, RT_SPEC_PHONG = 1 } rt_spec_model;

/* Pinhole camera: the paper's camera[6] argument (Section 3.9): position,
 * yaw and pitch (degrees), field of view (degrees, 0 < fov < 180) spanning
 * the shorter image side. */
typedef struct {
  float eye[3];
  float yaw_deg, pitch_deg, fov_deg;
} rt_camera;

/* Scene description (Section 3.4: every body has a position, a size, a
 * colour and a reflectivity; the paper's single reflectivity is split into a
 * specular exponent and a reflection ratio kr used to mix the body colour
 * with the reflected colour, Section 3.7).  All arrays are float32, packed
 * row-major with no padding.  Primitive ids: spheres 0..N-1, then planes
 * N..N+P-1.  With mem == RT_HOST the values are validated on the host; with
 * RT_DEVICE only counts and pointers are (values are the caller's
 * responsibility; non-finite values give non-finite pixels). */
typedef struct {
  int32_t n_spheres;          /* 0 .. RT_MAX_SPHERES                          */
  int32_t n_planes;           /* 0 .. RT_MAX_PLANES                           */
  int32_t n_lights;           /* 0 .. RT_MAX_LIGHTS                           */
  int32_t spec_model;         /* rt_spec_model                                */
  const float* sphere_geom;   /* [N][4] centre x y z, radius r (r > 0)        */
  const float* sphere_mat;    /* [N][4] albedo r g b, reflection ratio kr     */
  const float* sphere_shine;  /* [N]    specular exponent (> 0)               */
  const float* plane_geom;    /* [P][4] unit normal m x y z, offset h: m.x = h*/
  const float* plane_mat;     /* [P][4] albedo r g b, reflection ratio kr     */
  const float* plane_shine;   /* [P]    specular exponent (> 0)               */
  const float* light;         /* [L][4] position x y z, intensity I (>= 0)    */
  float ambient;              /* k_a, share of the colour always visible      */
  float spec_strength;        /* k_s, scale of the specular term              */
  float t_min;                /* roots at or below t_min are ignored (>= 0)   */
  float background[3];        /* colour of a ray that hits nothing            */
  int32_t mem;                /* rt_mem of the seven arrays above             */
} rt_scene_desc;

typedef struct rt_scene_s* rt_scene;

/* Per-segment hit records kept by the forward pass for the adjoint
 * (caller-owned device memory of rt_records_bytes() bytes in total):
 *   ids: int32 [depth+1][H][W]  primitive hit by segment k, -1 for a miss,
 *                               -2 for a segment not traced;
 *   lit: uint8 [depth+1][H][W]  bit l set when light l lit that hit
 *                               (n.L > 0 and no occluder). */
typedef struct {
  int32_t* ids;
  uint8_t* lit;
  int64_t bytes;              /* bytes available at ids + lit together        */
} rt_records;

/* Gradients of a scalar loss (caller-owned device float32, overwritten):
 * d_albedo [N][3], d_refl [N], d_center [N][3], d_light_pos [L][3],
 * d_light_int [L].  Any pointer may be NULL to skip that group. */
typedef struct {
  float* d_albedo;
  float* d_refl;
  float* d_center;
  float* d_light_pos;
  float* d_light_int;
} rt_grads;

/* Copy a scene into library-owned device memory, packed for the kernels
 * (the paper keeps the scene resident on the device between frames, Section
 * 2.3).  Allocates; not capture-safe.  Synchronises `stream` before it
 * returns when mem == RT_HOST. */
rt_status rt_scene_upload(const rt_scene_desc* desc, void* stream, rt_scene* out);

/* Replace the values of a scene in place (the paper's per-frame stream-in of
 * camera and body positions, Section 3.9).  Counts and spec_model must
 * match the uploaded scene.  No allocation; asynchronous on `stream` when
 * mem == RT_DEVICE. */
rt_status rt_scene_update(rt_scene scene, const rt_scene_desc* desc, void* stream);

/* Give a scene a skybox (Section 3.8): a distant panoramic HDR image that a
 * ray leaving the scene shows in place of the plain background.  `rgb` is
 * float32 [h][w][3], linear colour, finite (checked when mem == RT_HOST),
 * equirectangular: for a unit
 * direction d, column coordinate u = 1/2 + atan2(d_x, -d_z) / (2 pi) and row
 * coordinate v = 1/2 - asin(d_y) / pi, both in [0, 1] across the whole image
 * (row 0 straight up, u = 1/2 along -z); the colour is bilinear between
 * texel centres (x = u w - 1/2, y = v h - 1/2), wrapping around in x and
 * clamped to the edge rows in y.  Every render entry point then uses it on
 * a miss, and rt_render_backward differentiates through it.
 *   rgb   host or device pointer per `mem`; copied, the caller keeps it;
 *   w, h  1 .. RT_MAX_SKY_DIM; rgb == NULL with w == h == 0 removes the
 *         skybox.
 * Allocates the skybox's own device buffer when the scene has none of this
 * size (frees it on removal); not capture-safe.  With mem == RT_HOST the copy
 * is synchronous, through a host staging buffer of 16 bytes per texel that is
 * allocated first: if that fails, RT_ERR_OUT_OF_MEMORY and the scene's skybox
 * is unchanged.  With RT_DEVICE it is ordered on `stream`.  Renders already
 * queued on other streams must be finished first. */
rt_status rt_scene_set_sky(rt_scene scene, const float* rgb, int32_t w, int32_t h, rt_mem mem,
                           void* stream);

rt_status rt_scene_destroy(rt_scene scene);

/* Counts of an uploaded scene (any pointer may be NULL), so that a binding
 * can size gradient buffers and check the caller's: host-only, no HIP call. */
rt_status rt_scene_counts(rt_scene scene, int32_t* n_spheres, int32_t* n_planes,
                          int32_t* n_lights);

/* Bytes of records for a W x H image at the given depth. */
int64_t rt_records_bytes(int32_t W, int32_t H, int32_t depth);

/* Render one image (the paper's render method, Section 3.9): every pixel
 * traces its primary ray, shades each hit with shadow rays, and follows
 * mirror rays up to `depth` bounces (depth 0 = no reflection).
 *   rgb_out  device float32 [H][W][3], linear colour, not clamped;
 *   id_out   device int32 [H][W] primary hit id (-1 = miss), or NULL;
 *   rec      records for rt_render_backward, or NULL.
 * Launches two kernels: the preparation, then the render.  The preparation
 * writes the cones of the spheres seen from the camera's eye, and their
 * centres' offsets from the eye, into the scene's own buffer.  For images of 4096 to 131072 8x8 tiles the render
 * also records how long each of its tiles took (a byte per tile and a count
 * per duration bin, in the scene's buffer), and the preparation of the next
 * render of the scene at the same size turns that record into the order in
 * which the render takes its tiles: longest first (the first render of a
 * size takes row order).  The order changes no pixel, only how well the
 * tiles fill the GPU; a record from another view or before rt_scene_update
 * is still used, as a guess.  No allocation, capture-safe.  Because the
 * eye-cone, eye-offset, record and order tables live in the scene, calls that write them
 * (rt_render, rt_render_ex, rt_render_prepare, rt_render_soft,
 * rt_render_counts and rt_render_backward with rec == NULL) must not overlap
 * in time for one scene: on one stream they are ordered; on different
 * streams the caller orders them (events), or a render may read another
 * call's tables. */
rt_status rt_render(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H, int32_t depth,
                    float* rgb_out, int32_t* id_out, const rt_records* rec, void* stream);

/* Flags of rt_render_ex. */
#define RT_RENDER_NO_PREFILTER 1u  /* run the exact ray-sphere test on every
                                      pair: the cone tests that skip pairs
                                      (cones seen from the eye and from the
                                      lights) only skip pairs the exact test
                                      rejects, so the image is the same bits
                                      either way; this flag exists to check
                                      that */

#define RT_RENDER_CONES_READY 2u   /* rt_render_ex only: skip the
                                      preparation launch; the caller has
                                      called rt_render_prepare with a camera
                                      at the same eye position, on the same
                                      stream, after the last call that
                                      rewrote the scene's cones (any render,
                                      count or re-traced backward of the
                                      scene, or a scene update).  Stale cones
                                      give a wrong image, never an
                                      out-of-bounds access; the tile order of
                                      that preparation is used only if it was
                                      made for the same W x H */
#define RT_RENDER_ROW_ORDER 4u     /* rt_render_ex and rt_render_soft:
                                      take the tiles in row order and record
                                      no durations; the same image bits */

/* rt_render with flags (0 = rt_render); the same two launches (one with
 * RT_RENDER_CONES_READY) and the same rule for calls on one scene. */
rt_status rt_render_ex(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H, int32_t depth,
                       float* rgb_out, int32_t* id_out, const rt_records* rec, uint32_t flags,
                       void* stream);

/* The first of rt_render's two launches on its own: the cones of the scene's
 * spheres seen from the camera's eye and, where rt_render orders its tiles,
 * the tile order of a W x H image from the last recorded render of that
 * size, written into the scene's buffer, for a following rt_render_ex with
 * RT_RENDER_CONES_READY (so that the render kernel can be timed or captured
 * on its own; the first such render after it records its tile durations).
 * One launch, no allocation, capture-safe; the same overlap rule as
 * rt_render. */
rt_status rt_render_prepare(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H,
                            void* stream);

/* Render one image with soft shadows (the paper's soft cast shadows, Section
 * 3.6.1): every light is a sphere of radius light_radius about its position,
 * sampled at `samples` points of its great circle facing the hit point in the
 * sunflower arrangement (point i at radius 2 light_radius sqrt(i/samples) and
 * angle i times the golden angle pi (3 - sqrt 5), in the plane perpendicular
 * to the direction from the hit point to the light; the in-plane orientation
 * follows Duff et al., "Building an Orthonormal Basis, Revisited", 2017).  A
 * sample's shadow ray is blocked when the sample lies behind the tangent plane
 * at the hit point or a primitive has a root between t_min and the sample;
 * diffuse and specular of that light are scaled by the unblocked share.
 *   samples       1 .. RT_MAX_SAMPLES; samples == 1 or light_radius == 0 is
 *                 the point light, rendered exactly as rt_render_ex;
 *   light_radius  finite, >= 0, scene units;
 *   rgb_out, id_out as rt_render_ex; flags RT_RENDER_NO_PREFILTER and
 *   RT_RENDER_ROW_ORDER.  No records: the adjoint and the batched launch take
 *   point lights.
 * Without RT_RENDER_NO_PREFILTER a wave skips only tests whose outcome it has
 * shown, with FP32 error margins: spheres outside its bound, the sphere all
 * its lanes lie on, planes its sample rays cannot reach, and the whole sample
 * loop when every sample is visible; the image is the same bits as with the
 * flag, which tests every sample ray against every primitive.
 * Launches three kernels (the preparation as rt_render's, the sample table,
 * the render; images of up to 40 000 8 x 8 tiles share each pixel's samples
 * between two lanes, whose integer counts are added): like rt_render it
 * records every tile's duration and takes the
 * tiles longest first by the record of the last soft-shadow render of the
 * scene at this W x H (hard- and soft-shadow renders keep apart records; an
 * image takes the same bits in any order).  No allocation, capture-safe.
 * Renders of one scene must not overlap in time (the sample table, the eye
 * cones and the tile schedule live in the scene's buffer). */
rt_status rt_render_soft(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H,
                         int32_t depth, int32_t samples, float light_radius, float* rgb_out,
                         int32_t* id_out, uint32_t flags, void* stream);

/* Work counters of the render of one image.  Adds to counts (device int64
 * [RT_NUM_COUNTS], caller zeroes):
 *   [0] ray-sphere tests and [1] ray-plane tests as the method defines its
 *       work (Sections 3.4.1 and 3.6: every segment tests every primitive; a
 *       shadow ray is traced only when n.L > 0 and tests primitives in
 *       ascending id order up to its first occluder);
 *   [2] primary rays, [3] reflection rays, [4] shadow rays;
 *   [5] ray-sphere tests and [6] ray-plane tests the render kernel actually
 *       executes, once per ray whose result can still matter: pairs that the
 *       cone tests and wave bounds decide without the exact test are not
 *       counted.  With flags = RT_RENDER_NO_PREFILTER the counts are those of
 *       the kernel without them, whose executed tests equal [0] and [1].
 * Renders no image.  Launches the eye-cone kernel and the counting kernel (the
 * render's path code with per-lane counters), so it must not overlap other
 * renders of the same scene (see rt_render). */
#define RT_NUM_COUNTS 7
rt_status rt_render_counts(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H,
                           int32_t depth, int64_t* counts, uint32_t flags, void* stream);

/* Adjoint of rt_render with every discrete decision fixed (hit primitive per
 * segment, lit lights, path length): given dLoss/dRGB (device float32
 * [H][W][3]) it writes the gradients of the loss with respect to albedo,
 * reflection ratio and centre of every sphere and position and intensity of
 * every light.  Radii, exponents, planes, ambient and k_s are constants and
 * shadow occluders carry no gradient.  With rec == NULL the decisions are
 * recomputed by re-tracing; otherwise they are read from records written by
 * rt_render for the same scene, camera, size and depth.  The sum over pixels
 * is deterministic (fixed order; no two lanes or waves add into one float).  With a skybox,
 * a path that ends in a miss also feeds its last mirror direction through
 * the UV mapping and the bilinear weights (texels are constants).  The
 * per-wave gradient accumulators (7 N + 4 L + 4 floats) live in LDS: up to
 * 2335 spheres within 64 KiB per workgroup (four waves each for small
 * scenes), beyond that one wave per workgroup with up to the device's LDS
 * per workgroup (160 KiB on gfx950: every scene up to RT_MAX_SPHERES, whose
 * accumulators take 112 KiB); a scene that does not fit returns
 * RT_ERR_UNSUPPORTED and writes nothing.
 * No allocation; capture-safe.  With
 * rec == NULL the re-trace first rewrites the scene's eye-cone table, so it
 * must not overlap other renders of the same scene (see rt_render); the
 * per-workgroup gradient partials also live in the scene's buffer, so two
 * backward calls of one scene must not overlap either. */
rt_status rt_render_backward(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H,
                             int32_t depth, const float* grad_rgb, const rt_records* rec,
                             const rt_grads* grads, void* stream);

/* For callers that cannot allocate device memory at all (code under graph
 * capture, serving loops, harnesses that forbid hipMalloc): rt_render_backward
 * with the same arguments, kernels and grid, hence the same bits, but its
 * per-workgroup gradient partials (device scratch) live in a file-scope
 * device array of RT_STATIC_SCRATCH_BYTES (16 MiB) that each GPU the library
 * runs on holds until the process ends, instead of in the scene's buffer.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the first call on a device looks the array's address up once.
 * A problem whose partials need more than the array holds (grid rows x
 * (7 N + 4 L) floats, the grid being min(1024, 16x16 tiles of the image),
 * capped at 64 MiB as in rt_render_backward) returns RT_ERR_INVALID_ARG and
 * launches nothing.  Every row the reduction reads is written by the same
 * launch, so nothing needs clearing between calls.  All calls on one GPU
 * share the array: two calls that overlap on one GPU (on different streams,
 * or from different threads without ordering) race and give wrong gradients;
 * calls on one stream are ordered and safe.  The eye-cone rule of
 * rt_render_backward applies too. */
#define RT_STATIC_SCRATCH_BYTES 16777216u
rt_status rt_render_backward_static(rt_scene scene, const rt_camera* cam, int32_t W, int32_t H,
                                    int32_t depth, const float* grad_rgb, const rt_records* rec,
                                    const rt_grads* grads, void* stream);

typedef struct rt_batch_s* rt_batch;

/* Prepare one persistent launch that renders n scenes of any sizes and
 * depths (each image exactly as rt_render would), captured in a HIP graph.
 * Builds the tile table (largest estimated cost first), picks the launch
 * shape (autotuned once per problem signature when `autotune` is non-zero,
 * which runs and synchronises on `stream`; cached in memory and in the JSON
 * file of rt_tune_cache_get, so later processes skip the timing), allocates the
 * queue counter and captures the graph.  rgb_out[i] is device float32
 * [H[i]][W[i]][3].  Sizes, depths, cameras and the total tile count (at most
 * 2^31 - 1 tiles of 64 pixels, the queue's 32-bit tile numbers) are checked
 * before any scene is read: RT_ERR_INVALID_ARG.  A failed host or device
 * allocation returns RT_ERR_OUT_OF_MEMORY or RT_ERR_DEVICE and leaves nothing
 * allocated. */
rt_status rt_batch_create(int32_t n, const rt_scene* scenes, const rt_camera* cams,
                          const int32_t* W, const int32_t* H, const int32_t* depth,
                          float* const* rgb_out, int32_t autotune, void* stream, rt_batch* out);

/* Replay the batch's graph on `stream`.  Scenes may be updated in place
 * between launches (rt_scene_update, and rt_scene_set_sky with the size the
 * skybox had at creation); a skybox added, removed or resized since
 * rt_batch_create makes the launch return RT_ERR_INVALID_ARG.  The scenes
 * must outlive the batch. */
rt_status rt_batch_launch(rt_batch batch, void* stream);

/* The same launch without the graph (a plain kernel launch), with the same
 * skybox check. */
rt_status rt_batch_launch_direct(rt_batch batch, void* stream);

/* Work counters of one batch launch, as rt_render_counts gives them for a
 * single image (RT_NUM_COUNTS int64 added to counts, device memory, caller
 * zeroes): the batch kernel with its chosen launch shape, plus per-lane
 * counters, launched directly (no graph).  The algorithmic counts [0..4] are
 * the sum of the single renders'; the executed tests [5], [6] depend on how
 * the launch shape groups pixels into waves.  Renders the images as well. */
rt_status rt_batch_counts(rt_batch batch, int64_t* counts, void* stream);

/* Launch shape chosen for the batch: workgroups and pixel-tile width and
 * height (any pointer may be NULL). */
rt_status rt_batch_shape(rt_batch batch, int32_t* workgroups, int32_t* tile_w, int32_t* tile_h);

rt_status rt_batch_destroy(rt_batch batch);

/* The batch autotuner's cache.  A key is the device's architecture name and
 * compute-unit count followed by the batch signature (every job's W, H,
 * depth, sphere and light count and skybox flag); rt_batch_tune_key gives a
 * batch's key (a NUL-terminated copy of at most cap - 1 bytes into buf, and
 * its full length into *len).  Entries live in memory and in a JSON file:
 * $RT_TUNE_CACHE if set (empty: memory only), else
 * $XDG_CACHE_HOME/rtmi/tune.json, else $HOME/.cache/rtmi/tune.json, holding a
 * 64-bit FNV-1a digest of each key and its shape.  rt_batch_create with
 * autotune looks the key up before timing and stores what it timed.
 * rt_tune_cache_get sets *found to 1 and the shape (as rt_batch_shape gives
 * it) on a hit, else 0.  rt_tune_cache_put stores a shape the tuner could
 * have picked (tile_w 8, 16 or 64 columns, 64 / tile_w x 1, 2 or 4 rows,
 * 1 to 2^20 workgroups), else RT_ERR_INVALID_ARG; a file that cannot be
 * written gives RT_ERR_UNSUPPORTED (the entry stays in memory).
 * rt_tune_cache_forget drops the memory entries, so that the next lookup
 * reads the file.  A file entry that does not parse, or holds a shape
 * outside the tuner's candidates, is ignored. */
rt_status rt_batch_tune_key(rt_batch batch, char* buf, int64_t cap, int64_t* len);
rt_status rt_tune_cache_get(const char* key, int32_t* workgroups, int32_t* tile_w,
                            int32_t* tile_h, int32_t* found);
rt_status rt_tune_cache_put(const char* key, int32_t workgroups, int32_t tile_w, int32_t tile_h);
rt_status rt_tune_cache_forget(void);

/* ---- Interactive per-frame path ------------------------------------------
 * The paper's GUI loop streams the camera, the ray-tracing properties (shadow
 * samples, bounce limit) and the body positions in for every frame, renders,
 * and streams the pixels out (Section 3.9, its task schedule).  A frame object
 * holds that loop for one scene and one image size as a HIP graph replayed
 * once per frame with new node parameters: positions host -> device, one
 * kernel that moves the spheres and rebuilds their light and eye cones, the
 * render (rt_render_ex's or rt_render_soft's kernel), and optionally the image
 * device -> host.  Two slots alternate, so the host can stage frame k+1 while
 * the device renders frame k.  Each frame's image is bit-identical to
 * rt_scene_update (same centres) followed by rt_render_ex / rt_render_soft.
 *
 * Streamed-out formats: RT_FRAME_RGB32F, the float image itself;
 * RT_FRAME_ARGB8, the paper's integer pixels (one uint32 per pixel, alpha 255
 * in the top byte, then red, green, blue; each channel
 * floor(clamp(c, 0, 1) * 255 + 0.5) with the product and the sum rounded to
 * FP32), a third of the bytes, packed on the device before the copy. */
typedef struct rt_frame_s* rt_frame;

typedef enum { RT_FRAME_RGB32F = 0, RT_FRAME_ARGB8 = 1 } rt_frame_format;

typedef struct {
  int32_t W, H;         /* image size, 1 .. RT_MAX_DIM                          */
  int32_t soft;         /* 0: hard shadows (rt_render_ex), 1: soft (rt_render_soft) */
  int32_t stream_out;   /* non-zero: copy every image to library-owned pinned host
                           memory (rt_frame_result)                              */
  int32_t format;       /* rt_frame_format of the streamed-out image; ARGB8 needs
                           stream_out                                            */
  uint32_t flags;       /* RT_RENDER_* as rt_render_ex                          */
  float* rgb_out;       /* device float32 [H][W][3], caller-owned               */
} rt_frame_desc;

typedef struct {
  rt_camera cam;
  int32_t depth;            /* bounce limit, 0 .. RT_MAX_DEPTH                  */
  int32_t samples;          /* hard frames: 1; soft frames: 2 .. RT_MAX_SAMPLES */
  float light_radius;       /* soft frames: finite, > 0; hard frames: unused    */
  const float* sphere_pos;  /* host float32 [N][3] new sphere centres (radii and
                               everything else stay), or NULL to keep them      */
} rt_frame_input;

/* Allocates the device position buffer, two pinned staging and (stream_out)
 * two pinned image copies, for ARGB8 a device pixel buffer, and builds the
 * two graphs; not capture-safe.  The scene must outlive the frame and keep
 * its counts. */
rt_status rt_frame_create(rt_scene scene, const rt_frame_desc* desc, rt_frame* out);

/* Stage one frame and launch its graph on `stream` (every frame of one frame
 * object on the same stream).  Copies sphere_pos into the slot's pinned
 * staging before it returns, after waiting for the frame that used the slot
 * two submits ago.  Moving the spheres changes the scene itself, as
 * rt_scene_update does.  A skybox added or removed since the last frame
 * rebuilds the graphs (allocates); otherwise no allocation. */
rt_status rt_frame_submit(rt_frame frame, const rt_frame_input* in, void* stream);

/* Wait for the oldest submitted frame not yet returned, in submission order
 * (a submit that finds two frames not yet returned drops the older one, so
 * an interactive loop may submit frame k+1 before it takes frame k).  With
 * stream_out, *host_image (may be NULL) points at that frame's image, float32
 * [H][W][3] or uint32 [H][W] per the format, valid until the second
 * rt_frame_submit after the frame's own; else *host_image is NULL.
 * RT_ERR_INVALID_ARG when no frame is waiting. */
rt_status rt_frame_result(rt_frame frame, const void** host_image);

/* Waits for the frame's work, then frees it. */
rt_status rt_frame_destroy(rt_frame frame);

const char* rt_status_string(rt_status status);
const char* rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
