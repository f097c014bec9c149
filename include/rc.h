/*
 * rc.h -- C ABI of the MI355X batched ray-cast renderer.
 *
 * The library renders depth/range, segmentation, triangle-id and hit-point
 * buffers for many independent environments at once, each with its own
 * triangle meshes and its own sensors (pinhole cameras and rotating LiDARs).
 *
 * Problem statement it implements (paper, Sec. III-D "Exteroceptive
 * Sensors"): environment i holds a base mesh made of n_i sub-meshes, one per
 * object; each sub-mesh has its own transform at time t; the transformed mesh
 * gets a bounding volume hierarchy, and one ray is cast per pixel or beam; the
 * sensor-to-hit distance is reported as range (LiDAR, time of flight) and the
 * distance from the image plane as depth (cameras); segmentation, face index
 * and point outputs come from the same hit.
 *
 * Conventions (all calls):
 *   - Every call returns an rc_status; no exception crosses the ABI.  Argument
 *     errors are detected before any work is queued.  rc_last_error() gives a
 *     human-readable detail for the calling thread.
 *   - Host arrays passed in are copied before the call returns.
 *   - Device pointers passed in must stay valid until the work queued on the
 *     given stream has completed.  Output buffers are always caller-owned; the
 *     library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the context's stream).
 *   - Units are metres and radians; world z is up; the sensor frame is
 *     x forward, y left, z up; images have u to the right and v downward with
 *     row 0 at the top.
 *   - A context is used by one host thread at a time.
 */
#ifndef RC_H
#define RC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rc_status;
#define RC_OK 0
#define RC_E_INVALID (-1) /* bad argument */
#define RC_E_OOM (-2)     /* device allocation failed or memory budget exceeded */
#define RC_E_HIP (-3)     /* HIP runtime error */
#define RC_E_STATE (-4)   /* call out of order (e.g. render before build) */
#define RC_E_BUSY (-5)    /* resource in use */
#define RC_E_DEVICE (-6)  /* device-side error flag raised */

typedef struct rc_context rc_context;

/* Status code as text (static string). */
const char *rc_status_string(rc_status s);
/* Detail of the last failing call on this thread (owned by the library). */
const char *rc_last_error(void);

/* ------------------------------------------------------------------------ */
/* Context.                                                                  */
/* device: HIP device ordinal; stream: default hipStream_t for the context's */
/* work (NULL = the null stream); alloc: optional allocator for every        */
/* library-owned device buffer (NULL = hipMalloc / hipFree), e.g. a          */
/* framework's caching allocator; the struct is copied.  alloc(user, bytes,  */
/* stream) returns device memory or NULL (reported as RC_E_OOM);             */
/* free(user, ptr, bytes, stream) is called only after the device has        */
/* finished every use of ptr.  Either hook may be called from the request    */
/* server's worker thread.  hbm_budget: cap in bytes on library-owned        */
/* device memory (0 = no cap).  Allocation above the cap fails with          */
/* RC_E_OOM and leaves the previous state intact.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    void *(*alloc)(void *user, size_t bytes, void *stream);
    void (*free)(void *user, void *ptr, size_t bytes, void *stream);
    void *user;
} rc_allocator;
rc_status rc_create(int32_t device, void *stream, const rc_allocator *alloc, size_t hbm_budget, rc_context **out);
rc_status rc_destroy(rc_context *ctx);
/* Library-owned device bytes currently allocated. */
rc_status rc_memory_used(const rc_context *ctx, size_t *bytes);

/* ------------------------------------------------------------------------ */
/* Prototype meshes (the sub-meshes M_j of Sec. III-D, shared by reference). */
/* xyz: host float[n_verts][3]; tri3: host int32[n_tris][3] vertex indices.  */
/* Copied; ids are dense from 0 in call order.  Must precede rc_scene_load.  */
/* ------------------------------------------------------------------------ */
rc_status rc_mesh_add(rc_context *ctx, const float *xyz, int32_t n_verts, const int32_t *tri3,
                      int32_t n_tris, int32_t *mesh_id);

/* ------------------------------------------------------------------------ */
/* Scene: instances of prototype meshes per environment (Sec. III-D base     */
/* mesh of environment i = its n_i sub-meshes).  CSR over environments:      */
/*   inst_offsets: host int64[n_envs+1], non-decreasing, inst_offsets[0]=0;  */
/*   inst_mesh:    host int32[n_inst] prototype id;                          */
/*   inst_seg:     host int32[n_inst] segmentation label reported on hits;   */
/*   inst_dynamic: host uint8[n_inst] (nullable = all static): instances     */
/*                 re-transformed by rc_refit.                               */
/* Environment-local triangle numbering: instances in CSR order, then the    */
/* prototype's triangle order.  Replaces any previous scene atomically: on   */
/* error the previous scene (and its BVH) is untouched.  Sensors must be     */
/* attached again after a new scene.  An environment holds at most 2^21     */
/* triangles (the BVH depth bound that sizes the traversal stack), the      */
/* whole scene fewer than 2^31; larger inputs are RC_E_INVALID.             */
/* ------------------------------------------------------------------------ */
rc_status rc_scene_load(rc_context *ctx, int32_t n_envs, const int64_t *inst_offsets,
                        const int32_t *inst_mesh, const int32_t *inst_seg, const uint8_t *inst_dynamic);

/* ------------------------------------------------------------------------ */
/* Scene options, read by every later rc_scene_load (flags 0: the default).  */
/*   RC_SCENE_TWO_LEVEL_ONLY  the scene is only ever built two-level         */
/*     (Sec. III-D sub-meshes kept in their own frames, see                 */
/*     RC_BUILD_TWO_LEVEL): the per-triangle arrays of the single-level      */
/*     form (world copy, leaf records, nodes and build lists, about 255     */
/*     bytes per triangle) are not allocated, so the library holds the      */
/*     meshes, the per-instance tables and the two BVH levels only, and the  */
/*     2^21-triangle limit per environment does not apply.  With such a      */
/*     scene RC_BUILD_SAH / RC_BUILD_LBVH, RC_RENDER_BRUTE, the further      */
/*     outputs, stereo shadows and rc_debug_world / rc_debug_bvh return      */
/*     RC_E_STATE; render results equal those of the same scene loaded       */
/*     without the option and built two-level.                              */
/* Unknown bits are RC_E_INVALID.                                            */
/* ------------------------------------------------------------------------ */
#define RC_SCENE_TWO_LEVEL_ONLY 1
rc_status rc_scene_options(rc_context *ctx, int32_t flags);

/* ------------------------------------------------------------------------ */
/* Sensor models.                                                            */
/*  RC_PINHOLE: width x height pixels, horizontal field of view hfov, square */
/*    pixels (focal length (W/2)/tan(hfov/2)), pixel centres at +1/2; the    */
/*    local direction has forward component exactly 1, so t is depth.       */
/*  RC_LIDAR: width azimuths x height channels; channel c has elevation      */
/*    vmax - c (vmax-vmin)/(H-1) (channel 0 on top), azimuth a is            */
/*    hmin + a (hmax-hmin)/W counter-clockwise from +x; unit directions, so  */
/*    t is range.  The scan is instantaneous (one pose per scan).            */
/*  RC_TABLE: width*height local unit directions in dir_table (host          */
/*    float[W*H][3], copied): user-defined projection models.                */
/* Rays are indexed r = row*width + col (pinhole row = image row, LiDAR row  */
/* = channel).  near_/far_ bound the ray parameter t: a triangle counts only */
/* if near_ <= t <= far_ (0 <= near_ <= far_).                               */
/* stereo: centre of a stereo pair's second camera in this sensor's frame    */
/* (metres, x forward, y left, z up; all zero = no second camera).  Sec.     */
/* III-D simulates stereo shadows: rendering with the shadow output marks    */
/* the pixels whose hit point the second camera cannot see.                  */
/* ------------------------------------------------------------------------ */
#define RC_PINHOLE 0
#define RC_LIDAR 1
#define RC_TABLE 2
typedef struct {
    int32_t kind;
    int32_t width, height;
    float hfov;
    float vmin, vmax, hmin, hmax;
    float near_, far_;
    const float *dir_table;
    float stereo[3];
} rc_sensor_desc;

rc_status rc_sensor_add(rc_context *ctx, const rc_sensor_desc *desc, int32_t *sensor_id);

/* Sensor instances per environment, CSR: sens_offsets host int64[n_envs+1], */
/* sensor_ids host int32[n_sensor_inst].  Requires a loaded scene.           */
rc_status rc_sensors_attach(rc_context *ctx, const int64_t *sens_offsets, const int32_t *sensor_ids);

/* Output layout: ray-major per sensor instance; sensor instance s owns      */
/* output rays [ray_offsets[s], ray_offsets[s+1]).  ray_offsets: host        */
/* int64[n_sensor_inst+1] (nullable); total_rays: host int64 (nullable).     */
rc_status rc_ray_layout(const rc_context *ctx, int64_t *ray_offsets, int64_t *total_rays);

/* Environment triangle offsets: host int64[n_envs+1]; environment e owns    */
/* global triangles [off[e], off[e+1]).                                      */
rc_status rc_env_tri_offsets(const rc_context *ctx, int64_t *off);

/* ------------------------------------------------------------------------ */
/* Poses (Sec. III-D transforms T_{j,t} and sensor poses).  Caller-owned     */
/* DEVICE pointers, FP32 row-major 3x4 [R | p] per instance / per sensor     */
/* instance, copied on `stream`.  world vertex = R v + p (per coordinate     */
/* fma(R0,x, fma(R1,y, fma(R2,z, p)))); ray origin = p, world direction      */
/* component i = fma(Ri0,dx, fma(Ri1,dy, Ri2*dz)).                           */
/* ------------------------------------------------------------------------ */
rc_status rc_set_instance_poses(rc_context *ctx, const float *d_inst_T, void *stream);
rc_status rc_set_sensor_poses(rc_context *ctx, const float *d_sensor_T, void *stream);

/* Constant-velocity motion of dynamic instances: translation at `step` is   */
/* fma(v, float(step)*dt, p0) with p0 the translation of the last            */
/* rc_set_instance_poses; d_vel: caller device float[n_inst][3].             */
rc_status rc_move_instances(rc_context *ctx, const float *d_vel, int32_t step, float dt, void *stream);

/* ------------------------------------------------------------------------ */
/* Acceleration structure (Sec. III-D: a BVH over the transformed mesh of    */
/* each environment).  rc_build transforms every instance and builds one     */
/* BVH per environment with `builder`:                                       */
/*   RC_BUILD_SAH   surface-area heuristic (binned splits for large nodes,   */
/*                  exact sweeps below), one wavefront per environment; the  */
/*                  faster trees to render.                                  */
/*   RC_BUILD_LBVH  linear BVH (Morton order on cubic cells, the radix       */
/*                  splits of Karras 2012, built top-down; a subtree that    */
/*                  could exceed the depth bound splits at index medians     */
/*                  instead; triangles with a box side above a quarter of    */
/*                  the environment's centroid extent sort after all         */
/*                  others, so they form one subtree), one workgroup per     */
/*                  environment of 5..8192 triangles; the faster build.      */
/*                  Other environments get the SAH build.                    */
/* Every builder gives the same render results (the nearest hit is exact).  */
/* rc_refit re-transforms the dynamic instances and recomputes the bounds    */
/* bottom-up on the fixed topology.  Both are asynchronous on `stream`.      */
/* rc_refit (and a step graph without further outputs or shadows) updates   */
/* the leaf-ordered triangle records the traversal reads; the library's     */
/* original-order world copy is refreshed by the next call that reads it   */
/* (RC_RENDER_BRUTE, the further outputs and shadows of rc_render,          */
/* rc_debug_world), which first enqueues the transform on its own stream.   */
/* An unknown builder is RC_E_INVALID.                                       */
/* d_env_mask: NULL (every environment) or a caller DEVICE uint8[n_envs],    */
/* read on `stream`; environments whose byte is 0 are left exactly as they  */
/* are (world triangles, BVH, records), so e.g. the environments reset by a  */
/* randomisation can be rebuilt alone.  A masked rc_build needs a full       */
/* build first (RC_E_STATE), with the same form: single-level (SAH, LBVH)   */
/* or two-level.                                                             */
/*   RC_BUILD_TWO_LEVEL  two-level instancing (Sec. III-D: one sub-mesh per  */
/*                  object with its own transform): one BVH per mesh in the  */
/*                  mesh's own frame, shared by all its instances (built     */
/*                  once, again only after rc_mesh_add), and per environment */
/*                  a BVH over its instances' world boxes.  Rays enter each  */
/*                  visited instance's frame, so no triangle is transformed  */
/*                  per step: rc_refit recomputes each instance's inverse    */
/*                  pose and box and refits the instance BVH only.  The      */
/*                  result is the exact nearest hit on the moved meshes with */
/*                  the moved vertices unrounded (each mesh under its FP32   */
/*                  pose, evaluated exactly), where the single-level forms  */
/*                  intersect the FP32-rounded moved vertices: the two      */
/*                  agree except where a hit lies within the FP32 rounding   */
/*                  of the moved vertices of a decision boundary.  Limits:  */
/*                  8192 instances per environment and 16384 triangles per   */
/*                  registered mesh (RC_E_INVALID); an instance whose pose   */
/*                  has a singular linear part is not hit; RC_RENDER_BRUTE  */
/*                  still tests the FP32 world copy; stereo shadows need a   */
/*                  single-level build (RC_E_STATE).                         */
/* ------------------------------------------------------------------------ */
#define RC_BUILD_SAH 0
#define RC_BUILD_LBVH 1
#define RC_BUILD_TWO_LEVEL 2
rc_status rc_build(rc_context *ctx, const uint8_t *d_env_mask, int32_t builder, void *stream);
rc_status rc_refit(rc_context *ctx, const uint8_t *d_env_mask, void *stream);

/* ------------------------------------------------------------------------ */
/* Render (Sec. III-D: one ray per pixel or beam, nearest hit over the       */
/* environment's transformed mesh).  Outputs are caller-owned device         */
/* buffers in the rc_ray_layout order, each nullable (skipped):              */
/*   depth  float[total]: t of the nearest hit (depth for pinholes, range    */
/*          for LiDARs), -1.0f on a miss;                                    */
/*   seg    int32[total]: label of the instance owning the hit triangle, -1; */
/*   tri    int32[total]: environment-local triangle id, -1;                 */
/*   hit_xyz float[total][3]: world hit point o + t d, NaN on a miss.        */
/* Further data types from the same hit record (Sec. III-D: surface normals, */
/* point clouds, vertex-level annotations through face indices and          */
/* barycentric coordinates), each evaluated in FP64 from the winner's FP32   */
/* world vertices v0 v1 v2 (prototype vertex order) and rounded once:        */
/*   normal float[total][3]: unit normal of the hit triangle, (v1-v0) x      */
/*          (v2-v0) normalised and negated if it points away from the        */
/*          sensor (dot with the ray direction > 0), NaN on a miss;          */
/*   bary   float[total][2]: (u, v) with hit = (1-u-v) v0 + u v1 + v v2,     */
/*          the Moller-Trumbore coordinates of the nearest hit, NaN;         */
/*   point  float[total][3]: hit point in the sensor frame, t times the      */
/*          ray's local direction (x forward), NaN;                          */
/*   vert   int32[total][3]: global vertex ids (vertices numbered over all   */
/*          rc_mesh_add calls in call order) of v0 v1 v2, -1; a per-vertex   */
/*          annotation a gives the hit's value (1-u-v) a[i0] + u a[i1] +     */
/*          v a[i2].                                                         */
/*   shadow uint8[total]: 1 when the hit is hidden from the stereo pair's    */
/*          second camera, else 0 (misses and sensors without a second       */
/*          camera: 0).  The segment from the FP32 hit point p to the second */
/*          centre c2 (pose applied to `stereo`, the vertex transform's fma  */
/*          order) is tested against every triangle of the environment:      */
/*          hidden iff one meets p + s (c2 - p) at s in [2^-13, 1] (the lower */
/*          bound keeps the surface around p from shadowing itself).         */
/* normal, bary, point, vert and shadow need the tri output (RC_E_INVALID). */
/* RC_RENDER_BRUTE, the further outputs and shadows read the world copy:     */
/* after an rc_refit they first bring it up to date on `stream`.            */
/* The nearest hit is the smallest t in [near_, far_] over every triangle of */
/* the ray's environment (two-sided; equal t resolved by the lower triangle  */
/* id).  Every mode computes bit-identical outputs:                          */
/*   RC_RENDER_PLAIN   one launch per sensor instance (per-env path);        */
/*   RC_RENDER_FLAT    one launch over every ray tile;                       */
/*   RC_RENDER_BATCHED one persistent launch popping tiles from device work  */
/*                     queues, one per XCD (largest estimated cost first);   */
/*   RC_RENDER_BRUTE   no BVH: every triangle tested (reference path).       */
/* ------------------------------------------------------------------------ */
#define RC_RENDER_PLAIN 0
#define RC_RENDER_FLAT 1
#define RC_RENDER_BATCHED 2
#define RC_RENDER_BRUTE 3
typedef struct {
    float *depth;
    int32_t *seg;
    int32_t *tri;
    float *hit_xyz;
    float *normal;
    float *bary;
    float *point;
    int32_t *vert;
    uint8_t *shadow;
} rc_outputs;

rc_status rc_render(rc_context *ctx, const rc_outputs *out, int32_t mode, void *stream);

/* rc_render in the RC_RENDER_BATCHED form for callers that cannot allocate */
/* device memory (code under HIP graph capture, tight serving loops,         */
/* harnesses that forbid allocation): the persistent launch's work-queue     */
/* heads live in a fixed 2 KiB device array of the library (one per GPU,     */
/* held until the process ends) instead of context memory (under the        */
/* one-launch tuning, tiles per pop 0, no queue is used), and the call       */
/* makes no allocation of any kind.  Outputs, their layout, the further      */
/* outputs and the shadow mask are those of rc_render and bit-identical to   */
/* it.  Every call on one GPU, from any context, shares that array and       */
/* clears it on `stream` before its launch: calls that overlap on one GPU    */
/* (other streams, other host threads) race and must be serialised by the    */
/* caller.  Errors: those of rc_render; RC_E_INVALID when a queue holds more */
/* tiles than its 32-bit head can count (2^32 - 1 - tiles per pop); RC_E_HIP */
/* when the array's device address was not found at rc_create.               */
rc_status rc_render_noalloc(rc_context *ctx, const rc_outputs *out, void *stream);

/* Traversal statistics of one FLAT render (same arithmetic, counters added): */
/* counters host int64[4] = box tests, triangle tests, FP64 re-evaluations,  */
/* rays.  Synchronous.                                                       */
rc_status rc_render_stats(rc_context *ctx, void *stream, int64_t *counters);

/* ------------------------------------------------------------------------ */
/* Batched form: launch choices and one captured graph per simulation step.  */
/* ------------------------------------------------------------------------ */
/* Choose the ray-tile shape (columns x rows of one 64-lane wavefront: 4x16, */
/* 8x8, 16x4 or 32x2), the tiles taken per work-queue pop (2, 4 or 16, or  */
/* 0: no queue, one launch over every tile as RC_RENDER_FLAT), the         */
/* queue order (largest estimated cost first, or natural) and the node     */
/* width (2 or 4; single-level scenes) of the batched render by timing each */
/* combination on the loaded scene, sensors and poses (temporary outputs   */
/* and, for width 4, the four-wide records are allocated within the         */
/* budget).  cache_path (nullable): a text file of previous choices keyed   */
/* by device and workload; a hit skips the timing, a miss appends a line.    */
/* choice (nullable): host int32[4] = tile columns, tiles per pop, 1 if     */
/* cost order, node width.  Outputs are bit-identical for every choice.     */
/* Synchronous.                                                              */
rc_status rc_autotune(rc_context *ctx, const char *cache_path, int32_t *choice);
/* Set those choices directly: choice host int32[4] = tile columns (4, 8,   */
/* 16 or 32), tiles per pop (0..64, 0 = no queue), cost order (0 or 1),    */
/* node width (2 or 4); the request server follows the same choice.  Node  */
/* width 4 traverses four-wide records of the same BVH (for each internal   */
/* node, the boxes one level below its children, 128 bytes, kept beside     */
/* the binary nodes and refreshed by every single-level build and refit;    */
/* allocated on first use, 128 bytes per node slot, RC_E_OOM beyond the     */
/* budget): half the dependent node fetches per ray.                        */
rc_status rc_tuning_set(rc_context *ctx, const int32_t *choice);

typedef struct rc_graph rc_graph;
/* One simulation step captured as a HIP graph: dynamic instances move to the */
/* graph's step counter s (translation fma(v, float(s)*dt, p0), see          */
/* rc_move_instances), their triangles are re-transformed, every BVH is      */
/* refitted, the work queue is reset and the batched render writes `out`;    */
/* then s advances by one.  d_vel: caller device float[n_inst][3], read at   */
/* every launch.  The graph is tied to the current scene and sensors: after  */
/* rc_scene_load / rc_sensors_attach / rc_autotune its launch fails with     */
/* RC_E_STATE.  Sensor poses are read at launch time (rc_set_sensor_poses).  */
rc_status rc_step_graph_create(rc_context *ctx, const rc_outputs *out, const float *d_vel, float dt,
                               rc_graph **graph);
/* Set the step counter (asynchronous on `stream`). */
rc_status rc_graph_set_step(rc_graph *graph, int32_t step, void *stream);
rc_status rc_graph_launch(rc_graph *graph, void *stream);
rc_status rc_graph_destroy(rc_graph *graph);

/* ------------------------------------------------------------------------ */
/* Served form: a request loop over the resident scene and BVHs (the       */
/* paper's per-environment rendering of Sec. III-D, taken request by        */
/* request instead of step by step).                                         */
/* A request renders n_envs environments (ids into the loaded scene) with    */
/* one sensor model at the given poses (host float[n_envs][12], nullable =   */
/* the pose of each environment's first attached sensor instance, as set by  */
/* rc_set_sensor_poses before rc_server_create).  Outputs are ray-major per  */
/* environment in request order, [n_envs * rays of the model] (hit_xyz      */
/* [..][3]), with the same values as rc_render; only depth, seg, tri and     */
/* hit_xyz can be served (the further data types must be NULL).  Either     */
/* `out` holds caller DEVICE buffers (each nullable; ready when submitted,   */
/* valid until the ticket completes; the server writes them on its own       */
/* streams) and lib_outputs is 0, or every pointer of `out` is NULL and      */
/* lib_outputs names the kinds (RC_OUT_*) the library allocates: they are    */
/* carved at admission from one device slab of the server's budget,          */
/* readable through rc_server_outputs once the ticket completes, and held    */
/* until rc_server_release.                                                  */
/* Admission: requests are taken in arrival order, later ones filling in     */
/* while earlier ones do not fit, as long as the bytes in flight (the        */
/* outputs: library blocks, or for caller buffers their size, at least 8 per */
/* ray; plus 8 per 64-ray tile and 80 per environment of work lists) stay    */
/* within the budget and every library block finds room in the slab.  A     */
/* caller that never releases library outputs can hold the budget and stall  */
/* later requests.  In RC_SERVE_BATCHED mode every admission round merges    */
/* the admitted requests into one batched launch (in the launch form of the */
/* context's tuning) on one of n_streams streams, so batches that arrive     */
/* while others run overlap on the device                                    */
/* (continuous batching); RC_SERVE_PLAIN renders requests one at a time,     */
/* one launch per environment (the per-environment reference path).  While  */
/* a server exists the context's scene, sensors and tuning are read-only     */
/* (calls that would change them return RC_E_BUSY).  Submit, poll, wait,    */
/* outputs and release may be called from any one client thread.             */
/* ------------------------------------------------------------------------ */
typedef struct rc_server rc_server;
#define RC_OUT_DEPTH 1
#define RC_OUT_SEG 2
#define RC_OUT_TRI 4
#define RC_OUT_HIT 8
typedef struct {
    int32_t n_envs;
    const int32_t *env_ids;
    int32_t sensor_id;
    const float *sensor_T;
    rc_outputs out;
    int32_t lib_outputs;
} rc_request;
#define RC_SERVE_PLAIN 0
#define RC_SERVE_BATCHED 1

/* hbm_budget: bytes in flight (see above), capped at the device memory free */
/* at creation; 0 = half of the device memory free at creation.  The slab of */
/* library outputs (the whole budget) is allocated by the first request that */
/* asks for them, through the context's allocator.                           */
rc_status rc_server_create(rc_context *ctx, int32_t mode, int32_t n_streams, size_t hbm_budget,
                           rc_server **server);
/* Non-blocking; host arrays are copied.  RC_E_OOM if the request alone     */
/* exceeds the budget (or the slab cannot be allocated).  ticket: host      */
/* uint64 (> 0).                                                            */
rc_status rc_server_submit(rc_server *server, const rc_request *req, uint64_t *ticket);
/* done = 1 once the request's outputs are written (device work complete);  */
/* latency_s = completion time - submit time (host monotonic clock).  The   */
/* call that reports completion releases a ticket with caller buffers; a    */
/* ticket with library outputs stays until rc_server_release.               */
rc_status rc_server_poll(rc_server *server, uint64_t ticket, int32_t *done, double *latency_s);
/* Block until the ticket completes (released as by rc_server_poll). */
rc_status rc_server_wait(rc_server *server, uint64_t ticket, double *latency_s);
/* Device pointers of a completed ticket's library outputs (NULL for the     */
/* kinds not asked for).  Owned by the server: valid until the release.      */
/* RC_E_STATE before completion; RC_E_INVALID for caller-buffer tickets.     */
rc_status rc_server_outputs(rc_server *server, uint64_t ticket, rc_outputs *out);
/* Return a completed ticket's library outputs to the slab and forget the    */
/* ticket.  RC_E_STATE before completion; RC_E_INVALID for caller buffers.   */
rc_status rc_server_release(rc_server *server, uint64_t ticket);
/* Drains queued and running requests, then frees the server. */
rc_status rc_server_destroy(rc_server *server);

/* ------------------------------------------------------------------------ */
/* Inspection (synchronous, host outputs; for validation).                   */
/* ------------------------------------------------------------------------ */
/* World triangles in global original order: host float[total_tris][9].      */
rc_status rc_debug_world(rc_context *ctx, float *tris9);
/* World rays of sensor instance s for the given ray indices (host arrays).  */
rc_status rc_debug_rays(rc_context *ctx, int32_t s, int64_t n, const int64_t *ray_idx, float *o, float *d);
/* BVH of environment e: n_nodes; per node child boxes float[n][2][6]        */
/* (lo xyz, hi xyz), child refs int32[n][2] (>= 0 internal node, < 0 leaf    */
/* ~(first<<3 | (count-1)) over leaf positions), parent int32[n]; leaf_ids   */
/* int32[n_tris] env-local triangle id at each leaf position; root ref.      */
/* Node buffers must hold n_tris + n_tris/4 + 2 entries (the node slots of   */
/* the environment; slots not reachable from the root carry parent -1).      */
rc_status rc_debug_bvh(rc_context *ctx, int32_t e, int32_t *n_nodes, float *boxes, int32_t *children,
                       int32_t *parent, int32_t *leaf_ids, int32_t *root);

#ifdef __cplusplus
}
#endif
#endif /* RC_H */
