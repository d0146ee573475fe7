/*
 * grca.h -- C ABI of the MI355X (gfx950) emitter-centric closest-hit LiDAR
 * ray caster.
 *
 * The problem (section 1.1, "Problem Statement"): a LiDAR fires many rays into
 * a scene of triangles; for every ray find the closest triangle it intersects
 * and the distance to it.  No acceleration structure is built.  For every
 * (triangle, origin) pair the library computes the triangle's apparent
 * angular extent as seen from the emitter (sections 3.2-3.8: the channel cones
 * of section 3.2, channel and ray indexing of sections 3.3-3.4) and turns it
 * into the candidate channels and, within each channel, the candidate azimuth
 * rays (Observation 1).  Only those candidate pairs are run through a
 * ray-triangle test, and each ray keeps its closest (distance, triangle id)
 * through a 64-bit atomic minimum on a packed key (appendix "Per-Ray Distance
 * Encoding", extended by the triangle id).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units are metres and radians.  Vertex coordinates are FP32.
 *  - Status codes only; no C++ exception crosses this boundary.  On any
 *    non-OK status, grca_last_error() describes the failure and the prior
 *    state is left untouched unless stated otherwise.
 *  - A context binds one HIP device and is NOT thread-safe: callers serialise
 *    calls on one context.  Different contexts are independent.
 *  - `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it in order.
 *  - Pointers flagged GRCA_MEM_DEVICE are device pointers on the context's
 *    device; otherwise they are host pointers.  Input buffers are copied into
 *    library-owned device memory (in stream order for device pointers): the
 *    caller may reuse or free them once the call returns (host) or once the
 *    stream reaches the copy (device).
 */
#ifndef GRCA_H
#define GRCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct grca_context grca_context;
typedef struct grca_frame grca_frame;
typedef struct grca_workspace grca_workspace;

typedef enum {
  GRCA_OK = 0,
  GRCA_ERR_INVALID_ARG = 1, /* bad pointer, size, index, non-finite value, ...    */
  GRCA_ERR_OUT_OF_MEMORY = 2,
  GRCA_ERR_DEVICE = 3,      /* a HIP call failed (message carries the HIP error)   */
  GRCA_ERR_CAPACITY = 4,    /* a work queue overflowed and could not be regrown    */
  GRCA_ERR_NOT_FOUND = 5    /* unknown scene or sensor id                          */
} grca_status;

/* Triangle id written for rays that hit nothing (their distance is +inf,
 * the miss sentinel of appendix "Pipeline Overview"). */
#define GRCA_MISS_TRI 0xFFFFFFFFu

/* flags (bitwise OR) */
#define GRCA_MEM_HOST 0u             /* caller pointers are host memory                  */
#define GRCA_MEM_DEVICE 1u           /* caller pointers are device memory                */
#define GRCA_UPDATE_VERTICES_ONLY 2u /* scene_update: keep topology, indices may be NULL */
#define GRCA_CULL_BACKFACE 4u        /* cast: single-sided, only front faces count:
                                        d . ((v1 - v0) x (v2 - v0)) < 0 (counter-clockwise
                                        as seen by the ray, the Moller-Trumbore culling
                                        branch); the back-face filter of the appendix's
                                        early pass, applied per hit                      */
#define GRCA_CAST_ALL_PAIRS 8u       /* cast: test every ray against every triangle (no
                                        culling; the reference for "culling never drops
                                        a hit").  Same per-pair arithmetic, so culled and
                                        all-pairs outputs are bitwise equal.            */
/* The paper's lossy accelerations, opt-in per cast (grca_cast), off by default.
 * Each only drops candidate pairs, so every ray's result is the exact cast's or a
 * farther hit or a miss (the paper's accuracy section names them as the causes
 * of its below-100% hit rates). */
#define GRCA_LOSSY_AREA 16u          /* apparent-area cull (early pass step 1, Eq.
                                        apparent_area): skip a (triangle, origin) pair
                                        whose solid angle A (c - o) . n / |c - o|^3 is
                                        below grca_options.eps_area                    */
#define GRCA_LOSSY_CSPAN 32u         /* channel span by two binary searches with the
                                        GACP-T boolean predicate started at the channel
                                        midway between the vertices' nearest channels
                                        (section 3.6) instead of the exact elevation
                                        extent                                          */
#define GRCA_LOSSY_RSPAN 64u         /* ray span from the three vertex azimuths rounded
                                        to the nearest ray (section 3.7, Eq. all_cw),
                                        without margins; pairs failing the all-CW test
                                        take the large class                          */

/* ---- context ------------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
grca_status grca_create(int hip_device, grca_context** out);
/* Destroy a context and free every device buffer it owns (waits for its work). */
void grca_destroy(grca_context* ctx);
/* Message for the last non-OK status returned on `ctx` ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char* grca_last_error(const grca_context* ctx);

/* ---- scenes ---------------------------------------------------------------- */

/* Calls that change a scene or a sensor (grca_scene_update, _release,
 * _set_rigid, _set_deform, _pose, grca_sensor_config of an existing id,
 * grca_sensor_release) first wait for every cast and frame launch in flight
 * that reads it, on any workspace or stream, and complete any recast those
 * need with the state they were issued against.  Casts that do not read it
 * keep running. */

/* Create or replace scene `scene_id` (any 32-bit id; one context holds many
 * scenes, e.g. one per serving client): the triangle set of the problem
 * statement (section 1.1), in the world frame in which section 3.1 places the
 * emitters, as vertex and index buffers (the per-triangle vertex data the
 * appendix's early pass reads once per frame).
 *  vertices_xyz: num_vertices * 3 FP32, xyz-interleaved.  Stored on the device
 *                as 16-byte (x, y, z, 0) records, one load per vertex.
 *  indices:      num_triangles * 3 uint32; triangle k uses vertices
 *                indices[3k..3k+2] and is reported as id k.
 *  flags:        GRCA_MEM_DEVICE for device pointers; GRCA_UPDATE_VERTICES_ONLY
 *                rewrites positions only (num_vertices must equal the scene's).
 * Errors: INVALID_ARG for an index >= num_vertices, a non-finite coordinate
 * (host inputs are validated on the host; device inputs by a device pass
 * before the scene is replaced), num_triangles >= 2^28 or num_vertices >=
 * 2^28 (kernels address both by 32-bit byte offsets).  Synchronous with
 * respect to `hip_stream` for host inputs. */
grca_status grca_scene_update(grca_context* ctx, uint32_t scene_id, const float* vertices_xyz,
                              uint32_t num_vertices, const uint32_t* indices,
                              uint32_t num_triangles, uint32_t flags, void* hip_stream);
/* Copy the scene's current vertex positions (after any pose) into
 * vertices_xyz_host (num_vertices * 3 FP32, xyz-interleaved).  Waits for
 * `hip_stream`. */
grca_status grca_scene_download(grca_context* ctx, uint32_t scene_id, float* vertices_xyz_host,
                                void* hip_stream);
/* Free scene `scene_id` and its dynamic-geometry tables. */
grca_status grca_scene_release(grca_context* ctx, uint32_t scene_id);

/* Dynamic geometry (the per-frame re-posing of dynamic meshes, section 5
 * "Dynamic meshes"; evaluated on the device in FP64 and rounded once to FP32).
 *
 * grca_scene_set_rigid: declare `num_instances` rigid instances; instance i
 * owns vertices [vertex_start[i], vertex_start[i] + vertex_count[i]).  The
 * scene's current positions of those ranges become the instances' rest
 * positions.  Ranges must be disjoint and inside the scene (host arrays). */
grca_status grca_scene_set_rigid(grca_context* ctx, uint32_t scene_id, uint32_t num_instances,
                                 const uint32_t* vertex_start, const uint32_t* vertex_count,
                                 void* hip_stream);

/* One deformable vertex range: v = v_rest + amplitude * sin(omega * t + phase_v) * n_v. */
typedef struct {
  uint32_t vertex_start;
  uint32_t vertex_count;
  float amplitude; /* metres  */
  float omega;     /* rad / s */
} grca_deform_group;

/* grca_scene_set_deform: declare deformable ranges.  normals_xyz and phases
 * (host arrays) hold sum(vertex_count) entries in group order.  The current
 * positions of those ranges become the rest positions. */
grca_status grca_scene_set_deform(grca_context* ctx, uint32_t scene_id, uint32_t num_groups,
                                  const grca_deform_group* groups, const float* normals_xyz,
                                  const float* phases, void* hip_stream);

/* Re-pose the dynamic geometry: rigid instance i gets v = M_i[:, 0:3] v_rest +
 * M_i[:, 3] (instance_matrices: num_instances row-major 3x4 FP32, host or
 * device per flags; may be NULL if the scene has no rigid instances), and the
 * deformable ranges are evaluated at time `time_s`.  Asynchronous on
 * hip_stream. */
grca_status grca_scene_pose(grca_context* ctx, uint32_t scene_id, const float* instance_matrices,
                            double time_s, uint32_t flags, void* hip_stream);

/* ---- sensors ---------------------------------------------------------------- */

/* A spinning LiDAR (section 3.1).  Ray (C, R) has elevation
 * phi_C = channel_elevation_rad[C] and azimuth
 * theta_R = (R - floor(rays_per_channel / 2)) * fov_rad / rays_per_channel,
 * and direction d = cos(theta) cos(phi) f + sin(theta) cos(phi) r + sin(phi) u
 * (Eq. ray_dir).  theta grows from `forward` toward `right`. */
typedef struct {
  uint32_t scene_id;                  /* scene this sensor observes                        */
  float origin[3];                    /* o                                                 */
  float forward[3], right[3], up[3];  /* f, r, u: orthonormal within 1e-6                  */
  uint32_t num_channels;              /* gamma in [1, 65535]                               */
  const float* channel_elevation_rad; /* gamma host values, strictly ascending, in
                                         [-pi/2 - 1e-6, pi/2 + 1e-6]; C = 0 is the lowest   */
  uint32_t rays_per_channel;          /* chi in [1, 65535]                                 */
  float fov_rad;                      /* (0, 2 pi]; |fov - 2 pi| <= 1e-6 means a full spin
                                         whose azimuth index wraps                          */
  float range_min, range_max;         /* a hit counts iff t in [range_min, range_max];
                                         0 < range_min <= range_max < +inf                  */
  const float* azimuth_offset_rad;    /* optional (NULL = none), chi host values: ray R has
                                         azimuth theta_R + offset_R (angular noise, appendix
                                         "Ray Noise Simulation"); |offset_R| <= fov / chi   */
  const uint8_t* ray_mask;            /* optional (NULL = all on), gamma * chi host values
                                         at C * chi + R: 0 switches ray (C, R) off; it then
                                         reports a miss (non-spinning / animated patterns)  */
  const float* channel_elevation_offset_rad; /* optional (NULL = none), gamma host values:
                                         channel C's rays have elevation phi_C + offset_C
                                         (per-channel vertical noise, appendix "Ray Noise
                                         Simulation"); |phi_C + offset_C| <= pi/2; the
                                         perturbed elevations need not stay ascending       */
} grca_sensor_desc;

/* Create or replace sensor `sensor_id`.  Builds the per-sensor channel and
 * azimuth tables on the device.  Errors: INVALID_ARG (see field comments),
 * NOT_FOUND is NOT raised here: the scene is looked up at cast time. */
grca_status grca_sensor_config(grca_context* ctx, uint32_t sensor_id, const grca_sensor_desc* s);
grca_status grca_sensor_release(grca_context* ctx, uint32_t sensor_id);

/* ---- casting -------------------------------------------------------------- */

/* Cast every ray of the listed sensors in one batched pass (one bounds pass
 * over each referenced scene for all its listed sensors, one device work
 * queue for all of them).  Sensors may observe different scenes.
 *
 * Output layout (appendix, early pass step 5, g(j, i)): the result for list
 * position n, channel C, ray R is at O_n + C * chi_n + R with
 * O_n = sum_{m < n} gamma_m * chi_m.
 *  out_distance: metres along the unit ray, +INFINITY on a miss.
 *  out_tri:      triangle id, GRCA_MISS_TRI on a miss.  Either output may be
 *                NULL.  Host or device per GRCA_MEM_DEVICE.
 * With device outputs the call is asynchronous on hip_stream; with host
 * outputs it returns after the results are copied.  Equal FP32 distances
 * resolve to the smaller triangle id, so results are bitwise reproducible and
 * independent of batch composition.  A work-queue overflow is detected on
 * the device; the library grows the queue and recasts (at once for host
 * outputs, at grca_synchronize for device outputs). */
grca_status grca_cast(grca_context* ctx, const uint32_t* sensor_ids, uint32_t num_sensors,
                      float* out_distance, uint32_t* out_tri, uint32_t flags, void* hip_stream);

/* Wait for the context's work on hip_stream, surface asynchronous errors and
 * complete any recast an overflow requires. */
grca_status grca_synchronize(grca_context* ctx, void* hip_stream);

/* Counters of the most recent cast (waits for it). */
typedef struct {
  uint64_t rays;          /* rays cast                                               */
  uint64_t pairs_tested;  /* (triangle, origin) pairs the bounds pass examined       */
  uint64_t rect_items;    /* small-class (rectangle) work items                      */
  uint64_t large_records; /* large-class (triangle, origin) records                  */
  uint64_t row_items;     /* per-channel work items expanded from large records      */
  uint64_t rtic;          /* ray-triangle intersection checks executed               */
  uint32_t recasts;       /* overflow-driven recasts                                 */
  uint32_t overflowed;    /* casts (for a frame: launches since it was created) whose
                             work queues overflowed; each was recast or reported      */
  uint64_t pairs_evaluated; /* of pairs_tested: those whose span the bounds pass
                               computed (kept by the tile's and by the triangle's own
                               bounding-sphere test)                                 */
  uint64_t sphere_tests;    /* of pairs_tested: those not culled by the tile's bounding-
                               sphere test, tested against the triangle's own sphere */
  uint64_t atomics;         /* 64-bit atomic minima the intersection pass issued on the
                               per-ray keys (hits not ruled out by the key read first)  */
} grca_stats;
grca_status grca_last_stats(grca_context* ctx, grca_stats* out);

/* ---- options ----------------------------------------------------------------- */

/* Tunables.  The split between the small (rectangle) and large (per-channel)
 * classes follows Eq. sat_cond: a (triangle, origin) pair is small iff its
 * azimuth arc does not cover the full circle, gamma_span <= small_channels and
 * chi_span <= small_rays (the paper's default is (64, 64), Table
 * tunable_params). */
typedef struct {
  uint32_t small_channels;   /* gamma_T, 1..255                                        */
  uint32_t small_rays;       /* chi_T, 1..65535                                        */
  uint32_t row_chunk;        /* max rays per per-channel work item (W), 1..65535       */
  uint32_t bounds_block;     /* threads per block of the bounds pass: 64..1024, x64    */
  uint32_t persist_waves_cu; /* resident waves per CU of the persistent kernels, 1..32 */
  uint32_t group_cull;       /* 1: cull each wave's 128 triangles per sensor with one
                                bounding-sphere test first (the group-level cone test
                                of section 8, "Future Work"); never changes results */
  uint32_t inline_max;       /* small-class rectangles of at most this many candidate
                                rays are intersected inside the bounds pass (the early
                                pass's inline RTIC of Alg. 1); 0 sends every rectangle
                                through the work queue; never changes results          */
  uint32_t isect_ticket;     /* candidate pairs per ticket of the intersection pass
                                (a wave's unit of dynamic work), 64..2^20, multiple
                                of 64; never changes results                          */
  float eps_area;            /* epsilon_A of GRCA_LOSSY_AREA (steradians), finite, >= 0;
                                default 1e-6 (Table tunable_params)                   */
  uint64_t item_capacity;    /* initial work-queue capacity (items)                    */
  uint64_t large_capacity;   /* initial large-record queue capacity                    */
} grca_options;
grca_status grca_get_options(const grca_context* ctx, grca_options* out);
grca_status grca_set_options(grca_context* ctx, const grca_options* opt);

/* ---- frames: a hipGraph-captured pose + batched cast --------------------------- */

/* Capture "pose the scene's dynamic geometry, then cast the listed sensors"
 * into a HIP graph with its own work buffers.  Outputs are device pointers
 * that the graph writes on every launch; they must stay valid for the
 * frame's lifetime.  All sensors must observe `scene_id`. */
grca_status grca_frame_create(grca_context* ctx, uint32_t scene_id, const uint32_t* sensor_ids,
                              uint32_t num_sensors, float* out_distance_dev,
                              uint32_t* out_tri_dev, grca_frame** out);
/* Launch one frame: copy the instance matrices (host, may be NULL) and time
 * into the frame's pose block, then replay the graph on hip_stream.  Launches
 * may be issued back to back without synchronising; each one overwrites the
 * frame's outputs.  If the frame's scene or one of its sensors was
 * reallocated since the last launch (grca_scene_update with a new topology,
 * grca_scene_set_rigid / _set_deform, grca_sensor_config of one of its
 * sensors), the graph is re-captured first; NOT_FOUND if one was released,
 * INVALID_ARG if a sensor now observes another scene. */
grca_status grca_frame_launch(grca_frame* frame, const float* instance_matrices, double time_s,
                              void* hip_stream);
/* Wait for the frame's launches and check every launch since the last
 * synchronize for a work-queue overflow (the overflow record accumulates on
 * the device across launches).  On overflow the frame's queues are grown and
 * the graph is re-captured; if the last launch overflowed it is run again, so
 * the outputs are complete on return.  Returns CAPACITY (after growing) when
 * an EARLIER launch overflowed: its outputs, already overwritten or copied
 * out by the caller, were incomplete (the deferred list's capacity is "never
 * reached" in appendix "BAT list allocation"; here it is never exceeded
 * silently). */
grca_status grca_frame_synchronize(grca_frame* frame, void* hip_stream);
void grca_frame_destroy(grca_frame* frame);
/* One frame exactly as grca_frame_launch runs it (same kernels, buffers and
 * arguments), but launched stage by stage on hip_stream with HIP events
 * recorded between the stages; waits and returns the device time of each
 * stage in ms6: [0] pose, [1] key init, [2] bounds + binning, [3] large-class
 * expansion, [4] intersection, [5] resolve. */
grca_status grca_frame_profile(grca_frame* frame, const float* instance_matrices, double time_s,
                               void* hip_stream, float* ms6);

/* ---- workspaces: concurrent casts (serving) ------------------------------------ */

/* A workspace owns the transient buffers of one cast in flight (ray keys,
 * work queues, counters).  Casts on different workspaces may overlap on
 * different streams.  `max_rays` bounds the rays of one cast on it.
 * *bytes_out (optional) receives the device memory it holds. */
grca_status grca_workspace_create(grca_context* ctx, uint64_t max_rays, uint64_t item_capacity,
                                  grca_workspace** out, uint64_t* bytes_out);
void grca_workspace_destroy(grca_workspace* ws);
/* As grca_cast, on workspace `ws`; device outputs only (asynchronous). */
grca_status grca_cast_ws(grca_context* ctx, grca_workspace* ws, const uint32_t* sensor_ids,
                         uint32_t num_sensors, float* out_distance_dev, uint32_t* out_tri_dev,
                         void* hip_stream);
/* As grca_synchronize for one workspace: waits for its cast and recasts on overflow. */
grca_status grca_workspace_synchronize(grca_context* ctx, grca_workspace* ws, void* hip_stream);
/* As grca_last_stats for the most recent cast on workspace `ws` (waits for it). */
grca_status grca_workspace_stats(grca_context* ctx, grca_workspace* ws, grca_stats* out);

/* ---- a cast that allocates nothing ---------------------------------------------- */

/* For callers that cannot allocate device memory: code recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * As grca_cast with device outputs (GRCA_MEM_DEVICE must be set; the
 * optional flag is GRCA_CULL_BACKFACE), except that every transient buffer
 * (counters, the cast's sensor and scene descriptors, the per-ray keys and
 * the work queues) is carved from one static device array of
 * GRCA_NOALLOC_SCRATCH_BYTES per device, which the library holds from
 * grca_create until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree or host heap) and is asynchronous on hip_stream; the
 * scene and sensors must have been set up beforehand.
 * Limits and errors:
 *  - at most GRCA_NOALLOC_MAX_SENSORS sensors; INVALID_ARG beyond, for host
 *    outputs, or for GRCA_CAST_ALL_PAIRS;
 *  - CAPACITY at once when the cast's rays leave too little of the array for
 *    its work queues (8 bytes per ray of keys plus at least
 *    GRCA_NOALLOC_MIN_QUEUE_BYTES): the outputs are not written;
 *  - the work queues get the rest of the array, at most
 *    grca_options.item_capacity / large_capacity entries.  A queue overflow
 *    cannot be recast here (that would allocate): grca_synchronize on the
 *    same stream returns CAPACITY for it, and those outputs are incomplete.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (other streams, other
 * contexts, other threads) race and corrupt each other's results.  Calls
 * issued one after another on one stream do not overlap. */
#define GRCA_NOALLOC_SCRATCH_BYTES (64u << 20)
#define GRCA_NOALLOC_MAX_SENSORS 64u
#define GRCA_NOALLOC_MIN_QUEUE_BYTES (2u << 20)
grca_status grca_cast_noalloc(grca_context* ctx, const uint32_t* sensor_ids, uint32_t num_sensors,
                              float* out_distance_dev, uint32_t* out_tri_dev, uint32_t flags,
                              void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* GRCA_H */
