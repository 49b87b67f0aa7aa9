/*
 * rc.h - multi-camera depth ray casting for massively parallel robot
 * environments on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Sec. 3.2.2 and Algorithm 1, "Multi-Depth Ray Casting
 * Kernel"): for every environment e, camera c and pixel (x, y), cast the
 * camera ray against the environment's posed robot link meshes and one
 * shared static terrain mesh and report the closest hit clipped by a far
 * plane; then apply the sensor model the paper names (latency, noise and
 * dropout: Sec. 1, Sec. 4.1, Table 6).
 *
 * Conventions shared by every call:
 *  - Pointers named in a struct or argument as "device" must point to device
 *    memory of the current HIP device; "host" pointers to host memory.  All
 *    arrays are C-contiguous, little endian, with the shapes given.
 *  - The library never allocates device memory.  Every call that needs
 *    device storage takes a caller-owned workspace whose size the matching
 *    rc_*_size query returns; the workspace must be 256-byte aligned.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = the null stream) unless stated otherwise.  Inputs must stay
 *    valid until the stream reaches the call; outputs are valid after it.
 *  - Every call validates its arguments on the host before it enqueues
 *    anything; an error leaves outputs untouched.  No C++ exception crosses
 *    this interface.  rc_last_error() gives the text of the last error of
 *    the calling thread.
 *  - Threads: a scene's meshes and hierarchies are read-only after
 *    creation, and renders on different streams with their own outputs and
 *    workspaces may run concurrently from several threads.  The one mutable
 *    part of a scene is its pair of launch schedules (rc_set_render_config,
 *    rc_autotune), each stored as one word: a render reads a whole schedule,
 *    old or new, never a mix; the walk's stack cap (rc_set_walk_stack_limit)
 *    is one word too.  rc_robot_meshes, rc_scene_rebuild_sah and
 *    rc_scene_destroy must not overlap any other call on the same scene.
 *  - Frames: quaternions are (x, y, z, w) and rotate local vectors to world;
 *    they are normalised before use.  A camera's optical frame has x right,
 *    y down, z forward.  Intrinsics are (fx, fy, cx, cy) in pixels; pixel
 *    (x, y) looks through (x + 0.5, y + 0.5).
 *  - Ids: inst = b in [0, n_links) for link b, inst = n_links for the
 *    terrain, -1 for a miss; tri is the triangle's index in the mesh it came
 *    from (link-local index for links, input index for the terrain), -1 for
 *    a miss.  A miss reports depth = far plane.
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
#define RC_ERR_INVALID_ARG (-1)  /* bad argument, nothing enqueued */
#define RC_ERR_WORKSPACE (-2)    /* workspace too small or misaligned */
#define RC_ERR_DEVICE (-3)       /* a HIP call failed; see rc_last_error() */
#define RC_ERR_STATE (-4)        /* call out of order (e.g. a skipped step) */
#define RC_ERR_UNSUPPORTED (-5)  /* valid input the library cannot handle */

typedef void* rc_stream; /* hipStream_t */
typedef struct rc_scene rc_scene;
typedef struct rc_post rc_post;

/* Library version as 10000 * major + 100 * minor + patch. */
int32_t rc_version(void);
/* Static text for a status code. */
const char* rc_status_string(rc_status st);
/* Text of the last error on the calling thread ("" if none). */
const char* rc_last_error(void);

/* ---------------------------------------------------------------------
 * Static terrain (Algorithm 1's M_terrain, shared by all environments).
 * ------------------------------------------------------------------- */

/* Workspace bytes rc_scene_create needs for n_tri >= 1 terrain triangles. */
rc_status rc_scene_size(int64_t n_tri, size_t* ws_bytes);

/* Build the terrain's bounding volume hierarchy (a linear BVH over 63-bit
 * Morton codes, LDS radix sort, bottom-up boxes) into `ws`, and create the
 * scene handle (host memory, owned by the caller until rc_scene_destroy).
 *   tri  device float [n_tri][3][3]: world-frame vertices (m).  Not kept:
 *        it may be freed once `stream` has passed this call.
 *   ws   device, ws_bytes >= rc_scene_size(n_tri); must outlive the scene.
 * Synchronises `stream` once (to check the hierarchy depth).  Errors:
 * INVALID_ARG (n_tri < 1 or > 2^31 - 2, NULL pointers), WORKSPACE,
 * UNSUPPORTED (a hierarchy deeper than 64 levels), DEVICE. */
rc_status rc_scene_create(const float* tri, int64_t n_tri, void* ws, size_t ws_bytes,
                          rc_stream stream, rc_scene** out);

/* Rebuild hierarchies of the scene in place with a top-down binned
 * surface-area-heuristic split (MacDonald and Booth 1990; 32 bins per axis
 * over the centroid bounds, as in Wald 2007; one triangle per leaf), on the
 * host: the terrain (which & 1) and the link meshes present (which & 2).
 * Both are static (Sec. 3.2.2: built once, the links in their local frames),
 * so a build of higher quality than the Morton one pays for itself in every
 * later ray.  The workspace layout, the triangles' ids and every render's
 * results are the same; walks visit fewer records.  The Morton keys in the
 * workspace then no longer follow the leaf order, and a link's directory box
 * stays the Morton root's (a bound of the same mesh).  Reads each mesh back
 * from its workspace, builds on up to 16 host threads (the subtrees below
 * the top levels in parallel, with the same result; about 0.8 s for 2M
 * triangles on 8 cores), uploads the records, leaf-order triangles and ids and rebuilds
 * the 4-wide records on `stream`, and synchronises it.  Must not overlap any
 * other call on the scene.  Errors: INVALID_ARG (NULL scene, which not in
 * 1..3), UNSUPPORTED (a hierarchy would be deeper than 64 levels; that one
 * is unchanged), DEVICE (after which the scene must be destroyed). */
rc_status rc_scene_rebuild_sah(rc_scene* scene, int32_t which, rc_stream stream);

/* The same builder on host arrays, for tests and offline use: n_tri >= 1
 * triangles tri (host float [n_tri][3][3]) -> records (host float
 * [max(n_tri - 1, 1)][16], the node record layout of rc_bvh_layout_of),
 * tris_out (host float [n_tri][9], leaf order; must not alias tri), ids_out
 * (host int32 [n_tri], input index of each leaf), depth (deepest record,
 * root 0).  No device work.  Errors: INVALID_ARG. */
rc_status rc_sah_build_host(const float* tri, int64_t n_tri, float* records, float* tris_out,
                            int32_t* ids_out, int32_t* depth);

/* Release the handle (not the caller's workspaces). NULL is a no-op. */
rc_status rc_scene_destroy(rc_scene* scene);

/* ---------------------------------------------------------------------
 * Robot body meshes ({M_b}, kept canonical in their local frames, Sec. 3.2.2).
 * ------------------------------------------------------------------- */

/* Workspace bytes for n_links meshes; tri_offset host int64 [n_links + 1],
 * tri_offset[0] = 0, non-decreasing, each mesh >= 1 triangle. */
rc_status rc_robot_size(const int64_t* tri_offset, int32_t n_links, size_t* ws_bytes);

/* Build one hierarchy per link in its local frame into `ws` and attach them
 * to the scene (replacing any earlier set).  The meshes are shared by every
 * environment; only poses are per environment.
 *   link_tri   device float [tri_offset[n_links]][3][3], link-local (m)
 *   tri_offset host int64 [n_links + 1]
 * 0 <= n_links <= 64 (0 detaches the robot).  Synchronises `stream` once. */
rc_status rc_robot_meshes(rc_scene* scene, const float* link_tri, const int64_t* tri_offset,
                          int32_t n_links, void* ws, size_t ws_bytes, rc_stream stream);

/* ---------------------------------------------------------------------
 * Rendering (Algorithm 1).
 * ------------------------------------------------------------------- */

#define RC_DEPTH_PLANAR 0 /* optical-z depth (what depth cameras report) */
#define RC_DEPTH_RANGE 1  /* distance along the ray */

/* Perception randomisation of the cameras (the paper's Table 6: depth camera
 * translation, rotation as Euler angles and field of view, each uniform in a
 * symmetric range), drawn on the device per camera and launch.  For camera
 * uid u (plain form: env * n_cam + cam; batched form: the descriptor's
 * cam_uid) the words of Philox4x32-10 with key = seed and counter
 * (u, 0xFFFFFFFE, epoch_lo32, (epoch_hi16 << 16) | s) give, for s = 2,
 * (tx, ty, tz, phi) and, for s = 3, (theta, psi, dfov, unused), each as
 * a (2u - 1) with u = (w >> 8) 2^-24 and a the half-range.  The translation is
 * in the camera's own frame, the rotation is R Rx(phi) Ry(theta) Rz(psi)
 * (about the camera's x, y, z), and the field of view of both axes changes
 * by dfov: f' = c / tan(atan(c / f) + dfov / 2) (skipped when dfov_deg = 0).
 * Computed in FP64 once per camera; epoch lets the caller redraw (e.g. per
 * episode).  Half-ranges must be finite and >= 0, dfov_deg < 90. */
typedef struct {
    uint64_t seed;
    uint64_t epoch;
    float trans_m[3];    /* half-ranges of the offsets along the camera's x, y, z (m) */
    float euler_deg[3];  /* half-ranges of the rotations about x, y, z (degrees) */
    float dfov_deg;      /* half-range of the field-of-view change (degrees) */
    float reserved;
} rc_cam_rand;

typedef struct {
    int32_t n_env, n_cam, width, height;
    const float* link_pos;  /* device [n_env][n_links][3]: t_b per env (world, m) */
    const float* link_quat; /* device [n_env][n_links][4]: q_b per env */
    const float* cam_pos;   /* device [n_env][n_cam][3]: camera centre p_c (world) */
    const float* cam_quat;  /* device [n_env][n_cam][4]: optical -> world */
    const float* intr;      /* device [n_env][n_cam][4]: fx, fy, cx, cy (batched K) */
    float far_plane;        /* d_max (m), in (0, 1e20]: boxes that no ray may reach are
                               stored as the point (1e30, 1e30, 1e30) */
    int32_t depth_mode;     /* RC_DEPTH_PLANAR or RC_DEPTH_RANGE */
    float* depth;           /* device out [n_env][n_cam][height][width] (m) */
    int32_t* inst;          /* device out, same shape, or NULL */
    int32_t* tri;           /* device out, same shape, or NULL */
    void* const* timing;    /* NULL, or host array of two hipEvent_t recorded on the
                               stream just before and after the fast-pass kernel */
    const rc_cam_rand* cam_rand; /* NULL, or host struct: randomise the cameras */
} rc_render_args;

/* Workspace bytes of rc_render for n_env x n_cam images of width x height:
 * the per-environment top-level hierarchies over the link instances (rebuilt
 * on every call) and the list of rays handed to the exact pass. */
rc_status rc_render_size(const rc_scene* scene, int32_t n_env, int32_t n_cam, int32_t width,
                         int32_t height, size_t* ws_bytes);

/* Rebuild every environment's top-level hierarchy from its link poses, then
 * cast one ray per (env, cam, pixel): link hits first, then the terrain under
 * the shrunken bound, closest hit kept (ties: lower inst, then lower tri).
 * A hit counts when 0 < depth <= far_plane.  Hit decisions are exact: when
 * a ray's closest hit could hinge on triangle edge tests FP32 cannot decide,
 * a second pass repeats those tests in FP64 (for up to two such triangles
 * per ray) or re-casts the ray with FP64 decisions (more).  Errors:
 * INVALID_ARG (sizes < 1, width or height > 65535, more than 2^32 - 1 rays,
 * NULL required pointers, bad mode), WORKSPACE, STATE (no terrain), DEVICE.
 * The workspace's first bytes after the top level hold the exact-pass ray
 * counts (two uint32) of the last call; see rc_render_exact_count. */
rc_status rc_render(const rc_scene* scene, const rc_render_args* args, void* ws,
                    size_t ws_bytes, rc_stream stream);

/* rc_render for callers that cannot allocate device memory or hand over a
 * workspace (code under stream capture, tight serving loops, hosts that
 * forbid allocation).  Same arguments, results and errors as rc_render,
 * without ws: the workspace is a static device array of the library, 32 MiB
 * per GPU, held from the library's first use on that GPU until the process
 * ends, and the call itself allocates nothing.  It holds the top level of up
 * to about 7,200 environments of 30 links and two cameras and an exact-pass
 * list of 2^17 rays (a render that hands more rays to the exact pass re-casts every pixel
 * exactly: correct, slower).  A render whose workspace would exceed 32 MiB
 * fails with RC_ERR_WORKSPACE before anything is enqueued.  The array of the
 * current device is used (the stream must belong to it), and every call on
 * a GPU shares it: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Each call writes all
 * it reads, so no state carries over between calls. */
rc_status rc_render_noalloc(const rc_scene* scene, const rc_render_args* args, rc_stream stream);

/* Number of rays the last rc_render on this workspace sent to the exact pass
 * (a diagnostic), and how many of them it re-cast in full (`recast`, may be
 * NULL).  Synchronises `stream`. */
rc_status rc_render_exact_count(const rc_scene* scene, int32_t n_env, int32_t n_cam,
                                int32_t width, int32_t height, const void* ws, int64_t* count,
                                int64_t* recast, rc_stream stream);

/* Diagnostic render: rc_render (same workspace, same outputs) whose fast
 * pass also writes, per ray, the work it did as uint32 [n_env][n_cam]
 * [height][width][4] = (node records whose child boxes the ray's lane
 * tested, triangles tested, link instances entered, the part of the node
 * records that belong to link hierarchies) into `counts`
 * (device, 16-byte aligned, caller owned).  Node records read by a
 * wavefront's shared top-level walk and terrain entry descent count once per
 * lane.  The exact pass's re-casts are not counted.  The fast pass runs
 * unrolled one tile per wavefront at 6 waves per SIMD with the scene's tile
 * shape; it is slower than rc_render and meant for measurement of the
 * traversal (the paper prices its kernel by the early-termination bound,
 * Sec. 3.2.2).  Errors as rc_render, plus INVALID_ARG for a NULL or
 * misaligned `counts`. */
rc_status rc_render_counts(const rc_scene* scene, const rc_render_args* args, uint32_t* counts,
                           void* ws, size_t ws_bytes, rc_stream stream);

/* ---------------------------------------------------------------------
 * Batched uneven form: environments with different camera counts and image
 * sizes in one persistent launch (Algorithm 1 over a camera table; the
 * paper batches per-environment intrinsics K_e^-1, Sec. 3.2.2).
 * ------------------------------------------------------------------- */

/* One camera of a batch (64 bytes, device memory). */
typedef struct {
    int32_t env;         /* environment: row of link_pos / link_quat */
    int32_t width;       /* image size in pixels, 1..65535 */
    int32_t height;
    uint32_t out_offset; /* first pixel of this image in the packed outputs */
    uint32_t cam_uid;    /* camera id for the sensor model's counters */
    float pos[3];        /* camera centre (world, m) */
    float quat[4];       /* optical -> world, (x, y, z, w) */
    float intr[4];       /* fx, fy, cx, cy */
} rc_cam_desc;

typedef struct {
    int32_t n_env, n_desc;
    const float* link_pos;     /* device [n_env][n_links][3] */
    const float* link_quat;    /* device [n_env][n_links][4] */
    const rc_cam_desc* desc;   /* device [n_desc]; images packed row-major at out_offset */
    int64_t n_pixels;          /* pixels of the packed outputs */
    int32_t max_width;         /* no descriptor's image is wider (1..65535) */
    int32_t max_height;        /* ... or taller (1..65535) */
    float far_plane;           /* d_max (m), in (0, 1e20] as for rc_render */
    int32_t depth_mode;
    float* depth;              /* device out [n_pixels] */
    int32_t* inst;             /* device out [n_pixels] or NULL */
    int32_t* tri;              /* device out [n_pixels] or NULL */
    void* const* timing;       /* NULL, or two hipEvent_t around the fast-pass kernel */
    const rc_cam_rand* cam_rand; /* NULL, or host struct: randomise the cameras */
} rc_batch_args;

/* Workspace bytes of rc_render_batched. */
rc_status rc_render_batched_size(const rc_scene* scene, int32_t n_env, int32_t n_desc,
                                 int64_t n_pixels, size_t* ws_bytes);

/* Render every described camera in one launch: per-environment top levels
 * are rebuilt, a device prefix sum turns the cameras into a tile table, and
 * either persistent wavefronts pull chunks of tiles from a work counter or a
 * flat camera-major grid gives each tile a wavefront (the schedule says
 * which; rc_autotune picks).  Results equal rc_render's for the same camera
 * bit for bit.  Descriptors are read on the device: one that is out of range
 * (env, size beyond max_width x max_height, or an image that does not fit in
 * n_pixels) renders nothing and sets bit 0 of the status word that
 * rc_render_batched_status reports.  Nothing here allocates or synchronises,
 * so the call can be captured into a graph (rc_graph_capture_batched). */
rc_status rc_render_batched(const rc_scene* scene, const rc_batch_args* args, void* ws,
                            size_t ws_bytes, rc_stream stream);

/* Status word of the last batched render on `ws` (0 = all descriptors
 * valid) and the number of rays it re-cast exactly; synchronises `stream`. */
rc_status rc_render_batched_status(const rc_scene* scene, const rc_batch_args* args,
                                   const void* ws, uint32_t* status, int64_t* exact_rays,
                                   rc_stream stream);

/* ---------------------------------------------------------------------
 * Launch schedule and autotuning.
 * ------------------------------------------------------------------- */

typedef struct {
    int32_t tile_w, tile_h;  /* pixels per wavefront tile, tile_w * tile_h = 64 */
    int32_t rays_per_lane;   /* tiles per wavefront, stacked vertically: 1 or 2 */
    int32_t waves;           /* resident wavefronts per SIMD asked for: 6, 7 or 8 */
    int32_t persistent;      /* batched form only: 1 persistent work queue, 0 flat grid */
    int32_t terrain_packet;  /* 0: each lane walks the terrain hierarchy alone; 1: the
                                wavefront walks it as a packet (a node is entered if any
                                of its rays reaches it) */
    int32_t bodies_flat;     /* 0: links are found by walking the environment's top-level
                                hierarchy; 1: by testing every link's bounding sphere against
                                the cone of the wavefront's rays, then each ray against the
                                surviving spheres */
} rc_render_config;

/* Cap the per-lane stack of the 4-wide terrain walks (the fast pass's, the
 * height map's) at `entries` (1..16; 16 is the default).  A ray whose walk
 * would push onto a full stack is re-cast in full by the exact pass (a height
 * map column is walked again over the binary records), so results do not
 * depend on the cap;
 * fewer entries only make that fallback frequent, which is what tests of it
 * use this for (the nearest-first walk of Alg. 1, Sec. 3.2.2, with its
 * pending subtrees kept on the stack).  Read at each render's set-up, like
 * the schedules.  Errors: INVALID_ARG (NULL scene, entries outside 1..16). */
rc_status rc_set_walk_stack_limit(rc_scene* scene, int32_t entries);

/* Schedule used by rc_render (batched = 0) or rc_render_batched (batched = 1). */
rc_status rc_get_render_config(const rc_scene* scene, int32_t batched, rc_render_config* cfg);
rc_status rc_set_render_config(rc_scene* scene, int32_t batched, const rc_render_config* cfg);

/* Time every candidate schedule (tile 8x8, 16x4, 4x16, 32x2; 1 or 2 tiles
 * per wavefront; 6, 7 or 8 wavefronts per SIMD; per-lane or packet terrain
 * walk; top-level or cone-culled links; for the batched form also
 * persistent or flat) on this exact launch -
 * exactly one of `plain` and `batched` non-NULL - with `reps` timed runs
 * each after one warm-up, keep the fastest for that mode in the scene and
 * return it with its mean time.  Overwrites the launch's outputs.
 * Synchronises `stream`. */
rc_status rc_autotune(rc_scene* scene, const rc_render_args* plain, const rc_batch_args* batched,
                      void* ws, size_t ws_bytes, int32_t reps, rc_stream stream,
                      rc_render_config* best, float* best_ms);

/* ---------------------------------------------------------------------
 * Graph capture of the batched launch.  Sec. 3.2.2 replays its ray-casting
 * kernel from a captured graph to cut launch overhead across many
 * environments; here the whole batched render is captured once and
 * replayed per step.
 * ------------------------------------------------------------------- */

typedef struct rc_graph rc_graph;

/* Capture one rc_render_batched call (its top-level build, tile table,
 * persistent render and exact pass) into an executable HIP graph.  Replays
 * read the same device buffers, so the caller updates poses and descriptors
 * in place between replays.  `stream` must not be capturing already. */
rc_status rc_graph_capture_batched(const rc_scene* scene, const rc_batch_args* args, void* ws,
                                   size_t ws_bytes, rc_stream stream, rc_graph** out);
/* Enqueue one replay on `stream`. */
rc_status rc_graph_launch(rc_graph* graph, rc_stream stream);
rc_status rc_graph_destroy(rc_graph* graph);

/* ---------------------------------------------------------------------
 * Serving: a request loop over a device-resident scene.  Requests (each its
 * own environments, cameras and image size) wait in a FIFO queue, are
 * admitted when a stream slot is free and the arena has room for their
 * outputs, and are packed as they arrive into batched launches that run on
 * several streams at once (continuous batching).  Camera uids are
 * request-local, so a request's result does not depend on its batch.
 * ------------------------------------------------------------------- */

typedef struct rc_server rc_server;

typedef struct {
    int32_t n_streams;       /* concurrent batches (1..16) */
    int64_t max_batch_rays;  /* cap on the rays of one batch (a single larger request still runs) */
    int64_t out_pixels;      /* capacity of the output planes (pixels) */
    float far_plane;
    int32_t depth_mode;
} rc_server_config;

typedef struct {
    int32_t n_env, n_cam, width, height;
    const float* link_pos;   /* device [n_env][n_links][3] */
    const float* link_quat;  /* device [n_env][n_links][4] */
    const float* cam_pos;    /* device [n_env][n_cam][3] */
    const float* cam_quat;   /* device [n_env][n_cam][4] */
    const float* intr;       /* device [n_env][n_cam][4] */
} rc_request;

typedef struct {
    int64_t id;
    int32_t status;          /* RC_OK, or the error of the batch it ran in */
    int32_t reserved;
    int64_t n_pixels;        /* n_env * n_cam * height * width */
    const float* depth;      /* device [n_env][n_cam][height][width], valid until released */
    const int32_t* inst;
    const int32_t* tri;
    double arrival_s, launch_s, done_s;  /* caller clock; done = first poll that saw it finish */
} rc_result;

typedef struct {
    int64_t submitted, completed, rejected, queued, in_flight;
    int64_t batches, rays_completed;
    double p50_s, p99_s, mean_s, max_s;  /* arrival -> observed completion */
    double first_arrival_s, last_done_s;
} rc_server_stats;

/* Arena bytes a server with this configuration needs: three output planes
 * of out_pixels (depth, inst, tri) plus `scratch_bytes` for per-batch poses,
 * camera tables and render workspaces. */
rc_status rc_server_arena_size(const rc_server_config* cfg, size_t scratch_bytes, size_t* bytes);

/* Create a server over `scene` using the caller's device arena (256-byte
 * aligned).  It creates cfg->n_streams HIP streams of default priority and
 * allocates no device memory. */
rc_status rc_server_create(const rc_scene* scene, const rc_server_config* cfg, void* arena,
                           size_t arena_bytes, rc_server** out);

/* A server whose batches run on a model instead of the GPU: a batch started
 * at t finishes at t + launch_s + rays * s_per_ray.  Same queueing,
 * admission and batching; no device is touched.  For tests of the scheduler. */
rc_status rc_server_create_simulated(const rc_server_config* cfg, size_t arena_bytes,
                                     double launch_s, double s_per_ray, rc_server** out);

/* Queue a request that arrived at now_s (caller clock, seconds).  Device
 * pointers must stay valid until the request's result is released.  Errors:
 * INVALID_ARG, WORKSPACE (the request can never fit the arena). */
rc_status rc_server_submit(rc_server* srv, const rc_request* req, double now_s, int64_t* id);

/* Failure injection for testing a caller's error handling: the next
 * n_batches batches whose device work completes are reported as failed
 * (status RC_ERR_DEVICE on each of their requests, rc_last_error names the
 * injection) although the device did its work.  Nothing else changes: the
 * batch's memory is released as for any finished batch, and the resident
 * scene and later requests are unaffected.  n_batches = 0 cancels it. */
rc_status rc_server_fail_next(rc_server* server, int32_t n_batches);

/* Advance the server at time now_s: collect finished batches (non-blocking
 * event queries), then start new batches on free streams from the queue
 * head while memory allows.  *n_done = results now waiting to be taken. */
rc_status rc_server_poll(rc_server* srv, double now_s, int32_t* n_done);

/* Take the oldest finished result (RC_ERR_STATE if none is waiting). */
rc_status rc_server_next_result(rc_server* srv, rc_result* out);

/* Return a taken result's output memory to the arena. */
rc_status rc_server_release(rc_server* srv, int64_t id);

/* Counters and latency statistics (nearest-rank p50 / p99, mean, max over
 * every completed request).  Sorts a copy of all latencies: O(n log n) in
 * the requests completed so far, so a serving loop reads it rarely (not on
 * every poll). */
rc_status rc_server_stats_get(const rc_server* srv, rc_server_stats* out);

/* Wait for all batches in flight (GPU servers), then free the handle.  The
 * handle is freed in every case; DEVICE reports an error the wait met. */
rc_status rc_server_destroy(rc_server* srv);

/* ---------------------------------------------------------------------
 * Sensor model: latency, noise, dropout (Sec. 1, Sec. 4.1, Table 6).
 * ------------------------------------------------------------------- */

#define RC_POST_NOISE 1u
#define RC_POST_DROPOUT 2u
#define RC_POST_LATENCY 4u
/* Random side masking (Sec. 3.2, "Random Side Masking"): per environment and
 * mask epoch a mode in {none, small, large} is drawn from the probabilities
 * mask_p[type] of the environment's terrain type (word 0 of Philox with
 * counter (env, 0xFFFFFFFD, epoch_lo32, (epoch_hi16 << 16) | 4), u =
 * (w >> 8) 2^-24: none if u < p0, small if u < p0 + p1, else large).  A mode
 * masks the columns x < m and x >= width - m of every camera image of the
 * environment, m = round(mask_frac[mode - 1] * width); a masked pixel of
 * the frame shown at step s becomes near + (far - near) u, u from word 3 of
 * the pixel's own draw for step s, and its dropout mask is 0. */
#define RC_POST_SIDEMASK 8u

typedef struct {
    uint64_t seed;       /* Philox4x32-10 key (low word, high word) */
    float sigma_abs;     /* noise std = sigma_abs + sigma_rel * depth (m) */
    float sigma_rel;
    float p_drop;        /* per-pixel dropout probability in [0, 1] */
    float near_plane;    /* output clamp [near_plane, far_plane] (m) */
    float far_plane;
    float fill;          /* value written for a dropped pixel */
    int32_t lat_min;     /* latency in frames, uniform in [lat_min, lat_max] */
    int32_t lat_max;
    uint32_t flags;      /* RC_POST_NOISE | RC_POST_DROPOUT | RC_POST_LATENCY | RC_POST_SIDEMASK */
    float mask_frac[2];  /* side band per image side, fraction of the width: small, large */
    float mask_p[4][3];  /* per terrain type 0..3: P(none), P(small), P(large) */
    uint64_t mask_epoch; /* draw index of the modes (e.g. the episode) */
    const uint8_t* mask_type; /* device [n_env] terrain type per environment, or NULL (type 0) */
} rc_post_params;

/* Workspace bytes of a sensor-model state for frames [n_env][n_cam][height]
 * [width] with latencies up to max_latency frames (a device ring of
 * max_latency + 1 captures and their dropout masks). */
rc_status rc_post_size(int32_t n_env, int32_t n_cam, int32_t height, int32_t width,
                       int32_t max_latency, size_t* ws_bytes);

/* Create the state (host handle; the ring lives in the caller's `ws`). */
rc_status rc_post_create(int32_t n_env, int32_t n_cam, int32_t height, int32_t width,
                         int32_t max_latency, void* ws, size_t ws_bytes, rc_post** out);

/* Forget captured frames: the next rc_postprocess call starts a new sequence. */
rc_status rc_post_reset(rc_post* post);

/* Apply the sensor model to the frame rendered at `step` and emit the frame
 * the sensor shows at that step.  For capture step s, pixel p (row-major
 * index within its image) and camera uid u, Philox4x32-10 with key = seed
 * encrypts the counter (p, u, s mod 2^32, ((s >> 32) mod 2^16) << 16):
 * word 0 decides dropout (w0 < floor(p_drop * 2^32)), words 1-2 give a
 * Box-Muller normal g from u1 = ((w1 >> 8) + 1) 2^-24, u2 = (w2 >> 8) 2^-24.
 * A hit becomes clamp(z + (sigma_abs + sigma_rel z) g, near, far), a miss
 * becomes far, a dropped pixel becomes fill; the result enters the ring.
 * The latency of camera u at step s is k = lat_min + ((w0 * (lat_max -
 * lat_min + 1)) >> 32) with w from the counter (0xFFFFFFFF, u, s mod 2^32,
 * (((s >> 32) mod 2^16) << 16) | 1); the output is the capture of step
 * max(s - k, s0), s0 = the first step of the sequence.
 *   depth_in  device float [n_env][n_cam][height][width] (rc_render output)
 *   inst_in   device int32, same shape (hit <=> inst >= 0), or NULL (hit <=>
 *             depth < far_plane)
 *   cam_uid   device uint32 [n_env * n_cam] or NULL (uid = e * n_cam + c)
 *   depth_out device float, same shape; drop_out device uint8, same shape,
 *             dropout mask of the capture shown, or NULL; lat_out device
 *             uint8 [n_env][n_cam] or NULL.
 * Steps must be consecutive within a sequence (else STATE); s < 2^48. */
rc_status rc_postprocess(rc_post* post, const float* depth_in, const int32_t* inst_in,
                         const rc_post_params* params, uint64_t step, const uint32_t* cam_uid,
                         float* depth_out, uint8_t* drop_out, uint8_t* lat_out,
                         rc_stream stream);

/* Sensor-model state over packed outputs of n_pixels (the batched form). */
rc_status rc_post_size_packed(int64_t n_pixels, int32_t max_latency, size_t* ws_bytes);
rc_status rc_post_create_packed(int64_t n_pixels, int32_t max_latency, void* ws, size_t ws_bytes,
                                rc_post** out);

/* rc_postprocess that also writes, for checking, the raw Philox4x32-10 words
 * of every pixel's draw at this step into words_out (device, 16-byte
 * aligned, uint32 [n_env][n_cam][height][width][4]): w0 decides dropout, w1
 * and w2 feed Box-Muller, w3 the side-mask fill.  The words come from the
 * same code that computes the outputs, so they can be compared bit for bit
 * with an independent Philox (Salmon et al., SC'11) at the documented
 * counters; the outputs equal rc_postprocess's.  Errors as rc_postprocess,
 * plus INVALID_ARG for a NULL or misaligned words_out. */
rc_status rc_postprocess_words(rc_post* post, const float* depth_in, const int32_t* inst_in,
                               const rc_post_params* params, uint64_t step, const uint32_t* cam_uid,
                               float* depth_out, uint8_t* drop_out, uint8_t* lat_out,
                               uint32_t* words_out, rc_stream stream);

/* rc_postprocess over a batch: pixel p of camera d is packed at
 * desc[d].out_offset + p and uses desc[d].cam_uid; lat_out is [n_desc]. */
rc_status rc_postprocess_batched(rc_post* post, const float* depth_in, const int32_t* inst_in,
                                 const rc_post_params* params, uint64_t step,
                                 const rc_cam_desc* desc, int32_t n_desc, float* depth_out,
                                 uint8_t* drop_out, uint8_t* lat_out, rc_stream stream);

/* Release the handle (not the workspace). NULL is a no-op. */
rc_status rc_post_destroy(rc_post* post);

/* ---------------------------------------------------------------------
 * Privileged height map (the terrain experts' local grid, Sec. 3.1).
 * ------------------------------------------------------------------- */

typedef struct {
    int32_t n_env;
    const float* base_pos; /* device [n_env][3]: robot base (world, m) */
    const float* base_yaw; /* device [n_env]: heading about +z (rad) */
    int32_t nx, ny;        /* grid points along the heading and to the left (17 x 11 in the paper) */
    float dx, dy;          /* spacing (m; 0.1 in the paper) */
    float top;             /* rays start at base z + top (m) */
    float depth;           /* and reach down `depth` (m) */
    float miss;            /* value of a point with no terrain below */
    float* heights;        /* device out [n_env][ny][nx]: terrain z - base z (m) */
} rc_heightmap_args;

/* Height map of the terrain around each robot base: grid point (i, j) sits at
 * local ((i - (nx - 1) / 2) dx, (j - (ny - 1) / 2) dy), turned by the yaw
 * and placed at the base; a vertical ray from base z + top finds the highest
 * terrain surface below within `depth` (closed triangles, FP64 decisions, so a
 * point on a shared edge finds its surface).  Links are not seen.  Errors:
 * INVALID_ARG (NULL pointers, n_env < 1, nx or ny outside [1, 4096], dx or dy
 * not finite and > 0, depth not finite and > 0, top not finite), STATE (no
 * terrain), DEVICE.  Asynchronous on `stream`. */
rc_status rc_heightmap(const rc_scene* scene, const rc_heightmap_args* args, rc_stream stream);

/* Downsample rendered frames by block pooling (the paper feeds its policy
 * 240x135 depth downsampled to 48x27, Sec. 4.1; the pooling rule is not
 * stated): output pixel (y, x) of image i is the mean depth of the hit pixels
 * (inst >= 0, or depth < far_plane when inst is NULL) in rows [y f, y f + f)
 * and columns [x f, x f + f), summed in row-major order in FP32, or
 * far_plane when none of them hit.  depth_in, inst_in [n_img][height][width]
 * and depth_out [n_img][height / f][width / f] (floor division; rows and
 * columns beyond the last full block are ignored) are device memory owned by
 * the caller.  Asynchronous on `stream`.  Errors: INVALID_ARG (NULL depth
 * pointers, sizes < 1, factor < 1 or > min(height, width), an image of more
 * than 2^31 - 1 pixels, non-finite far_plane), DEVICE. */
rc_status rc_downsample(const float* depth_in, const int32_t* inst_in, int64_t n_img, int32_t height,
                        int32_t width, int32_t factor, float far_plane, float* depth_out,
                        rc_stream stream);

/* ---------------------------------------------------------------------
 * Inspection of built hierarchies (for tests; no compute).
 * ------------------------------------------------------------------- */

typedef struct {
    int64_t n_prim;        /* leaves (triangles or instances) */
    int64_t n_nodes;       /* internal node records (>= 1) */
    int64_t node_offset;   /* byte offset in the workspace: node records, 64 B each */
    int64_t tri_offset;    /* byte offset: float [n_prim][9] triangles in leaf order */
    int64_t tri_id_offset; /* byte offset: int32 [n_prim] input index of each leaf */
    int64_t key_offset;    /* byte offset: uint64 [n_prim] sorted Morton keys (of the Morton
                              build; not in leaf order after rc_scene_rebuild_sah) */
    int32_t max_depth;     /* deepest internal node (root = 0) */
    int32_t reserved;
    int64_t wide_offset;   /* byte offset: 4-wide records, 128 B each, one per node record */
} rc_bvh_layout;

/* Layout of the terrain hierarchy (which = -1) or of link `which` inside the
 * workspace given to rc_scene_create / rc_robot_meshes.  Node record:
 * float box0[6] = (lo.x, hi.x, lo.y, hi.y, lo.z, hi.z), float box1[6],
 * int32 child0, child1, parent, sibling; child >= 0 is an internal node,
 * child < 0 is leaf ~child; boxes are padded outwards for FP32 traversal.
 * 4-wide record of node n (the fast pass's terrain walk): the children of n,
 * each internal child replaced by its two children (2-4 slots, in the binary
 * children's order, unused slots the far point 1e30 with child word 0), as
 * float lo.x[4], hi.x[4], lo.y[4], hi.y[4], lo.z[4], hi.z[4], int32 child[4],
 * then 16 bytes of zeros. */
rc_status rc_bvh_layout_of(const rc_scene* scene, int32_t which, rc_bvh_layout* out);

#ifdef __cplusplus
}
#endif
#endif /* RC_H */
